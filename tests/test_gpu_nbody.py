"""GPU parity of hs_nbody (the all-pairs interaction on the two-array recipe)
against the FP64 oracle.

Error measures, per body i (oracle values a_i, phi_i):
  acceleration  max_c |a_ic - ahat_ic| / scale_i,
                scale_i = sum_{j != i} |m_j d_ij| / s_ij^(3/2) (the sum of the
                lengths of the terms, from the oracle);
  potential     |phi_i - phihat_i| / |phi_i| (all terms have one sign).
Bounds derived from the arithmetic, u the unit roundoff (2^-24 FP32,
2^-53 FP64): each term carries <= ~18 u relative error (a 1-ulp rsqrt and
about 17 roundings), each of the K partials is a sequential sum of n / K
terms (<= (n/K) u sum |terms|), and the FP64 combine plus the final rounding
add u.  So acceleration <= (n/K + 20) u and potential <= (n/K + 8) u; FP64
results are also held to 1e-12.  The bound is worst-case; a missing or
doubled pair is caught separately with one-hot masses, where each output
is a single term.  For FP32 the library rounds eps2 to float, and so do the
oracle's inputs here.  Output buffers are poisoned with NaN.
"""
import numpy as np
import pytest

import oracle
from paper_cs_9809105_amd import inputs
from tests._gpu import gpu_available, host, note, poisoned

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_cs_9809105_amd as hs

U = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}
TDT = {"f32": "float32", "f64": "float64"}


def _skip_no_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _stored(X, dt):
    """The bodies as stored (rounded to the storage type) and their float64 values."""
    t = torch.from_numpy(np.ascontiguousarray(X)).to(getattr(torch, TDT[dt]))
    return t.cuda(), t.to(torch.float64).numpy()


def _eps2(eps2, dt):
    return float(np.float32(eps2)) if dt == "f32" else float(eps2)


def _errors(got, ref, scale):
    ea = np.abs(got[:, :3] - ref[:, :3]).max(axis=1) / np.where(scale > 0, scale, 1.0)
    ep = np.abs(got[:, 3] - ref[:, 3]) / np.where(ref[:, 3] != 0, np.abs(ref[:, 3]), 1.0)
    return ea.max(initial=0.0), ep.max(initial=0.0)


def _bounds(n, K, dt):
    u = U[dt]
    ta, tp = (n / K + 20) * u, (n / K + 8) * u
    if dt == "f64":
        ta, tp = min(ta, 1e-12), min(tp, 1e-12)
    return ta, tp


def _run(Xd, eps2, dt, p, K):
    n = Xd.shape[0]
    out = poisoned((n, 4), getattr(torch, TDT[dt]))
    hs.hs_nbody(Xd, eps2, dtype=dt, p=p, K=K, out=out)
    torch.cuda.synchronize()
    return host(out)


# (n, p, K): several workgroups per block, ragged last block, blocks left
# empty (n < p S), K = 1 (systolic), K = p, prime p, K with 2, 3 and 4 replica
# groups per position, the largest ring (p = 4096, 32 replica groups, blocks
# of 2 bodies), and two workgroup slices per block (70000 bodies, p = 256).
CASES = [
    (4096, 16, 4),
    (4096, 16, 1),
    (4096, 16, 16),
    (1000, 8, 2),
    (777, 12, 3),
    (300, 64, 8),
    (3001, 7, 7),
    (600, 36, 6),
    (1200, 48, 12),
    (2600, 8, 8),
    (5, 4, 2),
    (2, 2, 2),
    (1, 1, 1),
    (5000, 4096, 64),
    (70000, 256, 16),
]


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n,p,K", CASES)
@pytest.mark.parametrize("eps2", [0.0, 1e-4])
def test_nbody_matches_oracle(dt, n, p, K, eps2):
    _skip_no_gpu()
    note("hs_nbody", dt, n, p, K, eps2)
    X = inputs.plummer(n, seed=inputs.BASE_SEED + n + p, unequal=True)
    Xd, X64 = _stored(X, dt)
    e2 = _eps2(eps2, dt)
    got = _run(Xd, e2, dt, p, K)
    ref, scale = oracle.nbody(X64, e2, with_scale=True)
    assert np.isfinite(got).all()
    ea, ep = _errors(got, ref, scale)
    ta, tp = _bounds(n, K, dt)
    assert ea <= ta and ep <= tp, (ea, ta, ep, tp)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_each_pair_once_one_hot_masses(dt):
    """Only body j has mass: every other body's output is the single term of
    the pair (i, j), and body j's own output is exactly zero."""
    _skip_no_gpu()
    n, p, K = 1000, 16, 4                         # S = 63: a ragged last block
    X = inputs.plummer(n, seed=77, unequal=False)
    for j in (0, 62, 63, 500, 944, 945, 999):
        Xj = X.copy()
        Xj[:, 3] = 0.0
        Xj[j, 3] = 1.0
        note("hs_nbody one-hot", dt, j)
        Xd, X64 = _stored(Xj, dt)
        got = _run(Xd, 1e-4, dt, p, K)
        ref = oracle.nbody(X64, _eps2(1e-4, dt))
        assert np.array_equal(got[j], np.zeros(4)), j
        rest = np.arange(n) != j
        rel = np.abs(got[rest] - ref[rest]) / np.abs(ref[rest]).max(axis=1, keepdims=True)
        assert rel.max() <= 40 * U[dt], (j, rel.max())


def test_two_bodies_and_lone_body():
    _skip_no_gpu()
    note("hs_nbody two bodies")
    X = np.array([[0.0, 0.0, 0.0, 1.0], [0.5, -0.25, 1.0, 3.0]])
    Xd, X64 = _stored(X, "f64")
    got = _run(Xd, 0.0, "f64", 2, 2)
    ref = oracle.nbody(X64, 0.0)
    assert np.allclose(got, ref, rtol=1e-15, atol=0)
    assert np.allclose(got[0, :3] * 1.0, -got[1, :3] * 3.0, rtol=1e-15)   # m0 a0 = -m1 a1
    one, _ = _stored(np.array([[1.0, 2.0, 3.0, 4.0]]), "f32")
    assert np.array_equal(_run(one, 0.0, "f32", 1, 1), np.zeros((1, 4)))


def test_empty_system():
    _skip_no_gpu()
    X = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    assert hs.hs_nbody(X, 0.0, p=4, K=2).shape == (0, 4)


def test_deterministic():
    _skip_no_gpu()
    note("hs_nbody determinism")
    Xd, _ = _stored(inputs.plummer(5000, seed=5), "f32")
    a = hs.hs_nbody(Xd, 1e-4, p=16, K=4)
    b = hs.hs_nbody(Xd, 1e-4, p=16, K=4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_bench_configuration_sampled():
    """The benchmark's workload in its launch configuration: n = 2^18 Plummer
    bodies, p = 64, K = 8, eps2 = 1e-4, FP32; 256 sampled bodies against the
    oracle, plus Newton's third law on the whole output."""
    _skip_no_gpu()
    n, p, K, eps2 = 1 << 18, 64, 8, 1e-4
    note("hs_nbody bench configuration", n, p, K)
    X = inputs.plummer(n, seed=inputs.BASE_SEED, unequal=False)
    Xd, X64 = _stored(X, "f32")
    e2 = _eps2(eps2, "f32")
    got = _run(Xd, e2, "f32", p, K)
    assert np.isfinite(got).all()
    rows = inputs.sample_rows(n, 256, seed=3)
    ref, scale = oracle.nbody_rows(X64, e2, rows)
    ea, ep = _errors(got[rows], ref, scale)
    ta, tp = _bounds(n, K, "f32")
    assert ea <= ta and ep <= tp, (ea, ta, ep, tp)
    # sum_i m_i a_i = 0 exactly; each a_i is off by at most ta * scale_i,
    # and scale_i is estimated from the sample (mean, times 4 for margin)
    m = X64[:, 3]
    tot = np.abs((m[:, None] * got[:, :3]).sum(axis=0)).max()
    assert tot <= ta * 4 * scale.mean() * m.sum(), tot


def test_profile_counts_interaction_launches():
    _skip_no_gpu()
    Xd, _ = _stored(inputs.plummer(512, seed=6), "f32")
    hs.hs_profile_begin()
    hs.hs_nbody(Xd, 1e-4, p=8, K=2)
    hs.hs_nbody(Xd, 1e-4, p=8, K=1)
    ms, launches = hs.hs_profile_end()
    assert launches == 2 and ms > 0
