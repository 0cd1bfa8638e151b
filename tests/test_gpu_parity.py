"""GPU parity: every entry point of the C ABI against the FP64 oracle.

Gates (tests/_gpu.py: ``check``):
  err_row  = max_r |C_r - Chat_r| / |Chat_r|:
             f64 1e-12; f32, split3_bf16, split2_f16 1e-5; bf16 1.5e-2 and
             f16 3e-3
             (reported forms: the inputs' rounding is in the stored values)
  err_term = element error over u sqrt(k sum_t (a_t b_t)^2), the
             statistical scale of its rounding errors: f64, f32 and
             the split forms 16 u (a lone wrong element is seen at its own scale,
             not diluted over a row)
  err_elem = max |dC| / (|A||B|) <= (c k + d) u, the worst-case rounding
             bound of each form's accumulation (derived beside ``elem_bound``)
Small-integer inputs are exact in every form and must match bit for bit.
Output buffers are poisoned with NaN so an element never written shows up.
"""
import numpy as np
import pytest

import oracle
from oracle.metrics import err_row
from paper_cs_9809105_amd import inputs
from tests._gpu import ROW_TOL, check, gpu_available, host, note, poisoned, to_dev

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_cs_9809105_amd as hs
    from paper_cs_9809105_amd import autograd as hs_autograd

TOL = ROW_TOL
# FP8 forms quantise inside the library; the refined form is also held to an
# element bound relative to sum |a||b| (err_elem).
FP8_R1_ELEM = 2.0 ** -10
OUT = {"f64": "float64"}


def _skip_no_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _out_dtype(dt):
    return torch.float64 if dt == "f64" else torch.float32


# (m, n, k, p, K): several tiles, ragged stripes, ragged contraction blocks,
# column tails, K = 1 (systolic), K = p, prime p
SMALL = [
    (256, 256, 256, 16, 4),
    (256, 256, 256, 16, 1),
    (256, 256, 256, 16, 16),
    (200, 136, 152, 8, 2),
    (77, 45, 333, 5, 5),
    (64, 300, 96, 12, 3),
    (33, 17, 9, 4, 2),
    (520, 600, 264, 4, 2),
]
DTYPES = ["f64", "f32", "split3_bf16", "bf16", "f16", "split2_f16"]


def _gemm_case(dt, m, n, k, p, K, tn, seed, gen=inputs.uniform):
    _skip_no_gpu()
    a_shape = (k, m) if tn else (m, k)
    A, A64 = to_dev(gen(a_shape, seed=seed), dt)
    B, B64 = to_dev(gen((k, n), seed=seed + 1), dt)
    C = poisoned((m, n), _out_dtype(dt))
    note("gemm%s" % ("_tn" if tn else ""), dt, (m, n, k), "p=%d K=%d" % (p, K), "seed", seed)
    f = hs.hs_gemm_tn if tn else hs.hs_gemm
    f(A, B, dtype=dt, p=p, K=K, out=C)
    torch.cuda.synchronize()
    ref = oracle.gemm_tn(A64, B64) if tn else oracle.gemm(A64, B64)
    return host(C), ref, A64, B64


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("tn", [False, True])
def test_gemm_small(dt, case, tn):
    m, n, k, p, K = case
    got, ref, A64, B64 = _gemm_case(dt, m, n, k, p, K, tn, seed=1000 + m + n + k)
    check(got, ref, dt, A64.T if tn else A64, B64, what="gemm%s %s" % ("_tn" if tn else "", case))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("case", [(256, 256, 256, 16, 4), (200, 136, 152, 8, 2), (96, 520, 1000, 8, 4)])
@pytest.mark.parametrize("tn", [False, True])
def test_gemm_small_int_bit_exact(dt, case, tn):
    m, n, k, p, K = case
    got, ref, _, _ = _gemm_case(dt, m, n, k, p, K, tn, seed=77, gen=inputs.small_int)
    assert np.array_equal(got, ref), (dt, case, tn, np.abs(got - ref).max())


def test_fp64_config_n256_p16():
    """C = A B, n = 256, FP64, p = 16, U[-1, 1] and the small-integer variant."""
    got, ref, A64, B64 = _gemm_case("f64", 256, 256, 256, 16, 0, False, seed=inputs.BASE_SEED)
    check(got, ref, "f64", A64, B64, what="fp64 n=256")
    got, ref, _, _ = _gemm_case("f64", 256, 256, 256, 16, 0, False, seed=inputs.BASE_SEED,
                                gen=inputs.small_int)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("tn", [False, True])
def test_fp32_config_n4096_p64(tn):
    """FP32 C = A B and C = A^T B at n = 4096, p = 64, N(0, 1); 64 sampled rows."""
    _skip_no_gpu()
    n = 4096
    A, A64 = to_dev(inputs.normal((n, n), seed=inputs.BASE_SEED + 1), "f32")
    B, B64 = to_dev(inputs.normal((n, n), seed=inputs.BASE_SEED + 2), "f32")
    note("f32 4096", "tn" if tn else "nn")
    C = (hs.hs_gemm_tn if tn else hs.hs_gemm)(A, B, dtype="f32", p=64, K=0)
    torch.cuda.synchronize()
    rows = inputs.sample_rows(n, 64, seed=5)
    ref = oracle.gemm_tn_rows(A64, B64, rows) if tn else oracle.gemm_rows(A64, B64, rows)
    got = host(C)
    check(got[rows], ref, "f32", A64[:, rows].T if tn else A64[rows], B64, what="f32 n=4096 %s" % ("tn" if tn else "nn"))


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("shape,p,K", [((8192, 8192), 64, 0), ((1000, 777), 8, 2), ((37, 5), 4, 4),
                                       ((64, 64), 1, 1), ((130, 4096), 16, 16)])
def test_gemv(dt, shape, p, K):
    _skip_no_gpu()
    m, n = shape
    A, A64 = to_dev(inputs.normal((m, n), seed=31 + m), dt)
    x, x64 = to_dev(inputs.normal((n,), seed=32 + n), dt)
    note("gemv", dt, shape, p, K)
    y = hs.hs_gemv(A, x, dtype=dt, p=p, K=K)
    torch.cuda.synchronize()
    ref = oracle.gemv(A64, x64)
    got = host(y)
    check(got, ref, dt, A64, x64[:, None], what="gemv %s p=%d K=%d" % (shape, p, K), vector=True)
    Ai, Ai64 = to_dev(inputs.small_int((m, n), seed=33), dt)
    xi, xi64 = to_dev(inputs.small_int((n,), seed=34), dt)
    yi = hs.hs_gemv(Ai, xi, dtype=dt, p=p, K=K)
    assert np.array_equal(host(yi), oracle.gemv(Ai64, xi64))


@pytest.mark.parametrize("dt", ["f32", "split3_bf16", "bf16", "f16", "split2_f16"])
@pytest.mark.parametrize("K", [0, 2])
def test_precision_config_n8192(dt, K):
    """n = 8192, p = 64, N(0, 1) rows scaled log-uniformly in [1e-3, 1e3]; 32 sampled rows."""
    _skip_no_gpu()
    n = 8192
    A, A64 = to_dev(inputs.row_scaled((n, n), seed=inputs.BASE_SEED + 2), dt)
    B, B64 = to_dev(inputs.row_scaled((n, n), seed=inputs.BASE_SEED + 3), dt)
    note("precision 8192", dt, "K", K)
    C = hs.hs_gemm(A, B, dtype=dt, p=64, K=K)
    torch.cuda.synchronize()
    rows = inputs.sample_rows(n, 32, seed=6)
    ref = oracle.gemm_rows(A64, B64, rows)
    got = host(C)[rows]
    check(got, ref, dt, A64[rows], B64, what="precision n=8192 K=%d" % K)


@pytest.mark.parametrize("dt", ["split3_bf16", "f32", "split2_f16"])
def test_headline_step_n8192(dt):
    """The benchmark's step exactly as bench.py times it: its own inputs
    (n = 8192, A and B row-scaled, G N(0, 1)), its step function (C = A.B,
    dA = G.B^T, dB = A^T.G on p = 64, K = 2); C, dA and dB on 16 sampled
    rows each."""
    _skip_no_gpu()
    import bench
    n, p, K = 8192, 64, 2
    A, A64 = to_dev(inputs.row_scaled((n, n), seed=inputs.BASE_SEED + 2), dt)
    B, B64 = to_dev(inputs.row_scaled((n, n), seed=inputs.BASE_SEED + 3), dt)
    G, G64 = to_dev(inputs.normal((n, n), seed=inputs.BASE_SEED + 4), dt)
    note("headline step", dt)
    C, dA, dB = bench.step(hs, A, B, G, dt, p, K)
    torch.cuda.synchronize()
    rows = inputs.sample_rows(n, 16, seed=46)
    check(host(C)[rows], oracle.gemm_rows(A64, B64, rows), dt, A64[rows], B64, what="headline step C")
    check(host(dA)[rows], oracle.grad_a_rows(G64, B64, rows), dt, G64[rows], B64.T, what="headline step dA")
    check(host(dB)[rows], oracle.grad_b_rows(A64, G64, rows), dt, A64[:, rows].T, G64, what="headline step dB")


@pytest.mark.parametrize("dt", ["f32", "split3_bf16", "split2_f16"])
def test_backward_config(dt):
    """A 4096 x 2048, B 2048 x 8192, G N(0, 1), p = 16: C, dA, dB on sampled rows."""
    _skip_no_gpu()
    m, k, n = 4096, 2048, 8192
    A, A64 = to_dev(inputs.normal((m, k), seed=41), dt)
    B, B64 = to_dev(inputs.normal((k, n), seed=42), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=43), dt)
    note("backward config", dt)
    C = hs.hs_gemm(A, B, dtype=dt, p=16)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=dt, p=16)
    torch.cuda.synchronize()
    rm = inputs.sample_rows(m, 32, seed=44)
    rk = inputs.sample_rows(k, 32, seed=45)
    check(host(C)[rm], oracle.gemm_rows(A64, B64, rm), dt, A64[rm], B64, what="C4 C")
    check(host(dA)[rm], oracle.grad_a_rows(G64, B64, rm), dt, G64[rm], B64.T, what="C4 dA")
    check(host(dB)[rk], oracle.grad_b_rows(A64, G64, rk), dt, A64[:, rk].T, G64, what="C4 dB")


@pytest.mark.parametrize("dt", ["f64", "f32", "split3_bf16", "split2_f16"])
@pytest.mark.parametrize("case", [(96, 80, 64, 8, 2), (200, 136, 152, 8, 4), (64, 64, 64, 16, 0)])
def test_backward_small(dt, case):
    _skip_no_gpu()
    m, n, k, p, K = case
    A, A64 = to_dev(inputs.normal((m, k), seed=51), dt)
    B, B64 = to_dev(inputs.normal((k, n), seed=52), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=53), dt)
    note("backward small", dt, case)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=dt, p=p, K=K)
    torch.cuda.synchronize()
    rA, rB = oracle.backward(A64, B64, G64)
    check(host(dA), rA, dt, G64, B64.T, what="backward small dA %s" % (case,))
    check(host(dB), rB, dt, A64.T, G64, what="backward small dB %s" % (case,))
    dA2, none = hs.hs_gemm_backward(A, B, G, dtype=dt, p=p, K=K, need_b=False)
    assert none is None and torch.equal(dA, dA2)
    Ai, Ai64 = to_dev(inputs.small_int((m, k), seed=54), dt)
    Bi, Bi64 = to_dev(inputs.small_int((k, n), seed=55), dt)
    Gi, Gi64 = to_dev(inputs.small_int((m, n), seed=56), dt)
    dAi, dBi = hs.hs_gemm_backward(Ai, Bi, Gi, dtype=dt, p=p, K=K)
    rAi, rBi = oracle.backward(Ai64, Bi64, Gi64)
    assert np.array_equal(host(dAi), rAi) and np.array_equal(host(dBi), rBi)


def test_autograd_fd_fp64_64cubed():
    """Finite differences through the GPU F64 forward match the GPU backward."""
    _skip_no_gpu()
    m = k = n = 64
    A, A64 = to_dev(inputs.normal((m, k), seed=61), "f64")
    B, B64 = to_dev(inputs.normal((k, n), seed=62), "f64")
    G, G64 = to_dev(inputs.normal((m, n), seed=63), "f64")
    A.requires_grad_(True)
    B.requires_grad_(True)
    note("autograd fd f64")
    C = hs_autograd.matmul(A, B, dtype="f64", p=16)
    (C * G).sum().backward()
    dA, dB = host(A.grad), host(B.grad)
    rA, rB = oracle.backward(A64, B64, G64)
    check(dA, rA, "f64", G64, B64.T, what="autograd f64 dA")
    check(dB, rB, "f64", A64.T, G64, what="autograd f64 dB")
    h = 2.0 ** -4
    g = inputs.rng(64)
    with torch.no_grad():
        for t in range(6):
            if t < 3:
                D = torch.from_numpy(g.standard_normal((m, k))).cuda()
                lp = (hs.hs_gemm(A + h * D, B, dtype="f64", p=16) * G).sum().item()
                lm = (hs.hs_gemm(A - h * D, B, dtype="f64", p=16) * G).sum().item()
                an = float(np.sum(dA * D.cpu().numpy()))
            else:
                D = torch.from_numpy(g.standard_normal((k, n))).cuda()
                lp = (hs.hs_gemm(A, B + h * D, dtype="f64", p=16) * G).sum().item()
                lm = (hs.hs_gemm(A, B - h * D, dtype="f64", p=16) * G).sum().item()
                an = float(np.sum(dB * D.cpu().numpy()))
            assert abs((lp - lm) / (2 * h) - an) <= 1e-9 * max(1.0, abs(an))


@pytest.mark.parametrize("dt", ["f32", "split3_bf16", "split2_f16"])
def test_autograd_matches_oracle(dt):
    _skip_no_gpu()
    m, k, n = 192, 160, 224
    A, A64 = to_dev(inputs.normal((m, k), seed=71), dt)
    B, B64 = to_dev(inputs.normal((k, n), seed=72), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=73), dt)
    A.requires_grad_(True)
    B.requires_grad_(True)
    note("autograd", dt)
    C = hs_autograd.matmul(A, B, dtype=dt, p=8, K=2)
    C.backward(G)
    rA, rB = oracle.backward(A64, B64, G64)
    check(host(C), oracle.gemm(A64, B64), dt, A64, B64, what="autograd C")
    check(host(A.grad), rA, dt, G64, B64.T, what="autograd dA")
    check(host(B.grad), rB, dt, A64.T, G64, what="autograd dB")


@pytest.mark.parametrize("dt", ["f32", "split3_bf16", "bf16", "split2_f16"])
def test_bitwise_deterministic(dt):
    _skip_no_gpu()
    A, _ = to_dev(inputs.normal((1024, 768), seed=81), dt)
    B, _ = to_dev(inputs.normal((768, 1100), seed=82), dt)
    note("determinism", dt)
    C1 = hs.hs_gemm(A, B, dtype=dt, p=8, K=4)
    C2 = hs.hs_gemm(A, B, dtype=dt, p=8, K=4)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)


def test_empty_and_zero_contraction():
    _skip_no_gpu()
    note("empty shapes")
    for dt in ["f32", "f64", "split3_bf16", "split2_f16"]:
        A, _ = to_dev(np.zeros((0, 5)), dt)
        B, _ = to_dev(np.zeros((5, 7)), dt)
        assert hs.hs_gemm(A, B, dtype=dt, p=4).shape == (0, 7)
        A, _ = to_dev(np.zeros((6, 0)), dt)
        B, _ = to_dev(np.zeros((0, 9)), dt)
        C = poisoned((6, 9), _out_dtype(dt))
        hs.hs_gemm(A, B, dtype=dt, p=2, out=C)
        torch.cuda.synchronize()
        assert not C.any()
    A, _ = to_dev(np.zeros((5, 0)), "f32")
    x, _ = to_dev(np.zeros((0,)), "f32")
    assert not hs.hs_gemv(A, x, dtype="f32", p=1).any()


def test_leading_dimension_views():
    """Row strides larger than the row length (sub-matrix views)."""
    _skip_no_gpu()
    for dt in ["f32", "split3_bf16", "f64", "split2_f16"]:
        Abig, Abig64 = to_dev(inputs.normal((130, 300), seed=91), dt)
        Bbig, Bbig64 = to_dev(inputs.normal((200, 170), seed=92), dt)
        A, B = Abig[:, 10:210], Bbig[:, 3:163]
        C = poisoned((250, 200), _out_dtype(dt))[5:135, 20:180]
        note("views", dt)
        hs.hs_gemm(A, B, dtype=dt, p=10, K=2, out=C)
        torch.cuda.synchronize()
        ref = oracle.gemm(Abig64[:, 10:210], Bbig64[:, 3:163])
        check(host(C), ref, dt, Abig64[:, 10:210], Bbig64[:, 3:163], what="views")


# Launches with fewer output tiles than CUs split each tile's step order over
# up to 4 workgroups (each at least 64 stages) and sum their planes in FP64:
# long contractions on one or a few tiles.
SPLIT_CASES = [(256, 256, 16384, 4, 2), (300, 200, 8192, 8, 4), (512, 256, 6144, 3, 1), (64, 96, 4096, 16, 16)]


@pytest.mark.parametrize("dt", ["f32", "split3_bf16", "split2_f16", "bf16", "f16", "f64"])
@pytest.mark.parametrize("case", SPLIT_CASES)
def test_split_stage_sequence(dt, case):
    """C = A.B, A^T.B and the backward pair where the stage sequence is split
    (tests/test_abi.py checks that such shapes take the split), against the
    oracle; small integers bit for bit; run to run bitwise."""
    _skip_no_gpu()
    m, n, k, p, K = case
    got, ref, A64, B64 = _gemm_case(dt, m, n, k, p, K, False, seed=1700 + m)
    check(got, ref, dt, A64, B64, what="split stages %s" % (case,))
    got_t, ref_t, At64, Bt64 = _gemm_case(dt, m, n, k, p, K, True, seed=1710 + m)
    check(got_t, ref_t, dt, At64.T, Bt64, what="split stages tn %s" % (case,))
    A, A64 = to_dev(inputs.normal((m, k), seed=1720), dt)
    B, B64 = to_dev(inputs.normal((k, n), seed=1721), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=1722), dt)
    note("split stages backward", dt, case)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=dt, p=p, K=K)
    dA2, dB2 = hs.hs_gemm_backward(A, B, G, dtype=dt, p=p, K=K)
    torch.cuda.synchronize()
    assert torch.equal(dA, dA2) and torch.equal(dB, dB2)
    rA, rB = oracle.backward(A64, B64, G64)
    check(host(dA), rA, dt, G64, B64.T, what="split stages dA %s" % (case,))
    check(host(dB), rB, dt, A64.T, G64, what="split stages dB %s" % (case,))
    got_i, ref_i, _, _ = _gemm_case(dt, m, n, k, p, K, False, seed=1730, gen=inputs.small_int)
    assert np.array_equal(got_i, ref_i)


@pytest.mark.parametrize("dt", ["fp8_e4m3", "fp8_e4m3_r1"])
@pytest.mark.parametrize("case", [(256, 256, 16384, 4, 2), (512, 256, 8192, 8, 2)])
def test_split_stage_sequence_fp8(dt, case):
    """The FP8 forms on split stage sequences (their block scales follow
    each workgroup's first stage): FP8 gates against the oracle, small
    integers bit for bit."""
    from oracle.metrics import err_elem
    m, n, k, p, K = case
    got, ref, A64, B64 = _gemm_case(dt, m, n, k, p, K, False, seed=1740 + m, gen=inputs.uniform)
    assert err_row(got, ref) <= TOL[dt], (dt, case, err_row(got, ref))
    if dt == "fp8_e4m3_r1":
        assert err_elem(got, ref, oracle.absprod(A64, B64)) <= FP8_R1_ELEM
    got_i, ref_i, _, _ = _gemm_case(dt, m, n, k, p, K, False, seed=1750, gen=inputs.small_int)
    assert np.array_equal(got_i, ref_i)


def test_many_virtual_processors():
    """p = 256 (K = 16) and p = 4096 (K = 64) on small matrices."""
    _skip_no_gpu()
    for (m, n, k, p, K) in [(512, 384, 512, 256, 16), (4096, 64, 4096, 4096, 64)]:
        got, ref, A64, B64 = _gemm_case("f32", m, n, k, p, K, False, seed=101)
        check(got, ref, "f32", A64, B64, what="p=%d K=%d" % (p, K))


# ---------------------------------------------------------------------------
# FP8 e4m3 with 128 x 128 power-of-two tile scales (plain and refined)
# ---------------------------------------------------------------------------
FP8 = ["fp8_e4m3", "fp8_e4m3_r1"]
# shapes with contraction blocks of whole 64-chunks and 32-row stripes
FP8_CASES = [(256, 256, 512, 4, 2), (512, 200, 1024, 8, 2), (320, 96, 640, 10, 1), (1024, 768, 2048, 16, 4),
             (256, 300, 4096, 8, 8)]


@pytest.mark.parametrize("dt", FP8)
@pytest.mark.parametrize("case", FP8_CASES)
@pytest.mark.parametrize("tn", [False, True])
def test_fp8_forms(dt, case, tn):
    from oracle.metrics import err_elem
    m, n, k, p, K = case
    got, ref, _, _ = _gemm_case(dt, m, n, k, p, K, tn, seed=2000 + m + k)
    assert not np.isnan(got).any()
    e = err_row(got, ref)
    assert e <= TOL[dt], (dt, case, tn, e)
    if dt == "fp8_e4m3_r1":
        A = inputs.uniform((k, m) if tn else (m, k), seed=2000 + m + k)
        B = inputs.uniform((k, n), seed=2001 + m + k)
        Af = A.astype(np.float32).astype(np.float64)
        Bf = B.astype(np.float32).astype(np.float64)
        absprod = oracle.gemm_tn(np.abs(Af), np.abs(Bf)) if tn else oracle.gemm(np.abs(Af), np.abs(Bf))
        assert err_elem(got, ref, absprod) <= FP8_R1_ELEM


@pytest.mark.parametrize("dt", FP8)
@pytest.mark.parametrize("case", [(256, 256, 512, 4, 2), (512, 200, 1024, 8, 1)])
def test_fp8_small_int_bit_exact(dt, case):
    """Integers |x| <= 8 are exact in e4m3 under a power-of-two tile scale."""
    m, n, k, p, K = case
    got, ref, _, _ = _gemm_case(dt, m, n, k, p, K, False, seed=78, gen=inputs.small_int)
    assert np.array_equal(got, ref)


def test_fp8_unsupported_alignment():
    _skip_no_gpu()
    A, _ = to_dev(inputs.uniform((100, 96), seed=1), "fp8_e4m3")
    B, _ = to_dev(inputs.uniform((96, 64), seed=2), "fp8_e4m3")
    with pytest.raises(hs.HsError) as e:
        hs.hs_gemm(A, B, dtype="fp8_e4m3", p=2)       # blocks of 48: not whole 64-chunks
    assert e.value.status == 2


def test_fp8_r1_config_16384():
    """A 16384 x 8192, B 8192 x 16384, U[-1, 1], FP8 refined, forward and
    backward; error on 256 seeded sampled rows of C, dA and dB."""
    _skip_no_gpu()
    from oracle.metrics import err_elem
    m, k, n = 16384, 8192, 16384
    A, A64 = to_dev(inputs.uniform((m, k), seed=inputs.BASE_SEED + 4), "fp8_e4m3_r1")
    B, B64 = to_dev(inputs.uniform((k, n), seed=inputs.BASE_SEED + 5), "fp8_e4m3_r1")
    G, G64 = to_dev(inputs.normal((m, n), seed=inputs.BASE_SEED + 6), "fp8_e4m3_r1")
    note("fp8 r1 16384")
    C = hs.hs_gemm(A, B, dtype="fp8_e4m3_r1", p=64)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype="fp8_e4m3_r1", p=64)
    torch.cuda.synchronize()
    rm = inputs.sample_rows(m, 256, seed=46)
    rk = inputs.sample_rows(k, 256, seed=47)
    refC = oracle.gemm_rows(A64, B64, rm)
    eC = err_row(host(C)[rm], refC)
    absC = oracle.gemm_rows(np.abs(A64), np.abs(B64), rm)
    eCe = err_elem(host(C)[rm], refC, absC)
    eA = err_row(host(dA)[rm], oracle.grad_a_rows(G64, B64, rm))
    eB = err_row(host(dB)[rk], oracle.grad_b_rows(A64, G64, rk))
    print("fp8 r1 16384: err_row C %.3e dA %.3e dB %.3e err_elem C %.3e" % (eC, eA, eB, eCe))
    assert max(eC, eA, eB) <= 1e-2 and eCe <= FP8_R1_ELEM


# ---------------------------------------------------------------------------
# The pieces themselves.  A product with a diagonal (or identity) operand
# has one nonzero term per output element, so the output shows each
# element's split or quantisation, for both operand roles and every
# orientation (NN, TN, and NT through the backward call).  The diagonal
# holds signed powers of two, so every partial sum is exact whatever the
# MFMA's internal alignment and rounding (which differ from a sequence of
# IEEE FP32 additions); the split is then pinned by exact reconstruction,
# a = a0 + a1 + a2, and the quantisation by oracle.precision bit for bit.
# ---------------------------------------------------------------------------
def _pow2_diag(n, seed):
    g = np.random.default_rng(seed)
    d = g.choice([-1.0, 1.0], n) * 2.0 ** g.integers(-6, 7, n)
    return np.diag(d), d


# Split products on contiguous sources, whose pieces the pack kernels form
# from 16-byte loads (whole 8-element units), and on the same values as
# views with odd row strides (element loads): three stripes per tile
# (640 x 512 x 384), ragged rows and columns, K = p, K = 1.
PACK_LOAD_CASES = [(640, 512, 384, 8, 2), (250, 300, 512, 4, 4), (1024, 1024, 1024, 16, 16), (77, 45, 64, 4, 1),
                (768, 768, 768, 3, 1), (512, 1024, 2048, 8, 4)]


def _strided(x64, dt, pad=1):
    """The same values as a view whose rows are cols + pad floats apart (not
    16-byte aligned: the pack kernels then read element by element)."""
    r, c = x64.shape
    big = np.zeros((r, c + pad))
    big[:, :c] = x64
    t, _ = to_dev(big, dt)
    return t[:, :c]


@pytest.mark.parametrize("dt", ["split3_bf16", "split2_f16"])
@pytest.mark.parametrize("case", PACK_LOAD_CASES)
def test_split_pack_load_paths(dt, case):
    """The split forms on contiguous sources against the oracle, and bit for
    bit against the same values read through odd row strides, for C = A.B,
    A^T.B and the backward pair (both source orientations of both
    operands; for the two-piece FP16 form also both row-amax kernels)."""
    _skip_no_gpu()
    m, n, k, p, K = case
    A, A64 = to_dev(inputs.row_scaled((m, k), seed=1601), dt)
    At, At64 = to_dev(np.ascontiguousarray(A64.T), dt)
    B_, B64 = to_dev(inputs.row_scaled((k, n), seed=1602), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=1603), dt)
    Av, Atv, Bv, Gv = _strided(A64, dt), _strided(At64, dt, 3), _strided(B64, dt), _strided(G64, dt, 2)
    note("split contiguous", dt, case)
    C = hs.hs_gemm(A, B_, dtype=dt, p=p, K=K)
    Ct = hs.hs_gemm_tn(At, B_, dtype=dt, p=p, K=K)
    dA, dB = hs.hs_gemm_backward(A, B_, G, dtype=dt, p=p, K=K)
    note("split strided", dt, case)
    Cp = hs.hs_gemm(Av, Bv, dtype=dt, p=p, K=K)
    Ctp = hs.hs_gemm_tn(Atv, Bv, dtype=dt, p=p, K=K)
    dAp, dBp = hs.hs_gemm_backward(Av, Bv, Gv, dtype=dt, p=p, K=K)
    torch.cuda.synchronize()
    for x, y in ((C, Cp), (Ct, Ctp), (dA, dAp), (dB, dBp)):
        assert torch.equal(x, y)
    ref = oracle.gemm(A64, B64)
    check(host(C), ref, dt, A64, B64, what="pack paths C %s" % (case,))
    check(host(Ct), ref, dt, A64, B64, what="pack paths C tn %s" % (case,))
    rA, rB = oracle.backward(A64, B64, G64)
    check(host(dA), rA, dt, G64, B64.T, what="pack paths dA %s" % (case,))
    check(host(dB), rB, dt, A64.T, G64, what="pack paths dB %s" % (case,))


@pytest.mark.parametrize("tn", [False, True])
@pytest.mark.parametrize("p", [4, 3])
def test_split3_pieces_reconstruct_exactly(tn, p):
    """p = 4 and p = 3 (contraction blocks of 80 and 107: whole and ragged
    chunks)."""
    _skip_no_gpu()
    m, k = 200, 320
    A, Af = to_dev(inputs.row_scaled((k, m) if tn else (m, k), seed=901), "split3_bf16")
    D64, d = _pow2_diag(k, 902)
    D, _ = to_dev(D64, "split3_bf16")
    note("split pieces, static side, tn=%s" % tn)
    C = (hs.hs_gemm_tn if tn else hs.hs_gemm)(A, D, dtype="split3_bf16", p=p, K=2 if p % 2 == 0 else 1)
    Aop = Af.T if tn else Af                       # the operand as it multiplies
    assert np.array_equal(host(C), Aop * d[None, :])
    # travelling side: diag(d) . B
    B, Bf = to_dev(inputs.row_scaled((k, m), seed=903), "split3_bf16")
    note("split pieces, travelling side, tn=%s" % tn)
    C2 = (hs.hs_gemm_tn if tn else hs.hs_gemm)(D, B, dtype="split3_bf16", p=p, K=2 if p % 2 == 0 else 1)
    assert np.array_equal(host(C2), d[:, None] * Bf)


@pytest.mark.parametrize("p", [4, 3])
def test_split3_pieces_reconstruct_exactly_backward(p):
    """dA = G . B^T (NT) with B diagonal, dB = A^T . G (TN) with A diagonal;
    p = 4 and p = 3 (whole and ragged chunks)."""
    _skip_no_gpu()
    n = 256
    G, Gf = to_dev(inputs.row_scaled((n, n), seed=904), "split3_bf16")
    DA64, da = _pow2_diag(n, 905)
    DB64, db = _pow2_diag(n, 906)
    DA, _ = to_dev(DA64, "split3_bf16")
    DB, _ = to_dev(DB64, "split3_bf16")
    note("split pieces, backward")
    dA, dB = hs.hs_gemm_backward(DA, DB, G, dtype="split3_bf16", p=p, K=1)
    assert np.array_equal(host(dA), Gf * db[None, :])
    assert np.array_equal(host(dB), da[:, None] * Gf)


@pytest.mark.parametrize("tn", [False, True])
@pytest.mark.parametrize("p", [4, 3])
def test_split2_pieces_bit_exact(tn, p):
    """The two-piece FP16 form's pieces and row scales, bit for bit against
    oracle.precision: C = A . D with D a diagonal of signed powers of two is
    exactly (a0 + a1) 2^-e d (D's rows scale to 2^14 exactly, one nonzero
    product per output), the value the oracle assigns to each element; the
    same on the travelling side (D . B, scales per column of B)."""
    from oracle import precision as P
    _skip_no_gpu()
    dt = "split2_f16"
    m, k = 200, 320
    A, Af = to_dev(inputs.row_scaled((k, m) if tn else (m, k), seed=911), dt)
    D64, d = _pow2_diag(k, 912)
    D, _ = to_dev(D64, dt)
    note("split2 pieces, static side, tn=%s p=%d" % (tn, p))
    C = (hs.hs_gemm_tn if tn else hs.hs_gemm)(A, D, dtype=dt, p=p, K=2 if p % 2 == 0 else 1)
    Aop = Af.T if tn else Af                       # the operand as it multiplies
    assert np.array_equal(host(C), P.split2_f16_value(Aop) * d[None, :])
    B, Bf = to_dev(inputs.row_scaled((k, m), seed=913), dt)
    note("split2 pieces, travelling side, tn=%s p=%d" % (tn, p))
    C2 = (hs.hs_gemm_tn if tn else hs.hs_gemm)(D, B, dtype=dt, p=p, K=2 if p % 2 == 0 else 1)
    assert np.array_equal(host(C2), d[:, None] * P.split2_f16_value(Bf, row_axis=1))


@pytest.mark.parametrize("p", [4, 3])
def test_split2_pieces_bit_exact_backward(p):
    """dA = G . B^T with B diagonal (G's rows scaled and split), dB = A^T . G
    with A diagonal (G's columns scaled and split)."""
    from oracle import precision as P
    _skip_no_gpu()
    dt = "split2_f16"
    n = 256
    G, Gf = to_dev(inputs.row_scaled((n, n), seed=914), dt)
    DA64, da = _pow2_diag(n, 915)
    DB64, db = _pow2_diag(n, 916)
    DA, _ = to_dev(DA64, dt)
    DB, _ = to_dev(DB64, dt)
    note("split2 pieces, backward p=%d" % p)
    dA, dB = hs.hs_gemm_backward(DA, DB, G, dtype=dt, p=p, K=1)
    assert np.array_equal(host(dA), P.split2_f16_value(Gf) * db[None, :])
    assert np.array_equal(host(dB), da[:, None] * P.split2_f16_value(Gf, row_axis=1))


def test_split2_extreme_row_scales():
    """Rows spanning 2^-100 .. 2^100 (each row scaled to its own range) and
    a zero row: every row at FP32 accuracy, the zero row exactly zero."""
    _skip_no_gpu()
    dt = "split2_f16"
    m, n, k = 96, 80, 512
    g = np.random.default_rng(917)
    A64 = g.standard_normal((m, k)) * 2.0 ** g.integers(-100, 101, (m, 1))
    A64[7] = 0.0
    B64 = g.standard_normal((k, n)) * 2.0 ** g.integers(-20, 21, (1, n))
    A, Af = to_dev(A64, dt)
    B, Bf = to_dev(B64, dt)
    note("split2 extreme row scales")
    C = hs.hs_gemm(A, B, dtype=dt, p=4, K=2)
    torch.cuda.synchronize()
    got = host(C)
    check(got, oracle.gemm(Af, Bf), dt, Af, Bf, what="split2 extreme rows")
    assert not got[7].any()


@pytest.mark.parametrize("dt", FP8)
@pytest.mark.parametrize("tn", [False, True])
@pytest.mark.parametrize("mkp", [(256, 384, 2), (254, 256, 4)])
def test_fp8_quantisation_bit_exact(dt, tn, mkp):
    """A . I and I . B return the dequantised operand exactly (products with
    an exact 1 and at most one nonzero term per element).  m = 254: ragged
    scale tiles and, read along A's columns (tn), a line length that is not
    a whole number of 16-byte units."""
    _skip_no_gpu()
    from oracle import precision as P
    refine = dt == "fp8_e4m3_r1"
    m, k, p = mkp
    A, Af = to_dev(inputs.row_scaled((k, m) if tn else (m, k), seed=911), dt)
    I_k, _ = to_dev(np.eye(k), dt)
    note("fp8 quantisation, static side", dt, tn)
    C = (hs.hs_gemm_tn if tn else hs.hs_gemm)(A, I_k, dtype=dt, p=p)
    Aop = P.fp8_dequantized(Af, refine)            # 128 x 128 tiles from the origin
    assert np.array_equal(host(C), Aop.T if tn else Aop)
    B, Bf = to_dev(inputs.row_scaled((m, k), seed=912), dt)
    I_m, _ = to_dev(np.eye(m), dt)
    note("fp8 quantisation, travelling side", dt, tn)
    C2 = (hs.hs_gemm_tn if tn else hs.hs_gemm)(I_m, B, dtype=dt, p=p)
    assert np.array_equal(host(C2), P.fp8_dequantized(Bf, refine))


@pytest.mark.parametrize("dt", FP8)
def test_fp8_quantisation_ties_bit_exact(dt):
    """Every tie of the e4m3 rounding: each 128 x 128 scale tile holds 448
    (so its scale is 2^0) and every midpoint between neighbouring e4m3
    values, both signs, subnormal ones included; A . I must return the
    oracle's round-to-nearest-even dequantisation bit for bit."""
    _skip_no_gpu()
    from oracle import precision as P
    refine = dt == "fp8_e4m3_r1"
    vals = P.e4m3_table()
    mids = 0.5 * (vals[:-1] + vals[1:])
    special = np.concatenate([[448.0], mids, -mids, -vals[:8]])
    A = inputs.uniform((256, 256), seed=915) * 400.0
    for r0 in (0, 128):
        for c0 in (0, 128):
            t = A[r0:r0 + 128, c0:c0 + 128].reshape(-1)
            t[:len(special)] = special
            A[r0:r0 + 128, c0:c0 + 128] = t.reshape(128, 128)
    Ad, Af = to_dev(A, dt)
    I, _ = to_dev(np.eye(256), dt)
    note("fp8 ties", dt)
    C = hs.hs_gemm(Ad, I, dtype=dt, p=2)
    assert np.array_equal(host(C), P.fp8_dequantized(Af, refine))


@pytest.mark.parametrize("dt", FP8)
def test_fp8_quantisation_unaligned_rows(dt):
    """Operands whose rows are not 16-byte aligned (a view with row stride
    259 floats, starting one float in): the scale pass and the pack read
    them element by element; the quantisation is still bit-exact."""
    _skip_no_gpu()
    from oracle import precision as P
    refine = dt == "fp8_e4m3_r1"
    m, k = 224, 192
    big, big64 = to_dev(inputs.row_scaled((m, 259), seed=914), dt)
    A, Af = big[:, 1:1 + k], big64[:, 1:1 + k]
    I_k, _ = to_dev(np.eye(k), dt)
    note("fp8 quantisation, unaligned rows", dt)
    C = hs.hs_gemm(A, I_k, dtype=dt, p=1)
    assert np.array_equal(host(C), P.fp8_dequantized(np.ascontiguousarray(Af), refine))


@pytest.mark.parametrize("dt", FP8)
def test_fp8_quantisation_bit_exact_backward(dt):
    _skip_no_gpu()
    from oracle import precision as P
    n = 256
    G, Gf = to_dev(inputs.row_scaled((n, n), seed=913), dt)
    I, _ = to_dev(np.eye(n), dt)
    note("fp8 quantisation, backward", dt)
    dA, dB = hs.hs_gemm_backward(I, I, G, dtype=dt, p=2)
    ref = P.fp8_dequantized(Gf, dt == "fp8_e4m3_r1")
    assert np.array_equal(host(dA), ref)
    assert np.array_equal(host(dB), ref)


# ---------------------------------------------------------------------------
# Complex data (the complex workload of Sec. 7): hs_gemm on complex64, run as
# one real product of A (m x 2k) and the 2 x 2 block embedding of B.
# ---------------------------------------------------------------------------
CPLX = ["c32", "c32_split3_bf16", "c32_split2_f16"]
CPLX_CASES = [(64, 48, 80, 4, 2), (77, 45, 333, 5, 1), (256, 200, 320, 8, 0), (512, 384, 640, 16, 4),
              (130, 260, 90, 3, 3), (1, 1, 1, 1, 1)]


def _cplx_dev(shape, seed, gen=inputs.normal):
    x = gen(shape, seed) + 1j * gen(shape, seed + 1)
    t = torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64)))
    return t.cuda(), t.numpy().astype(np.complex128)


@pytest.mark.parametrize("dt", CPLX)
@pytest.mark.parametrize("case", CPLX_CASES)
def test_complex_product(dt, case):
    _skip_no_gpu()
    m, n, k, p, K = case
    A, Ah = _cplx_dev((m, k), 950 + m)
    B, Bh = _cplx_dev((k, n), 960 + n)
    out = poisoned((m, n), torch.complex64)
    note("complex", dt, case)
    C = hs.hs_gemm(A, B, dtype=dt, p=p, K=K, out=out)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.complex128)
    check(got, oracle.complex_gemm(Ah, Bh), dt, Ah, Bh, what="complex %s" % (case,))


@pytest.mark.parametrize("dt", CPLX)
def test_complex_gaussian_integers_bit_exact(dt):
    _skip_no_gpu()
    m, n, k = 200, 136, 264
    A, Ah = _cplx_dev((m, k), 970, inputs.small_int)
    B, Bh = _cplx_dev((k, n), 972, inputs.small_int)
    note("complex small int", dt)
    C = hs.hs_gemm(A, B, dtype=dt, p=8, K=2)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.complex128), oracle.complex_gemm(Ah, Bh))


@pytest.mark.parametrize("dt", CPLX)
@pytest.mark.parametrize("case", CPLX_CASES)
def test_complex_transposed_product(dt, case):
    """C = A^T B (transposed, not conjugated), A stored k x m."""
    _skip_no_gpu()
    m, n, k, p, K = case
    A, Ah = _cplx_dev((k, m), 1950 + m)
    B, Bh = _cplx_dev((k, n), 1960 + n)
    out = poisoned((m, n), torch.complex64)
    note("complex tn", dt, case)
    C = hs.hs_gemm_tn(A, B, dtype=dt, p=p, K=K, out=out)
    torch.cuda.synchronize()
    got = C.cpu().numpy().astype(np.complex128)
    check(got, oracle.complex_gemm(Ah.T, Bh), dt, Ah.T, Bh, what="complex tn %s" % (case,))


@pytest.mark.parametrize("dt", CPLX)
def test_complex_transposed_gaussian_integers_bit_exact(dt):
    _skip_no_gpu()
    m, n, k = 200, 136, 264
    A, Ah = _cplx_dev((k, m), 1970, inputs.small_int)
    B, Bh = _cplx_dev((k, n), 1972, inputs.small_int)
    note("complex tn small int", dt)
    C = hs.hs_gemm_tn(A, B, dtype=dt, p=8, K=2)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.complex128), oracle.complex_gemm(Ah.T, Bh))


# (m, n, p, K): the 8192^2 workload, ragged stripes and blocks, odd n (8-byte
# loads), the systolic case, K = p
CGEMV_CASES = [(8192, 8192, 64, 8), (1000, 778, 12, 3), (33, 17, 4, 2), (64, 64, 1, 1), (256, 300, 16, 16)]


@pytest.mark.parametrize("case", CGEMV_CASES)
def test_complex_gemv(case):
    _skip_no_gpu()
    m, n, p, K = case
    A, Ah = _cplx_dev((m, n), 2950 + m)
    x, xh = _cplx_dev((n,), 2960 + n)
    y = torch.full((m,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    note("complex gemv", case)
    hs.hs_gemv(A, x, dtype="c32", p=p, K=K, out=y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.complex128)
    check(got, oracle.complex_gemv(Ah, xh), "c32", Ah, xh[:, None], what="complex gemv %s" % (case,), vector=True)
    Ai, Aih = _cplx_dev((m, n), 2970, inputs.small_int)
    xi, xih = _cplx_dev((n,), 2972, inputs.small_int)
    yi = hs.hs_gemv(Ai, xi, dtype="c32", p=p, K=K)
    torch.cuda.synchronize()
    assert np.array_equal(yi.cpu().numpy().astype(np.complex128), oracle.complex_gemv(Aih, xih))


def test_complex_gemv_empty_contraction():
    _skip_no_gpu()
    A = torch.zeros((5, 0), dtype=torch.complex64, device="cuda")
    x = torch.zeros((0,), dtype=torch.complex64, device="cuda")
    y = hs.hs_gemv(A, x, dtype="c32", p=2, K=1)
    torch.cuda.synchronize()
    assert torch.equal(y.cpu(), torch.zeros(5, dtype=torch.complex64))


@pytest.mark.parametrize("dt", ["c32_split3_bf16", "c32_split2_f16"])
def test_complex_strided_views(dt):
    _skip_no_gpu()
    Abig, Ahb = _cplx_dev((100, 150), 980)
    Bbig, Bhb = _cplx_dev((130, 90), 982)
    A, B = Abig[:, 10:130], Bbig[5:125, :70]        # row strides 150 and 90 complex elements
    note("complex views", dt)
    C = hs.hs_gemm(A, B, dtype=dt, p=6, K=2)
    torch.cuda.synchronize()
    ref = oracle.complex_gemm(Ahb[:, 10:130], Bhb[5:125, :70])
    check(C.cpu().numpy().astype(np.complex128), ref, dt, Ahb[:, 10:130], Bhb[5:125, :70],
          what="complex views")


def _c_split2_value(Z, axis):
    """What each element of complex Z stands for in the complex two-piece
    FP16 form: re and im split as in oracle.precision, with one scale per
    row (axis 0) or column (axis 1) from the largest |re| or |im| in it."""
    from oracle import precision as P
    Zr = Z if axis == 0 else Z.T
    out = np.empty_like(Zr)
    for r in range(Zr.shape[0]):
        e = P.row_exponent(max(np.max(np.abs(Zr[r].real)), np.max(np.abs(Zr[r].imag))))

        def v(x):
            xs = x * 2.0 ** e
            a0 = P.f16(xs)
            return (a0 + P.f16(xs - a0)) * 2.0 ** -e
        out[r] = v(Zr[r].real) + 1j * v(Zr[r].imag)
    return out if axis == 0 else out.T


@pytest.mark.parametrize("p", [4, 3])
def test_complex_split2_pieces_bit_exact(p):
    """Every embedding of the complex two-piece FP16 form against the pieces
    and scales oracle.precision assigns, bit for bit, through diagonals of
    signed powers of two (one nonzero product per output element): A.D
    (rows of A scaled), D.B (columns of B), At^T.D (columns of At), and the
    backward pair with G = D: dA = D.B^H (rows of B), dB = A^H.D (columns
    of A)."""
    _skip_no_gpu()
    dt = "c32_split2_f16"
    n, k = 120, 96
    g = np.random.default_rng(990 + p)
    d = g.choice([-1.0, 1.0], n) * 2.0 ** g.integers(-6, 7, n)
    dk = d[:k]
    Dn = torch.from_numpy(np.diag(d).astype(np.complex64)).cuda()
    Dk = torch.from_numpy(np.diag(dk).astype(np.complex64)).cuda()
    A, Ah = _cplx_dev((n, k), 991, inputs.row_scaled)         # A n x k
    B, Bh = _cplx_dev((k, n), 993, inputs.row_scaled)         # B k x n
    B2, B2h = _cplx_dev((n, k), 995, inputs.row_scaled)       # travelling side of Dn . B2
    At, Ath = _cplx_dev((n, k), 997, inputs.row_scaled)       # At^T . Dn
    note("complex split2 pieces p=%d" % p)
    C1 = hs.hs_gemm(A, Dk, dtype=dt, p=p, K=1)
    C2 = hs.hs_gemm(Dn, B2, dtype=dt, p=p, K=1)
    C3 = hs.hs_gemm_tn(At, Dn, dtype=dt, p=p, K=1)
    dA, dB = hs.hs_gemm_backward(A, B, Dn, dtype=dt, p=p, K=1)
    torch.cuda.synchronize()
    host_c = lambda t: t.cpu().numpy().astype(np.complex128)
    assert np.array_equal(host_c(C1), _c_split2_value(Ah, 0) * dk[None, :])
    assert np.array_equal(host_c(C2), d[:, None] * _c_split2_value(B2h, 1))
    assert np.array_equal(host_c(C3), _c_split2_value(Ath, 1).T * d[None, :])
    assert np.array_equal(host_c(dA), d[:, None] * np.conj(_c_split2_value(Bh, 0)).T)
    assert np.array_equal(host_c(dB), np.conj(_c_split2_value(Ah, 1)).T * d[None, :])


def test_complex_4096_sampled_rows():
    """n = 4096 complex, p = 64, both forms, on 32 sampled rows."""
    _skip_no_gpu()
    n = 4096
    A, Ah = _cplx_dev((n, n), 990)
    B, Bh = _cplx_dev((n, n), 992)
    rows = inputs.sample_rows(n, 32, seed=994)
    ref = oracle.complex_gemm_rows(Ah, Bh, rows)
    for dt in CPLX:
        note("complex 4096", dt)
        C = hs.hs_gemm(A, B, dtype=dt, p=64, K=8)
        torch.cuda.synchronize()
        check(C.cpu().numpy().astype(np.complex128)[rows], ref, dt, Ah[rows], Bh, what="complex n=4096")


def test_complex_bench_step_n8192():
    """The complex workload exactly as bench.py times it: n = 8192 complex64
    N(0, 1) inputs with its seeds, its step (C = A.B, dA = G.B^H,
    dB = A^H.G on p = 64, K = 2), both forms; 8 sampled rows of each."""
    _skip_no_gpu()
    import bench
    n, p, K = 8192, 64, 2
    g = inputs.normal
    A64 = g((n, n), inputs.BASE_SEED + 20) + 1j * g((n, n), inputs.BASE_SEED + 21)
    B64 = g((n, n), inputs.BASE_SEED + 22) + 1j * g((n, n), inputs.BASE_SEED + 23)
    G64 = g((n, n), inputs.BASE_SEED + 24) + 1j * g((n, n), inputs.BASE_SEED + 25)
    A = torch.from_numpy(A64.astype(np.complex64)).cuda()
    B = torch.from_numpy(B64.astype(np.complex64)).cuda()
    G = torch.from_numpy(G64.astype(np.complex64)).cuda()
    Ah, Bh, Gh = (t.cpu().numpy().astype(np.complex128) for t in (A, B, G))
    del A64, B64, G64
    rows = inputs.sample_rows(n, 8, seed=47)
    refs = (oracle.complex_gemm_rows(Ah, Bh, rows),
            oracle.complex_gemm_rows(Gh, np.conj(Bh).T, rows),
            oracle.complex_gemm_rows(np.conj(Ah).T, Gh, rows))
    ops = ((Ah[rows], Bh), (Gh[rows], Bh.T), (Ah[:, rows].T, Gh))
    for dt in CPLX:
        note("complex bench step", dt)
        outs = bench.step(hs, A, B, G, dt, p, K)
        torch.cuda.synchronize()
        for o, r, (X, Y), name in zip(outs, refs, ops, ("C", "dA", "dB")):
            check(o.cpu().numpy().astype(np.complex128)[rows], r, dt, X, Y, what="complex step " + name)


CPLX_BW_CASES = [(64, 48, 80, 4, 2), (77, 45, 133, 5, 1), (256, 200, 320, 8, 0), (130, 260, 90, 3, 3)]


@pytest.mark.parametrize("dt", CPLX)
@pytest.mark.parametrize("case", CPLX_BW_CASES)
def test_complex_backward(dt, case):
    """dA = G . B^H and dB = A^H . G (PyTorch's convention for complex
    gradients) against the oracle."""
    _skip_no_gpu()
    m, n, k, p, K = case
    A, Ah = _cplx_dev((m, k), 1000 + m)
    B, Bh = _cplx_dev((k, n), 1010 + n)
    G, Gh = _cplx_dev((m, n), 1020 + k)
    note("complex backward", dt, case)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=dt, p=p, K=K)
    torch.cuda.synchronize()
    check(dA.cpu().numpy().astype(np.complex128), oracle.complex_gemm(Gh, np.conj(Bh).T), dt, Gh, Bh.T,
          what="complex backward dA %s" % (case,))
    check(dB.cpu().numpy().astype(np.complex128), oracle.complex_gemm(np.conj(Ah).T, Gh), dt, Ah.T, Gh,
          what="complex backward dB %s" % (case,))


@pytest.mark.parametrize("dt", CPLX)
def test_complex_backward_gaussian_integers_bit_exact(dt):
    _skip_no_gpu()
    m, n, k = 136, 200, 72
    A, Ah = _cplx_dev((m, k), 1030, inputs.small_int)
    B, Bh = _cplx_dev((k, n), 1032, inputs.small_int)
    G, Gh = _cplx_dev((m, n), 1034, inputs.small_int)
    note("complex backward small int", dt)
    dA, dB = hs.hs_gemm_backward(A, B, G, dtype=dt, p=8, K=2)
    torch.cuda.synchronize()
    assert np.array_equal(dA.cpu().numpy().astype(np.complex128), oracle.complex_gemm(Gh, np.conj(Bh).T))
    assert np.array_equal(dB.cpu().numpy().astype(np.complex128), oracle.complex_gemm(np.conj(Ah).T, Gh))


@pytest.mark.parametrize("dt", ["c32_split3_bf16", "c32_split2_f16"])
def test_complex_autograd(dt):
    _skip_no_gpu()
    m, k, n = 96, 64, 80
    A, Ah = _cplx_dev((m, k), 1040)
    B, Bh = _cplx_dev((k, n), 1042)
    G, Gh = _cplx_dev((m, n), 1044)
    A.requires_grad_(True)
    B.requires_grad_(True)
    note("complex autograd", dt)
    C = hs_autograd.matmul(A, B, dtype=dt, p=4, K=2)
    C.backward(G)
    torch.cuda.synchronize()
    check(C.detach().cpu().numpy().astype(np.complex128), oracle.complex_gemm(Ah, Bh), dt, Ah, Bh,
          what="complex autograd C")
    check(A.grad.cpu().numpy().astype(np.complex128), oracle.complex_gemm(Gh, np.conj(Bh).T), dt, Gh, Bh.T,
          what="complex autograd dA")
    check(B.grad.cpu().numpy().astype(np.complex128), oracle.complex_gemm(np.conj(Ah).T, Gh), dt, Ah.T, Gh,
          what="complex autograd dB")


@pytest.mark.parametrize("dt", ["f32", "split3_bf16"])
def test_tall_product_k8(dt):
    """M = 16384, p = 64, K = 8: stripes of 256 rows, one per tile, eight
    partials per output tile collected in registers; a ragged last column
    tile."""
    _skip_no_gpu()
    m, k, n, p, K = 16384, 256, 2000, 64, 8
    A, A64 = to_dev(inputs.normal((m, k), seed=1101), dt)
    B, B64 = to_dev(inputs.normal((k, n), seed=1102), dt)
    note("tall product K=8", dt)
    C = hs.hs_gemm(A, B, dtype=dt, p=p, K=K, out=poisoned((m, n), torch.float32))
    torch.cuda.synchronize()
    got = host(C)
    assert not np.isnan(got).any()
    rows = inputs.sample_rows(m, 64, seed=1103)
    check(got[rows], oracle.gemm_rows(A64, B64, rows), dt, A64[rows], B64, what="M=16384 K=8")
    Ai, Ai64 = to_dev(inputs.small_int((m, k), seed=1104), dt)
    Bi, Bi64 = to_dev(inputs.small_int((k, n), seed=1105), dt)
    Ci = host(hs.hs_gemm(Ai, Bi, dtype=dt, p=p, K=K))
    assert np.array_equal(Ci[rows], oracle.gemm_rows(Ai64, Bi64, rows))


def test_packed_operand_of_3gib():
    """Split A of 32768 x 16384: 3 GiB of packed pieces, including the copies
    of the last K - 1 stripes ahead of stripe 0."""
    _skip_no_gpu()
    m, k, n, p, K = 32768, 16384, 256, 64, 2
    Ai, Ai64 = to_dev(inputs.small_int((m, k), seed=1201), "split3_bf16")
    Bi, Bi64 = to_dev(inputs.small_int((k, n), seed=1202), "split3_bf16")
    note("near 4 GiB packed operand")
    C = host(hs.hs_gemm(Ai, Bi, dtype="split3_bf16", p=p, K=K))
    rows = np.concatenate([inputs.sample_rows(m, 32, seed=1203), [0, m - 1]])
    assert np.array_equal(C[rows], oracle.gemm_rows(Ai64, Bi64, rows))
    del Ai, Bi
    torch.cuda.empty_cache()


def test_operand_above_4gib():
    """FP32 A of 40960 x 32768 packs to 5.4 GB: more than 32-bit offsets
    reach, so each workgroup addresses its own region of it (K stripe groups
    of A, one column group of B).  Small integers, exact on sampled rows."""
    _skip_no_gpu()
    m, k, n, p, K = 40960, 32768, 256, 64, 2
    g = inputs.rng(1301)
    A8 = g.integers(-8, 9, size=(m, k), dtype=np.int8)
    B64 = inputs.small_int((k, n), seed=1302)
    A = torch.from_numpy(A8).cuda().float()
    B = torch.from_numpy(B64).float().cuda()
    note("operand above 4 GiB")
    C = host(hs.hs_gemm(A, B, dtype="f32", p=p, K=K))
    rows = np.concatenate([inputs.sample_rows(m, 24, seed=1303), [0, m - 1]])
    assert np.array_equal(C[rows], oracle.gemm_rows(A8[rows].astype(np.float64), B64, np.arange(len(rows))))
    del A, B
    torch.cuda.empty_cache()


def test_expanded_operand_rejected_before_launch():
    """An expanded A (row stride 0) is refused by the binding, not read
    past its 32-byte storage."""
    _skip_no_gpu()
    A = torch.randn(1, 8, device="cuda").expand(5, 8)
    B = torch.randn(8, 4, device="cuda")
    note("expanded operand")
    with pytest.raises(ValueError, match="overlapping rows"):
        hs.hs_gemm(A, B, dtype="f32", p=1)
    with pytest.raises(ValueError, match="overlapping rows"):
        hs_autograd.matmul(A, B, dtype="f32", p=1)


@pytest.mark.parametrize("dt", ["f32", "split3_bf16"])
def test_explicit_side_stream(dt):
    """Calls given a stream that is not the current one allocate their
    workspace and outputs on that stream; results equal the current-stream
    calls bit for bit, for every entry point."""
    _skip_no_gpu()
    m, k, n, p, K = 640, 384, 520, 8, 2
    A, A64 = to_dev(inputs.normal((m, k), seed=1401), dt)
    Bm, B64 = to_dev(inputs.normal((k, n), seed=1402), dt)
    G, G64 = to_dev(inputs.normal((m, n), seed=1403), dt)
    x, _ = to_dev(inputs.normal((k,), seed=1404), "f32")
    X = torch.from_numpy(inputs.plummer(700, seed=1405, unequal=True)).float().cuda()
    At = A.t().contiguous()
    torch.cuda.synchronize()
    note("side stream", dt)
    ref = (hs.hs_gemm(A, Bm, dtype=dt, p=p, K=K), hs.hs_gemm_tn(At, Bm, dtype=dt, p=p, K=K),
           *hs.hs_gemm_backward(A, Bm, G, dtype=dt, p=p, K=K), hs.hs_gemv(A.float(), x, p=p, K=K),
           hs.hs_nbody(X, 1e-4, p=p, K=K))
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for _ in range(3):                 # the allocator gets to reuse freed blocks in between
        got = (hs.hs_gemm(A, Bm, dtype=dt, p=p, K=K, stream=s),
               hs.hs_gemm_tn(At, Bm, dtype=dt, p=p, K=K, stream=s),
               *hs.hs_gemm_backward(A, Bm, G, dtype=dt, p=p, K=K, stream=s),
               hs.hs_gemv(A.float(), x, p=p, K=K, stream=s), hs.hs_nbody(X, 1e-4, p=p, K=K, stream=s))
        junk = torch.randn(4 << 20, device="cuda")   # current-stream work on freshly freed memory
        junk.mul_(2.0)
        s.synchronize()
        for r, g in zip(ref, got):
            assert torch.equal(r, g)
    check(host(ref[0]), oracle.gemm(A64, B64), dt, A64, B64, what="side stream C")
