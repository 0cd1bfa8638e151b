"""Helpers for the GPU parity tests: device transfer and storage rounding.

Inputs are drawn in float64 (paper_cs_9809105_amd.inputs), rounded once to
the storage type, and the *same* rounded values go to the GPU and, promoted
back to float64, to the oracle.
"""
import sys

import numpy as np

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None

STORAGE = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16",
           "split3_bf16": "float32", "fp8_e4m3": "float32", "fp8_e4m3_r1": "float32",
           "split2_f16": "float32"}


def gpu_available():
    return torch is not None and torch.cuda.is_available()


def note(*args):
    """Name the case before a GPU step, so a fault can be traced to it."""
    print("[gpu-case]", *args, file=sys.stderr, flush=True)


def to_dev(x64, dtype):
    """float64 numpy -> (device tensor in storage type, float64 numpy of the stored values)."""
    t = torch.from_numpy(np.ascontiguousarray(x64)).to(getattr(torch, STORAGE[dtype]))
    stored = t.to(torch.float64).numpy()
    return t.cuda(), stored


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def poisoned(shape, dtype, device="cuda"):
    """Output buffer pre-filled with NaN to expose elements never written."""
    return torch.full(shape, float("nan"), dtype=dtype, device=device)


# ---------------------------------------------------------------------------
# parity gates
# ---------------------------------------------------------------------------
# err_row (relative 2-norm per row): the stated tolerances of each form
ROW_TOL = {"f64": 1e-12, "f32": 1e-5, "split3_bf16": 1e-5, "split2_f16": 1e-5, "bf16": 1.5e-2, "f16": 3e-3,
           "fp8_e4m3": 1e-1, "fp8_e4m3_r1": 1e-2, "c32": 1e-5, "c32_split3_bf16": 1e-5, "c32_split2_f16": 1e-5}
# err_term (element error over u sqrt(k sum_t (a_t b_t)^2), the statistical
# scale of a dot product's rounding errors) for the FP32-accurate and FP64
# forms: 16 u.  Round-to-nearest FP32 accumulation of the workloads' inputs
# measures 0.5 - 0.7 u; a lone wrong element is caught once its error
# passes 16 u sqrt(k) of its own magnitude (8.6e-5 at k = 8192), where the
# row gate needs 1e-5 sqrt(n) (9e-4 at n = 8192).
TERM_C = {"f64": 16, "f32": 16, "split3_bf16": 16, "split2_f16": 16}
# Element-wise bound |dC_ij| <= (c k + d) u (|A||B|)_ij, u the unit roundoff
# of the accumulator (FP32 2^-24, FP64 2^-53), k the contraction length:
#   * every product a_ik b_kj of the stored inputs enters one accumulator
#     chain; each addition errs by less than one unit in the last place of
#     its result (< 2u relative, also where the MFMA truncates the aligned
#     smaller addend), and every partial sum is at most sum |a||b|;
#   * plain forms: at most k additions plus the final rounding:
#     (2k + 1) u <= 3 k u;
#   * split-BF16: 6 products per term, so at most 6k additions (12 k u), plus
#     the dropped pieces a1 b2 + a2 b1 + a2 b2 and the residual of the
#     3-piece split (each operand a = a0 + a1 + a2 + r, |r| <= u |a|):
#     under 4.1 u per term, and the kept pieces' absolute sum exceeds
#     |a||b| by at most 2^-6: (13 k + 5) u;
#   * two-piece FP16 (products of the row-scaled operands, scaled back
#     exactly): 3 products per term, so at most 3k additions (6 k u) on
#     partial sums up to (1 + 2^-10) sum |a||b|; the representation
#     a' = a0 + a1 + r with |r| <= 2^-22 |a'| (4 u) and the dropped a1 b1
#     (|a1| <= 2^-11 |a'|: 4 u) leave at most 3 (4 u) + 4 u = 12 u per term
#     (elements under 2^-17 of their row's max can carry a further absolute
#     2^-39 of that max from a subnormal a1, far inside the margin of the
#     round-up below): (7 k + 13) u;
#   * complex forms run as a real product of contraction 2k.
ELEM_C = {"f64": (3, 0), "f32": (3, 0), "bf16": (3, 0), "f16": (3, 0), "split3_bf16": (13, 5),
          "split2_f16": (7, 13)}
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -24, "f16": 2.0 ** -24, "split3_bf16": 2.0 ** -24,
        "split2_f16": 2.0 ** -24}
COMPLEX_BASE = {"c32": "f32", "c32_split3_bf16": "split3_bf16", "c32_split2_f16": "split2_f16"}


def _base(dt, k):
    """(real form, contraction of the real product) of form ``dt``."""
    return (COMPLEX_BASE[dt], 2 * k) if dt in COMPLEX_BASE else (dt, k)


def elem_bound(dt, k):
    """(c k + d) u of the element-wise gate for form ``dt`` and contraction ``k``."""
    b, kk = _base(dt, k)
    c, d = ELEM_C[b]
    return (c * max(int(kk), 1) + d) * UNIT[b]


def term_bound(dt, k):
    """The err_term gate of form ``dt`` (None: not gated)."""
    b, _ = _base(dt, k)
    return TERM_C[b] * UNIT[b] if b in TERM_C else None


def check(got, ref, dt, X=None, Y=None, what="", vector=False):
    """Assert the parity gates of form ``dt`` on a result ``got`` of the
    product X . Y (X, Y the FP64 operands as they multiply, sampled rows of
    X where only those rows were compared): err_row always; err_elem <=
    (c k + d) u and, for the FP32-accurate and FP64 forms, err_term <= 16 u
    when the operands are given.  ``vector``: got and ref are the vector
    y = X . Y[:, 0], gated as one row.  Returns (err_row, err_term, err_elem)."""
    import oracle
    from oracle.metrics import err_elem, err_row, err_term
    got, ref = np.asarray(got), np.asarray(ref)
    assert not np.isnan(got).any(), (what, "NaN in the result")
    ap = sq = None
    k = None
    if X is not None:
        k = X.shape[1]
        if np.iscomplexobj(X) or np.iscomplexobj(Y):
            ap, sq = oracle.complex_absprod(X, Y), oracle.complex_sqprod(X, Y)
        else:
            ap, sq = oracle.absprod(X, Y), oracle.sqprod(X, Y)
    if vector:
        got, ref = got.reshape(1, -1), ref.reshape(1, -1)
        if ap is not None:
            ap, sq = ap.reshape(1, -1), sq.reshape(1, -1)
    er = err_row(got, ref)
    ee = err_elem(got, ref, ap) if ap is not None else None
    b, kk = _base(dt, k or 1)
    et = err_term(got, ref, sq, kk) if sq is not None else None
    tb = term_bound(dt, k or 1)
    print("[parity] %s %s: err_row %.3e err_term %s err_elem %s" %
          (what, dt, er, "-" if et is None else "%.2f u" % (et / UNIT[b]),
           "-" if ee is None else "%.3e (bound %.3e)" % (ee, elem_bound(dt, k))))
    assert er <= ROW_TOL[dt], (what, dt, "err_row", er)
    if ee is not None:
        assert ee <= elem_bound(dt, k), (what, dt, "err_elem", ee, elem_bound(dt, k))
    if et is not None and tb is not None:
        assert et <= tb, (what, dt, "err_term", et / UNIT[b])
    return er, et, ee
