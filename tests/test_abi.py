"""Host-side tests of the C ABI (CPU only: no kernel is launched).

* the library loads and exports every function include/hs.h declares;
* the schedule (index map) equals the event trace of the ring simulator of
  Algorithm HYPER-SYSTOLIC applied to C^T = B^T A^T;
* every invalid argument is rejected with its status code before any launch.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import bases, ring
from paper_cs_9809105_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert {"hs_gemm", "hs_gemm_tn", "hs_gemv", "hs_gemm_backward"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_binding_names_match_abi():
    import paper_cs_9809105_amd as pkg
    for name in _declared():
        assert hasattr(B, name), name
    for name in ("hs_gemm", "hs_gemm_tn", "hs_gemv", "hs_gemm_backward"):
        assert getattr(pkg, name) is getattr(B, name)


def test_status_strings():
    for s in range(6):
        assert B.hs_status_string(s).startswith("HS_")
    assert B.hs_status_string(99) == "unknown hs_status"
    assert B.hs_status_string(-1) == "unknown hs_status"


@pytest.mark.parametrize("p", [1, 2, 4, 6, 9, 12, 16, 36, 64, 100])
def test_default_K_minimises_shifts(p):
    _, K = B.hs_schedule_resolve(p, 0)
    cost = K + p // K - 1
    assert p % K == 0
    assert cost == min(d + p // d - 1 for d in range(1, p + 1) if p % d == 0)
    if int(round(p ** 0.5)) ** 2 == p:
        assert K == int(round(p ** 0.5))


@pytest.mark.parametrize("p,K", [(0, 0), (-1, 1), (4097, 1), (8, 3), (8, 16), (6, -2)])
def test_invalid_schedules(p, K):
    with pytest.raises(B.HsError) as e:
        B.hs_schedule_resolve(p, K)
    assert e.value.status == B.HS_ERR_INVALID_VALUE


def _sim_table(p, K):
    """(output stripe, contraction block) per (v, j, l) from the ring simulator.

    The paper's algorithm keeps columns and moves A; the library keeps rows
    and moves B, i.e. it runs the algorithm on C^T = B^T A^T.  Paper element
    PA[r, c] stands for B block (c, r) and PB[r, c] for A block (c, r)."""
    PA, PB = ring.leaves("PA", p), ring.leaves("PB", p)
    trace = []
    ring.hyper_systolic(PA, PB, K, ring.Term(), trace=trace)
    ev = {}
    for (i, j, l, n, ae, be) in trace:
        assert ae.c == be.r                     # contraction blocks agree
        ev.setdefault((i, j, l), set()).add((be.c, ae.c))
    rows = []
    for v in range(p):
        for j in range(p // K):
            for l in range(K):
                s = ev[(v, j, l)]
                assert len(s) == 1
                rows.append(next(iter(s)))
    return np.array(rows, dtype=np.int32)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8, 9, 12, 16])
def test_schedule_table_equals_ring_simulation(p):
    for K in [d for d in range(1, p + 1) if p % d == 0]:
        assert np.array_equal(B.hs_schedule_table(p, K), _sim_table(p, K)), (p, K)


@pytest.mark.parametrize("p,K", [(64, 8), (64, 2), (256, 16), (48, 6), (4096, 64)])
def test_schedule_covers_every_block_product_once(p, K):
    t = B.hs_schedule_table(p, K)
    pairs = {(int(r), int(kb)) for r, kb in t}
    assert len(t) == p * p and len(pairs) == p * p
    # base A: successive steps of one virtual processor differ by K
    t3 = t.reshape(p, p // K, K, 2)
    assert np.all((np.diff(t3[:, :, 0, 1], axis=1) % p) == K % p)
    # pre-shift base B and back-shift base C: partial l of v feeds stripe v - l
    v = np.arange(p)[:, None]
    assert np.array_equal(t3[:, 0, :, 0], (v - np.arange(K)[None, :]) % p)
    # shift count of Thm. GAIN3 for this (p, K)
    assert bases.shifts_matrix_product(K, p // K) == K + p // K - 1


def test_schedule_table_small_buffer():
    buf = (ctypes.c_int32 * 7)()
    st = B.lib().hs_schedule_table(B.hs_schedule(4, 2), buf, 7)
    assert st == B.HS_ERR_INVALID_VALUE


def test_fp8_workspace_sizes():
    ws = B.hs_workspace_size
    s1 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "fp8_e4m3", 8, 2)
    s2 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "fp8_e4m3_r1", 8, 2)
    assert s1 != B.SIZE_MAX and s2 > s1            # q1 pieces
    assert ws(B.HS_OP_GEMM, 64, 64, 96, "fp8_e4m3", 2) == B.SIZE_MAX
    assert ws(B.HS_OP_BACKWARD, 16384, 16384, 8192, "fp8_e4m3_r1", 64) != B.SIZE_MAX


def test_workspace_sizes():
    ws = B.hs_workspace_size
    assert ws(B.HS_OP_GEMM, 0, 10, 10, "f32", 2) == 0
    assert ws(B.HS_OP_GEMM, 10, 10, 0, "f32", 2) == 0
    assert ws(B.HS_OP_GEMV, 100, 100, 0, "f32", 4) == 0
    assert ws(B.HS_OP_GEMV, 100, 100, 0, "bf16", 4) == B.SIZE_MAX
    assert ws(B.HS_OP_GEMM, 10, 10, 10, "f32", 3, 2) == B.SIZE_MAX
    assert ws(B.HS_OP_GEMM, 10, 10, 10, 99, 2) == B.SIZE_MAX
    # dtype and op are plain ints in the ABI: any value is a defined input
    assert ws(B.HS_OP_GEMM, 10, 10, 10, -1, 2) == B.SIZE_MAX
    assert ws(99, 10, 10, 10, "f32", 2) == B.SIZE_MAX
    assert ws(-7, 10, 10, 10, "f32", 2) == B.SIZE_MAX
    s1 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "f32", 8, 1)
    s2 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "f32", 8, 2)
    s8 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "f32", 8, 8)
    # no partial planes: the collector keeps the K partials in registers,
    # so the workspace (the packed operands) does not grow with K
    assert s1 == s2 == s8
    # K may exceed the tile's rows (one stripe per tile then)
    assert ws(B.HS_OP_GEMM, 64, 64, 64, "f32", 512, 512) not in (0, B.SIZE_MAX)
    s3 = ws(B.HS_OP_GEMM, 1024, 1024, 1024, "split3_bf16", 8, 1)
    assert s3 > s1                                 # three bf16 pieces per operand
    for n in (B.HS_OP_GEMM, B.HS_OP_GEMM_TN, B.HS_OP_BACKWARD):
        assert ws(n, 512, 384, 256, "f64", 16, 4) % 256 == 0
    assert ws(B.HS_OP_BACKWARD, 64, 128, 32, "f32", 4, 2) >= ws(B.HS_OP_GEMM, 64, 32, 128, "f32", 4, 2)


# ---------------------------------------------------------------------------
# argument validation: every failure returns before any launch
# ---------------------------------------------------------------------------
FAKE = 1 << 20          # aligned, never dereferenced on the host


def _gemm(**kw):
    a = dict(m=8, n=8, k=8, dt=B.HS_F32, p=2, K=0, A=FAKE, lda=8, Bp=FAKE, ldb=8, C=FAKE,
             ldc=8, ws=FAKE, wsb=1 << 30, st=None)
    a.update(kw)
    return B.lib().hs_gemm(a["m"], a["n"], a["k"], a["dt"], B.hs_schedule(a["p"], a["K"]), a["A"],
                           a["lda"], a["Bp"], a["ldb"], a["C"], a["ldc"], a["ws"], a["wsb"], a["st"])


@pytest.mark.parametrize("kw,code", [
    (dict(m=-1), B.HS_ERR_INVALID_VALUE),
    (dict(lda=7), B.HS_ERR_INVALID_VALUE),
    (dict(ldb=4), B.HS_ERR_INVALID_VALUE),
    (dict(ldc=0), B.HS_ERR_INVALID_VALUE),
    (dict(A=None), B.HS_ERR_INVALID_VALUE),
    (dict(Bp=None), B.HS_ERR_INVALID_VALUE),
    (dict(C=None), B.HS_ERR_INVALID_VALUE),
    (dict(A=FAKE + 2), B.HS_ERR_INVALID_VALUE),
    (dict(p=0), B.HS_ERR_INVALID_VALUE),
    (dict(p=4, K=3), B.HS_ERR_INVALID_VALUE),
    (dict(dt=17), B.HS_ERR_NOT_SUPPORTED),
    (dict(ws=None), B.HS_ERR_WORKSPACE_TOO_SMALL),
    (dict(wsb=16), B.HS_ERR_WORKSPACE_TOO_SMALL),
    (dict(ws=FAKE + 64), B.HS_ERR_INVALID_VALUE),
    # FP8: contraction blocks must be whole 64-element chunks, stripes 32-row aligned
    (dict(dt=B.HS_FP8_E4M3, m=64, n=64, k=96, lda=96, ldb=64, ldc=64, p=2), B.HS_ERR_NOT_SUPPORTED),
    (dict(dt=B.HS_FP8_E4M3_R1, m=48, n=64, k=128, lda=128, ldb=64, ldc=64, p=2), B.HS_ERR_NOT_SUPPORTED),
    (dict(dt=B.HS_FP8_E4M3_R1, m=256, n=64, k=768, lda=768, ldb=64, ldc=64, p=4, K=3), B.HS_ERR_INVALID_VALUE),
    # complex: 8-byte elements, ld in complex elements, workspace of the 2k x 2n embedding
    (dict(dt=B.HS_C32, A=FAKE + 4), B.HS_ERR_INVALID_VALUE),
    (dict(dt=B.HS_C32_SPLIT3_BF16, C=FAKE + 4), B.HS_ERR_INVALID_VALUE),
    (dict(dt=B.HS_C32, ldb=7), B.HS_ERR_INVALID_VALUE),
    (dict(dt=B.HS_C32, wsb=16), B.HS_ERR_WORKSPACE_TOO_SMALL),
    (dict(dt=B.HS_C32, k=-1), B.HS_ERR_INVALID_VALUE),
])
def test_gemm_rejects(kw, code):
    assert _gemm(**kw) == code


def test_gemm_tn_rejects_bad_lda():
    L = B.lib()
    # A is k x m: lda must be >= m
    st = L.hs_gemm_tn(8, 8, 16, B.HS_F32, B.hs_schedule(2, 0), FAKE, 4, FAKE, 8, FAKE, 8,
                      FAKE, 1 << 30, None)
    assert st == B.HS_ERR_INVALID_VALUE


def test_gemv_rejects():
    L = B.lib()
    s = B.hs_schedule(2, 0)
    assert L.hs_gemv(8, 8, B.HS_BF16, s, FAKE, 8, FAKE, FAKE, None, 0, None) == B.HS_ERR_NOT_SUPPORTED
    assert L.hs_gemv(8, 8, B.HS_F32, s, FAKE, 4, FAKE, FAKE, None, 0, None) == B.HS_ERR_INVALID_VALUE
    assert L.hs_gemv(8, 8, B.HS_F32, s, FAKE, 8, None, FAKE, None, 0, None) == B.HS_ERR_INVALID_VALUE
    assert L.hs_gemv(8, 8, B.HS_F32, s, FAKE, 8, FAKE, None, None, 0, None) == B.HS_ERR_INVALID_VALUE
    assert L.hs_gemv(8, 8, B.HS_F32, B.hs_schedule(3, 2), FAKE, 8, FAKE, FAKE, None, 0, None) == \
        B.HS_ERR_INVALID_VALUE
    assert L.hs_gemv(0, 8, B.HS_F32, s, None, 8, None, None, None, 0, None) == B.HS_OK


def test_backward_rejects():
    L = B.lib()
    s = B.hs_schedule(2, 0)
    args = [8, 8, 8, B.HS_F32, s, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 1 << 30, None]
    bad = list(args)
    bad[9] = None                      # G missing
    assert L.hs_gemm_backward(*bad) == B.HS_ERR_INVALID_VALUE
    bad = list(args)
    bad[16] = 8                        # workspace too small
    assert L.hs_gemm_backward(*bad) == B.HS_ERR_WORKSPACE_TOO_SMALL
    bad = list(args)
    bad[12] = 4                        # ldda < k
    assert L.hs_gemm_backward(*bad) == B.HS_ERR_INVALID_VALUE
    both_null = list(args)
    both_null[11] = None
    both_null[13] = None
    assert L.hs_gemm_backward(*both_null) == B.HS_OK   # nothing to do


def test_empty_problems_need_nothing():
    assert _gemm(m=0, A=None, C=None, ws=None, wsb=0) == B.HS_OK
    assert _gemm(n=0, Bp=None, C=None, ws=None, wsb=0) == B.HS_OK


def test_profile_end_without_begin():
    assert B.lib().hs_profile_end(None, None) == B.HS_ERR_INVALID_VALUE


def test_complex_forms_argument_checks():
    L = B.lib()
    s = B.hs_schedule(2, 0)
    for dt in (B.HS_C32, B.HS_C32_SPLIT3_BF16, B.HS_C32_SPLIT2_F16):
        # transposed product: checks in complex elements, before any launch
        tn = [8, 8, 8, dt, s, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 1 << 30, None]
        bad = list(tn)
        bad[5] = FAKE + 4                      # A not 8-byte aligned
        assert L.hs_gemm_tn(*bad) == B.HS_ERR_INVALID_VALUE
        bad = list(tn)
        bad[6] = 7                             # lda < m (A is k x m)
        assert L.hs_gemm_tn(*bad) == B.HS_ERR_INVALID_VALUE
        bad = list(tn)
        bad[12] = 8
        assert L.hs_gemm_tn(*bad) == B.HS_ERR_WORKSPACE_TOO_SMALL
        # backward: argument checks in complex elements, before any launch
        args = [8, 8, 8, dt, s, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 1 << 30, None]
        bad = list(args)
        bad[9] = FAKE + 4                      # G not 8-byte aligned
        assert L.hs_gemm_backward(*bad) == B.HS_ERR_INVALID_VALUE
        bad = list(args)
        bad[16] = 8
        assert L.hs_gemm_backward(*bad) == B.HS_ERR_WORKSPACE_TOO_SMALL
    # matrix-vector: complex64 in FP32 arithmetic only
    gv = [8, 8, B.HS_C32, s, FAKE, 8, FAKE, FAKE, None, 0, None]
    assert L.hs_gemv(8, 8, B.HS_C32_SPLIT3_BF16, s, FAKE, 8, FAKE, FAKE, None, 0, None) == B.HS_ERR_NOT_SUPPORTED
    assert L.hs_gemv(8, 8, B.HS_C32_SPLIT2_F16, s, FAKE, 8, FAKE, FAKE, None, 0, None) == B.HS_ERR_NOT_SUPPORTED
    bad = list(gv)
    bad[4] = FAKE + 4                          # A not 8-byte aligned
    assert L.hs_gemv(*bad) == B.HS_ERR_INVALID_VALUE
    bad = list(gv)
    bad[5] = 7                                 # lda < n
    assert L.hs_gemv(*bad) == B.HS_ERR_INVALID_VALUE
    bad = list(gv)
    bad[6] = FAKE + 4                          # x not 8-byte aligned
    assert L.hs_gemv(*bad) == B.HS_ERR_INVALID_VALUE
    assert B.hs_workspace_size(B.HS_OP_GEMV, 64, 64, 0, "c32", 4) == 0
    assert B.hs_workspace_size(B.HS_OP_GEMV, 64, 64, 0, "c32_split3_bf16", 4) == B.SIZE_MAX


def test_complex_workspace_is_that_of_the_real_embedding():
    ws = B.hs_workspace_size
    for (m, n, k, p, K) in [(64, 48, 80, 4, 2), (300, 200, 100, 8, 0), (128, 128, 128, 16, 4)]:
        assert ws(B.HS_OP_GEMM, m, n, k, "c32", p, K) == ws(B.HS_OP_GEMM, m, 2 * n, 2 * k, "f32", p, K)
        assert ws(B.HS_OP_GEMM, m, n, k, "c32_split3_bf16", p, K) == \
            ws(B.HS_OP_GEMM, m, 2 * n, 2 * k, "split3_bf16", p, K)
        assert ws(B.HS_OP_GEMM, m, n, k, "c32_split2_f16", p, K) == \
            ws(B.HS_OP_GEMM, m, 2 * n, 2 * k, "split2_f16", p, K)
        assert ws(B.HS_OP_GEMM_TN, m, n, k, "c32", p, K) == ws(B.HS_OP_GEMM_TN, m, 2 * n, 2 * k, "f32", p, K)
        # backward: dA = G . B^H (m x 2k reals, contraction 2n), dB = A^H . G (k x 2n, contraction 2m)
        assert ws(B.HS_OP_BACKWARD, m, n, k, "c32", p, K) == max(ws(B.HS_OP_GEMM, m, 2 * k, 2 * n, "f32", p, K),
                                                                ws(B.HS_OP_GEMM, k, 2 * n, 2 * m, "f32", p, K))


def test_size_limits_are_reported_not_run():
    """A workgroup addresses its region of each packed operand (its stripe
    groups of the static operand, one column group of the travelling one)
    with 32-bit offsets, so operands far above 4 GiB are fine, but a region
    above 4 GiB is HS_ERR_NOT_SUPPORTED."""
    ws = B.hs_workspace_size
    # split A of 3 x 32768 x 24576 x 2 bytes = 4.5 GiB packed: fine
    assert ws(B.HS_OP_GEMM, 32768, 256, 24576, "split3_bf16", 64, 2) != B.SIZE_MAX
    # a column group of B: 3 pieces x 2^21 x 256 columns x 2 bytes = 3 GiB: fine
    assert ws(B.HS_OP_GEMM, 4096, 256, 1 << 21, "split3_bf16", 64, 2) != B.SIZE_MAX
    # 6 GiB: too large for one workgroup's offsets
    assert ws(B.HS_OP_GEMM, 4096, 256, 1 << 22, "split3_bf16", 64, 2) == B.SIZE_MAX
    assert _gemm(m=4096, n=256, k=1 << 22, dt=B.HS_SPLIT3_BF16, p=64, K=2, lda=1 << 22, ldb=256,
                 ldc=256) == B.HS_ERR_NOT_SUPPORTED


# ---------------------------------------------------------------------------
# hs_nbody: argument checks and workspace (no launch)
# ---------------------------------------------------------------------------
FAKE = 1 << 40          # a 256-aligned address that is never dereferenced


def _nbody(n, dt=B.HS_F32, p=4, K=2, bodies=FAKE, eps2=0.0, out=FAKE + (1 << 32), ws=FAKE + (1 << 33),
           nb=1 << 30):
    return B.lib().hs_nbody(n, dt, B.hs_schedule(p, K), bodies, eps2, out, ws, nb, None)


def test_nbody_workspace_is_k_partial_planes():
    ws = B.hs_workspace_size
    assert ws(B.HS_OP_NBODY, 1000, 0, 0, "f32", 16, 4) == 4 * 1000 * 16
    assert ws(B.HS_OP_NBODY, 1000, 0, 0, "f64", 16, 4) == 4 * 1000 * 32
    assert ws(B.HS_OP_NBODY, 1000, 0, 0, "f32", 16, 1) == 0          # systolic: writes out directly
    assert ws(B.HS_OP_NBODY, 1001, 0, 0, "f32", 8, 2) % 256 == 0
    assert ws(B.HS_OP_NBODY, 0, 0, 0, "f32", 8, 2) == 0
    assert ws(B.HS_OP_NBODY, 100, 0, 0, "bf16", 8, 2) == B.SIZE_MAX
    assert ws(B.HS_OP_NBODY, -1, 0, 0, "f32", 8, 2) == B.SIZE_MAX
    assert ws(B.HS_OP_NBODY, 100, 0, 0, "f32", 8, 3) == B.SIZE_MAX
    assert ws(B.HS_OP_NBODY, 1 << 31, 0, 0, "f32", 8, 2) == B.SIZE_MAX


def test_nbody_rejects_bad_arguments():
    E = B.HS_ERR_INVALID_VALUE
    assert _nbody(0) == B.HS_OK                                    # nothing to do
    assert _nbody(10, dt=B.HS_BF16) == B.HS_ERR_NOT_SUPPORTED
    assert _nbody(10, dt=B.HS_SPLIT3_BF16) == B.HS_ERR_NOT_SUPPORTED
    assert _nbody(-1) == E
    assert _nbody(10, p=6, K=4) == E                               # K must divide p
    assert _nbody(10, eps2=-1e-3) == E
    assert _nbody(10, eps2=float("nan")) == E
    assert _nbody(10, eps2=float("inf")) == E
    assert _nbody(10, eps2=1e39) == E                              # not a float
    assert _nbody(10, bodies=None) == E
    assert _nbody(10, out=None) == E
    assert _nbody(10, bodies=FAKE + 8) == E                        # one body = 16 bytes
    assert _nbody(10, dt=B.HS_F64, bodies=FAKE + 16) == E          # one body = 32 bytes
    assert _nbody(10, out=FAKE + 16 * 9) == E                      # overlaps the bodies
    assert _nbody(10, out=FAKE - 16 * 9) == E
    assert _nbody(10, ws=None) == B.HS_ERR_WORKSPACE_TOO_SMALL
    assert _nbody(10, nb=2 * 10 * 16 - 1) == B.HS_ERR_WORKSPACE_TOO_SMALL
    assert _nbody(10, ws=FAKE + (1 << 33) + 64) == E               # workspace alignment
    assert _nbody(1 << 31, ws=None, nb=0, K=1) == B.HS_ERR_NOT_SUPPORTED


def test_dimensions_of_2_31_or_more_are_not_supported():
    """Each dimension must stay below 2^31 (products of two then fit in 64
    bits); above, every call is rejected before any launch."""
    ws = B.hs_workspace_size
    big = 1 << 31
    for op in (B.HS_OP_GEMM, B.HS_OP_GEMM_TN, B.HS_OP_BACKWARD):
        assert ws(op, big, 8, 8, "f32", 4, 2) == B.SIZE_MAX
        assert ws(op, 8, big, 8, "f32", 4, 2) == B.SIZE_MAX
        assert ws(op, 8, 8, big, "f32", 4, 2) == B.SIZE_MAX
        assert ws(op, 1 << 40, 1 << 40, 1 << 30, "f32", 1, 1) == B.SIZE_MAX
    assert ws(B.HS_OP_GEMM, 8, 1 << 30, 8, "c32", 4, 2) == B.SIZE_MAX     # 2n reals
    assert _gemm(m=big, n=8, k=8, lda=8, ldb=8, ldc=8) == B.HS_ERR_NOT_SUPPORTED
    L = B.lib()
    assert L.hs_gemv(big, 8, B.HS_F32, B.hs_schedule(4, 2), FAKE, 8, FAKE, FAKE, None, 0, None) == \
        B.HS_ERR_NOT_SUPPORTED


def test_row_layout_rejects_overlapping_rows():
    """A view whose rows overlap (an expanded tensor: row stride 0) would let
    the pack kernels read past its storage; the binding refuses it before
    any launch.  Shapes and strides as torch reports them."""
    # torch.randn(1, 8).expand(5, 8): shape (5, 8), strides (0, 1)
    with pytest.raises(ValueError, match="overlapping rows"):
        B.row_layout((5, 8), (0, 1), "A")
    # a row stride below the row length
    with pytest.raises(ValueError, match="overlapping rows"):
        B.row_layout((3, 8), (4, 1), "A")
    # elements of a row not contiguous (a transposed view)
    with pytest.raises(ValueError, match="unit stride"):
        B.row_layout((4, 6), (1, 4), "A")
    # contiguous, padded rows, one row (any row stride), empty
    assert B.row_layout((5, 8), (8, 1)) == 8
    assert B.row_layout((5, 8), (10, 1)) == 10
    assert B.row_layout((1, 8), (0, 1)) == 8
    assert B.row_layout((0, 8), (8, 1)) == 8
    assert B.row_layout((3, 0), (1, 1)) == 1
    # a single column: any row stride >= 1 addresses distinct rows
    assert B.row_layout((4, 1), (3, 2)) == 3


def test_noalloc_rejects_before_any_launch():
    """hs_gemm_noalloc refuses a call whose workspace exceeds its static
    scratch (and keeps hs_gemm's status for invalid arguments) before it
    touches the device."""
    L = B.lib()
    s = B.hs_schedule(8, 2)
    assert B.hs_workspace_size(B.HS_OP_GEMM, 4096, 4096, 4096, "split3_bf16", 8, 2) > B.HS_NOALLOC_SCRATCH_BYTES
    assert L.hs_gemm_noalloc(4096, 4096, 4096, B.HS_SPLIT3_BF16, s, FAKE, 4096, FAKE, 4096, FAKE, 4096,
                             None) == B.HS_ERR_EXCEEDS_SCRATCH
    assert L.hs_gemm_noalloc(8, 8, 8, B.HS_F32, B.hs_schedule(4, 3), FAKE, 8, FAKE, 8, FAKE, 8,
                             None) == B.HS_ERR_INVALID_VALUE
    assert L.hs_gemm_noalloc(8, 8, 8, 99, s, FAKE, 8, FAKE, 8, FAKE, 8, None) == B.HS_ERR_NOT_SUPPORTED
    assert L.hs_gemm_noalloc(8, 8, 8, B.HS_F32, s, FAKE, 4, FAKE, 8, FAKE, 8, None) == B.HS_ERR_INVALID_VALUE
    assert B.hs_status_string(B.HS_ERR_EXCEEDS_SCRATCH).startswith("HS_ERR_EXCEEDS_SCRATCH")


def test_split_planes_in_workspace():
    """One 256 x 256 output tile pair (p = 4, K = 2: two classes) over a long
    contraction splits each tile's 1024 stages over 4 workgroups, whose FP32
    planes (4 x 256 x 256 x 4 bytes) join the packed operands (16 MiB each:
    4 stripes x 4 blocks x 512 chunks x 64 rows x 32 bytes, and 4 blocks x
    512 chunks x 256 columns x 32 bytes); with 64 stages (k = 1024) there is
    no split and the workspace is the packed operands alone (1 MiB each)."""
    ws = B.hs_workspace_size
    assert ws(B.HS_OP_GEMM, 256, 256, 16384, "f32", 4, 2) == 32 * 2 ** 20 + 4 * 256 * 256 * 4
    assert ws(B.HS_OP_GEMM, 256, 256, 1024, "f32", 4, 2) == 2 * 2 ** 20
    # 1024 output tiles (n = 8192): no split, operands only
    assert ws(B.HS_OP_GEMM, 8192, 8192, 8192, "f32", 64, 2) == 2 * 8192 * 8192 * 4


def test_header_is_plain_c(tmp_path):
    """include/hs.h compiles as C99 and as C++ with every warning an error,
    and a C caller can name every declared entry point, type and constant
    (a C ABI: no C++ in the signatures)."""
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use_hs.c"
    src.write_text(
        '#include "hs.h"\n'
        "int use(void) {\n"
        "    hs_schedule s = {64, 2};\n"
        "    hs_schedule r;\n"
        "    int32_t table[8];\n"
        "    size_t ws = hs_workspace_size(HS_OP_GEMM, 8, 8, 8, HS_SPLIT2_F16, s);\n"
        "    hs_status st = hs_schedule_resolve(s, &r);\n"
        "    (void)hs_schedule_table(s, table, 8);\n"
        "    (void)hs_status_string(st);\n"
        "    (void)hs_gemm(8, 8, 8, HS_F32, s, 0, 8, 0, 8, 0, 8, 0, 0, 0);\n"
        "    (void)hs_gemm_tn(8, 8, 8, HS_C32_SPLIT2_F16, s, 0, 8, 0, 8, 0, 8, 0, 0, 0);\n"
        "    (void)hs_gemv(8, 8, HS_F64, s, 0, 8, 0, 0, 0, 0, 0);\n"
        "    (void)hs_gemm_backward(8, 8, 8, HS_SPLIT3_BF16, s, 0, 8, 0, 8, 0, 8, 0, 8, 0, 8, 0, 0, 0);\n"
        "    (void)hs_nbody(8, HS_F32, s, 0, 0.0, 0, 0, 0, 0);\n"
        "    (void)hs_gemm_noalloc(8, 8, 8, HS_FP8_E4M3_R1, s, 0, 8, 0, 8, 0, 8, 0);\n"
        "    (void)hs_profile_begin();\n"
        "    return (int)ws + (int)HS_NOALLOC_SCRATCH_BYTES + HS_ERR_EXCEEDS_SCRATCH;\n"
        "}\n")
    for cmd in (["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-c"],
                ["g++", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-x", "c++", "-c"]):
        r = subprocess.run(cmd + ["-I", inc, str(src), "-o", str(tmp_path / "use_hs.o")],
                           stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert r.returncode == 0, (cmd[0], r.stdout)
