"""hs_gemm_noalloc: the product with the library's static scratch array as its
workspace (for callers that cannot allocate), called through the C ABI and
compared with hs_gemm bit for bit on the same inputs: two calls in a row,
the second smaller, so a result cannot lean on what the first left in the
scratch array; plus the size limit, refused before any launch."""
import numpy as np
import pytest

import oracle
from paper_cs_9809105_amd import binding as B
from paper_cs_9809105_amd import inputs
from tests._gpu import check, gpu_available, note, poisoned, to_dev

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_cs_9809105_amd as hs


def _skip_no_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dt", ["split3_bf16", "f32", "f64", "fp8_e4m3_r1", "split2_f16"])
def test_noalloc_equals_gemm_two_calls(dt):
    _skip_no_gpu()
    fp8 = dt.startswith("fp8")
    # (m, n, k, p, K): a large call, then a smaller one with another schedule
    cases = ([(1024, 768, 1024, 8, 2), (256, 320, 512, 4, 4)] if fp8 else
             [(1100, 900, 1000, 8, 2), (300, 200, 150, 5, 1)])
    for i, (m, n, k, p, K) in enumerate(cases):
        A, A64 = to_dev(inputs.normal((m, k), seed=1500 + i), dt)
        Bm, B64 = to_dev(inputs.normal((k, n), seed=1510 + i), dt)
        od = torch.float64 if dt == "f64" else torch.float32
        need = B.hs_workspace_size(B.HS_OP_GEMM, m, n, k, dt, p, K)
        assert 0 < need <= B.HS_NOALLOC_SCRATCH_BYTES
        note("noalloc", dt, (m, n, k), (p, K), "call", i)
        ref = hs.hs_gemm(A, Bm, dtype=dt, p=p, K=K, out=poisoned((m, n), od))
        got = hs.hs_gemm_noalloc(A, Bm, poisoned((m, n), od), dtype=dt, p=p, K=K)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (dt, i)
        if not fp8:
            check(got.cpu().double().numpy(), oracle.gemm(A64, B64), dt, A64, B64, what="noalloc %d" % i)


@pytest.mark.parametrize("dt", ["split3_bf16", "split2_f16", "f32"])
def test_noalloc_split_stage_sequence(dt):
    """A long contraction on few output tiles (its stage sequence split over
    workgroups, their planes in the scratch array), then a small product:
    both equal to hs_gemm."""
    _skip_no_gpu()
    for i, (m, n, k, p, K) in enumerate([(256, 256, 16384, 4, 2), (96, 80, 200, 4, 1)]):
        A, A64 = to_dev(inputs.normal((m, k), seed=1540 + i), dt)
        Bm, B64 = to_dev(inputs.normal((k, n), seed=1545 + i), dt)
        assert 0 < B.hs_workspace_size(B.HS_OP_GEMM, m, n, k, dt, p, K) <= B.HS_NOALLOC_SCRATCH_BYTES
        note("noalloc split", dt, (m, n, k), (p, K), "call", i)
        ref = hs.hs_gemm(A, Bm, dtype=dt, p=p, K=K, out=poisoned((m, n), torch.float32))
        got = hs.hs_gemm_noalloc(A, Bm, poisoned((m, n), torch.float32), dtype=dt, p=p, K=K)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (dt, i)
        check(got.cpu().double().numpy(), oracle.gemm(A64, B64), dt, A64, B64, what="noalloc split %d" % i)


def test_noalloc_on_a_stream_in_a_row():
    """Back-to-back calls on one side stream (ordered by the stream), each
    equal to hs_gemm."""
    _skip_no_gpu()
    s = torch.cuda.Stream()
    outs, refs = [], []
    for i, (m, n, k) in enumerate([(700, 500, 600), (129, 65, 257), (512, 512, 512)]):
        A, _ = to_dev(inputs.uniform((m, k), seed=1520 + i), "split3_bf16")
        Bm, _ = to_dev(inputs.uniform((k, n), seed=1530 + i), "split3_bf16")
        refs.append(hs.hs_gemm(A, Bm, dtype="split3_bf16", p=4, K=2))
        torch.cuda.synchronize()
        out = torch.empty((m, n), dtype=torch.float32, device="cuda")
        note("noalloc stream", i)
        outs.append(hs.hs_gemm_noalloc(A, Bm, out, dtype="split3_bf16", p=4, K=2, stream=s))
    s.synchronize()
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)


def test_noalloc_limit_refused_before_launch():
    _skip_no_gpu()
    m = n = k = 4096           # split-BF16: about 200 MB of packed operands
    assert B.hs_workspace_size(B.HS_OP_GEMM, m, n, k, "split3_bf16", 8, 2) > B.HS_NOALLOC_SCRATCH_BYTES
    A = torch.zeros((m, k), device="cuda")
    Bm = torch.zeros((k, n), device="cuda")
    C = torch.full((m, n), 7.0, device="cuda")
    with pytest.raises(B.HsError) as e:
        hs.hs_gemm_noalloc(A, Bm, C, dtype="split3_bf16", p=8, K=2)
    assert e.value.status == B.HS_ERR_EXCEEDS_SCRATCH
    torch.cuda.synchronize()
    assert bool((C == 7.0).all())          # nothing was launched
    # invalid arguments keep hs_gemm's own status
    L = B.lib()
    st = L.hs_gemm_noalloc(8, 8, 8, B.HS_F32, B.hs_schedule(4, 3), A.data_ptr(), 8, Bm.data_ptr(), 8,
                           C.data_ptr(), 8, None)
    assert st == B.HS_ERR_INVALID_VALUE
    # empty shapes: nothing to do, no scratch needed
    assert L.hs_gemm_noalloc(0, 8, 8, B.HS_F32, B.hs_schedule(4, 2), A.data_ptr(), 8, Bm.data_ptr(), 8,
                             C.data_ptr(), 8, None) == B.HS_OK
