"""The C ABI under HIP graph capture (GPU).

The library launches kernels only on the caller's stream and needs no
memset (zero fills are kernels), so its calls can be captured into a graph.
Each test captures calls into a torch.cuda.CUDAGraph, then replays it
several times with eager calls of the library and synchronisations in
between, and checks every replay bit for bit against the eager result (the
library is deterministic run to run).
"""
import numpy as np
import pytest

from paper_cs_9809105_amd import inputs
from tests._gpu import gpu_available, note

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_cs_9809105_amd as hs


def _skip_no_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def test_graph_replays_match_eager():
    _skip_no_gpu()
    m, k, n, p, K = 1024, 768, 1536, 8, 2
    A = torch.from_numpy(inputs.normal((m, k), 51)).float().cuda()
    B = torch.from_numpy(inputs.normal((k, n), 52)).float().cuda()
    G = torch.from_numpy(inputs.normal((m, n), 53)).float().cuda()
    X = torch.from_numpy(inputs.plummer(3000, 54)).float().cuda()
    note("graph: eager reference")
    C_ref = hs.hs_gemm(A, B, dtype="split3_bf16", p=p, K=K)
    dA_ref, dB_ref = hs.hs_gemm_backward(A, B, G, dtype="split3_bf16", p=p, K=K)
    F_ref = hs.hs_nbody(X, 1e-4, p=16, K=4)
    torch.cuda.synchronize()

    C = torch.empty_like(C_ref)
    F = torch.empty_like(F_ref)
    outs = {}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):                  # warm the allocator outside capture
        hs.hs_gemm(A, B, dtype="split3_bf16", p=p, K=K, out=C)
        hs.hs_nbody(X, 1e-4, p=16, K=4, out=F)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    note("graph: capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hs.hs_gemm(A, B, dtype="split3_bf16", p=p, K=K, out=C)
        outs["dA"], outs["dB"] = hs.hs_gemm_backward(A, B, G, dtype="split3_bf16", p=p, K=K)
        hs.hs_nbody(X, 1e-4, p=16, K=4, out=F)
    for r in range(4):
        C.fill_(float("nan"))
        F.fill_(float("nan"))
        outs["dA"].fill_(float("nan"))
        outs["dB"].fill_(float("nan"))
        torch.cuda.synchronize()
        note("graph: replay", r)
        g.replay()
        # eager work of the program between replays
        hs.hs_gemm(B.t().contiguous(), A.t().contiguous(), dtype="f32", p=4, K=2)
        torch.cuda.synchronize()
        assert torch.equal(C, C_ref), r
        assert torch.equal(outs["dA"], dA_ref) and torch.equal(outs["dB"], dB_ref), r
        assert torch.equal(F, F_ref), r


def test_graph_of_k8_product_and_complex():
    """A K = 8 product (every output tile collects eight partials) at a
    size with many workgroups, and a complex product, captured together."""
    _skip_no_gpu()
    m, k, n = 4096, 512, 4096                   # p = 64, K = 8: 64-row stripes, 4 per tile
    A = torch.from_numpy(inputs.normal((m, k), 61)).float().cuda()
    B = torch.from_numpy(inputs.normal((k, n), 62)).float().cuda()
    Z = torch.from_numpy((inputs.normal((300, 200), 63) + 1j * inputs.normal((300, 200), 64))
                         .astype(np.complex64)).cuda()
    W = torch.from_numpy((inputs.normal((200, 100), 65) + 1j * inputs.normal((200, 100), 66))
                         .astype(np.complex64)).cuda()
    note("graph k8: eager reference")
    C_ref = hs.hs_gemm(A, B, dtype="f32", p=64, K=8)
    Y_ref = hs.hs_gemm(Z, W, dtype="c32_split3_bf16", p=4, K=2)
    torch.cuda.synchronize()
    C = torch.empty_like(C_ref)
    Y = torch.empty_like(Y_ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        hs.hs_gemm(A, B, dtype="f32", p=64, K=8, out=C)
        hs.hs_gemm(Z, W, dtype="c32_split3_bf16", p=4, K=2, out=Y)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    note("graph k8: capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hs.hs_gemm(A, B, dtype="f32", p=64, K=8, out=C)
        hs.hs_gemm(Z, W, dtype="c32_split3_bf16", p=4, K=2, out=Y)
    for r in range(3):
        C.fill_(float("nan"))
        Y.fill_(complex(float("nan"), 0.0))
        torch.cuda.synchronize()
        note("graph k8: replay", r)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, C_ref), r
        assert torch.equal(Y, Y_ref), r
