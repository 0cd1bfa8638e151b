"""torch.autograd.Function over the hyper-systolic product.

Forward is hs_gemm; backward is hs_gemm_backward (dA = G . B^T on the NT
form of the schedule, dB = A^T . G on the transposed-product form).  Both run
in the library's HIP kernels; this module only routes tensors.
"""
import torch

from . import binding


class HsMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, dtype="f32", p=1, K=0):
        if binding._dt(dtype) in (binding.HS_BF16, binding.HS_F16):
            # the gradient G arrives in fp32; a 16-bit backward would need a
            # cast outside the library, so these forms are forward-only
            raise NotImplementedError("autograd needs an fp32/fp64-input form")
        ctx.save_for_backward(A, B)
        ctx.cfg = (dtype, p, K)
        return binding.hs_gemm(A, B, dtype=dtype, p=p, K=K)

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        dtype, p, K = ctx.cfg
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        G = G.contiguous()
        dA, dB = binding.hs_gemm_backward(A, B, G, dtype=dtype, p=p, K=K,
                                          need_a=need_a, need_b=need_b)
        return dA, dB, None, None, None


def matmul(A, B, dtype="f32", p=1, K=0):
    """Differentiable C = A . B on the hyper-systolic schedule (p, K)."""
    return HsMatmul.apply(A, B, dtype, p, K)
