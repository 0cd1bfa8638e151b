"""Hyper-systolic matrix products (and the all-pairs n-body interaction on
the two-array recipe) on AMD MI355X (gfx950).

The computation lives in ``libhs.so`` (HIP kernels + C ABI, include/hs.h);
``binding`` marshals PyTorch tensors into it and ``autograd`` wraps the
forward and backward products as a ``torch.autograd.Function``.  Importing
the package loads nothing; the library is loaded on first use and its
absence is an error.
"""
from .binding import (  # noqa: F401
    HsError, hs_gemm, hs_gemm_backward, hs_gemm_noalloc, hs_gemm_tn, hs_gemv, hs_nbody, hs_profile_begin,
    hs_profile_end, hs_schedule_resolve, hs_schedule_table, hs_status_string,
    hs_workspace_size,
)
