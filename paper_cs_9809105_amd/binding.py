"""Thin Python binding of the C ABI in include/hs.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Tensors
are PyTorch device tensors (PyTorch supplies device memory and streams;
every step of the computation runs in the library's HIP kernels).  If the
library is missing this module raises; there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhs.so")

# hs_dtype
(HS_F64, HS_F32, HS_BF16, HS_F16, HS_SPLIT3_BF16, HS_FP8_E4M3, HS_FP8_E4M3_R1,
 HS_C32, HS_C32_SPLIT3_BF16, HS_SPLIT2_F16, HS_C32_SPLIT2_F16) = range(11)
DTYPES = {"f64": HS_F64, "f32": HS_F32, "bf16": HS_BF16, "f16": HS_F16,
          "split3_bf16": HS_SPLIT3_BF16, "fp8_e4m3": HS_FP8_E4M3, "fp8_e4m3_r1": HS_FP8_E4M3_R1,
          "c32": HS_C32, "c32_split3_bf16": HS_C32_SPLIT3_BF16, "split2_f16": HS_SPLIT2_F16,
          "c32_split2_f16": HS_C32_SPLIT2_F16}
# hs_status
(HS_OK, HS_ERR_INVALID_VALUE, HS_ERR_NOT_SUPPORTED, HS_ERR_WORKSPACE_TOO_SMALL, HS_ERR_LAUNCH_FAILED,
 HS_ERR_EXCEEDS_SCRATCH) = range(6)
HS_NOALLOC_SCRATCH_BYTES = 64 << 20
# hs_op
HS_OP_GEMM, HS_OP_GEMM_TN, HS_OP_GEMV, HS_OP_BACKWARD, HS_OP_NBODY = range(5)
SIZE_MAX = ctypes.c_size_t(-1).value


class HsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s" % (where, hs_status_string(status)))


class hs_schedule(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("K", ctypes.c_int32)]


_lib = None


def lib():
    """Load libhs.so (built in-tree by paper_cs_9809105_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhs.so is not built (%s); run paper_cs_9809105_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    L.hs_status_string.argtypes = [ctypes.c_int]
    L.hs_status_string.restype = ctypes.c_char_p
    L.hs_schedule_resolve.argtypes = [hs_schedule, ctypes.POINTER(hs_schedule)]
    L.hs_schedule_resolve.restype = ctypes.c_int
    L.hs_schedule_table.argtypes = [hs_schedule, ctypes.POINTER(i32), sz]
    L.hs_schedule_table.restype = ctypes.c_int
    L.hs_workspace_size.argtypes = [ctypes.c_int, i64, i64, i64, ctypes.c_int, hs_schedule]
    L.hs_workspace_size.restype = sz
    mm = [i64, i64, i64, ctypes.c_int, hs_schedule, vp, i64, vp, i64, vp, i64, vp, sz, vp]
    L.hs_gemm.argtypes = mm
    L.hs_gemm.restype = ctypes.c_int
    L.hs_gemm_tn.argtypes = mm
    L.hs_gemm_tn.restype = ctypes.c_int
    L.hs_gemm_noalloc.argtypes = [i64, i64, i64, ctypes.c_int, hs_schedule, vp, i64, vp, i64, vp, i64, vp]
    L.hs_gemm_noalloc.restype = ctypes.c_int
    L.hs_gemv.argtypes = [i64, i64, ctypes.c_int, hs_schedule, vp, i64, vp, vp, vp, sz, vp]
    L.hs_gemv.restype = ctypes.c_int
    L.hs_gemm_backward.argtypes = [i64, i64, i64, ctypes.c_int, hs_schedule, vp, i64, vp, i64,
                                   vp, i64, vp, i64, vp, i64, vp, sz, vp]
    L.hs_gemm_backward.restype = ctypes.c_int
    L.hs_nbody.argtypes = [i64, ctypes.c_int, hs_schedule, vp, ctypes.c_double, vp, vp, sz, vp]
    L.hs_nbody.restype = ctypes.c_int
    L.hs_profile_begin.argtypes = []
    L.hs_profile_begin.restype = ctypes.c_int
    L.hs_profile_end.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.hs_profile_end.restype = ctypes.c_int
    _lib = L
    return L


def _check(status, where):
    if status != HS_OK:
        raise HsError(status, where)


def _dt(dtype):
    return DTYPES[dtype] if isinstance(dtype, str) else int(dtype)


# ---------------------------------------------------------------------------
# host-only entry points
# ---------------------------------------------------------------------------
def hs_status_string(status):
    return lib().hs_status_string(int(status)).decode()


def hs_schedule_resolve(p, K=0):
    out = hs_schedule()
    _check(lib().hs_schedule_resolve(hs_schedule(p, K), ctypes.byref(out)), "hs_schedule_resolve")
    return out.p, out.K


def hs_schedule_table(p, K=0):
    """[(r, kb)] for v, j, l in nesting order (see include/hs.h)."""
    import numpy as np
    buf = (ctypes.c_int32 * (2 * p * p))()
    _check(lib().hs_schedule_table(hs_schedule(p, K), buf, 2 * p * p), "hs_schedule_table")
    return np.frombuffer(buf, dtype=np.int32).reshape(-1, 2).copy()


def hs_workspace_size(op, m, n, k, dtype, p, K=0):
    return lib().hs_workspace_size(int(op), m, n, k, _dt(dtype), hs_schedule(p, K))


def hs_profile_begin():
    _check(lib().hs_profile_begin(), "hs_profile_begin")


def hs_profile_end():
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().hs_profile_end(ctypes.byref(ms), ctypes.byref(n)), "hs_profile_end")
    return ms.value, n.value


# ---------------------------------------------------------------------------
# device entry points (torch tensors)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


IN_TYPES = {HS_F64: "float64", HS_F32: "float32", HS_BF16: "bfloat16", HS_F16: "float16",
            HS_SPLIT3_BF16: "float32", HS_FP8_E4M3: "float32", HS_FP8_E4M3_R1: "float32",
            HS_C32: "complex64", HS_C32_SPLIT3_BF16: "complex64", HS_SPLIT2_F16: "float32",
            HS_C32_SPLIT2_F16: "complex64"}


def _out_type(dt):
    if dt in (HS_C32, HS_C32_SPLIT3_BF16, HS_C32_SPLIT2_F16):
        return "complex64"
    return "float64" if dt == HS_F64 else "float32"


def row_layout(shape, strides, name="tensor"):
    """Leading dimension of a 2-D row-major view with this shape and these
    strides (in elements), or ValueError if the C ABI cannot address it: the
    elements of a row must be contiguous, and rows may not overlap (a view
    whose row stride is below its row length, such as an expanded tensor
    with stride 0, would make the library read past its storage)."""
    rows, cols = shape
    if rows == 0 or cols == 0:
        return max(cols, 1)
    if cols > 1 and strides[1] != 1:
        raise ValueError("%s must have unit stride along rows" % name)
    if rows > 1 and strides[0] < cols:
        raise ValueError("%s has overlapping rows (row stride %d < row length %d); pass a "
                         "contiguous copy" % (name, strides[0], cols))
    return max(strides[0] if rows > 1 else cols, cols, 1)


def _mat(t, name, dt):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.dtype != getattr(torch, IN_TYPES[dt]):
        raise TypeError("%s must be %s for this dtype, got %s" % (name, IN_TYPES[dt], t.dtype))
    return t.data_ptr(), row_layout(tuple(t.shape), t.stride(), name)


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context under which the workspace, temporaries and outputs of a call
    are allocated: the caller's stream, so that PyTorch's caching allocator
    does not hand their memory to other work while the call's kernels, which
    run on that stream, still use it."""
    import contextlib
    torch = _torch()
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _workspace(nbytes, device):
    torch = _torch()
    if nbytes == SIZE_MAX or nbytes == 0:
        # SIZE_MAX: the arguments are invalid; the entry point itself then
        # rejects them (before any launch) with the precise status code
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def _new_out(shape, dt, device, out, name):
    torch = _torch()
    if out is None:
        return torch.empty(shape, dtype=getattr(torch, _out_type(dt)), device=device)
    if tuple(out.shape) != tuple(shape) or out.dtype != getattr(torch, _out_type(dt)):
        raise ValueError("%s must be %s %s" % (name, shape, _out_type(dt)))
    row_layout(tuple(out.shape), out.stride(), name)
    return out


def hs_gemm(A, B, dtype="f32", p=1, K=0, out=None, stream=None):
    """C = A . B on the hyper-systolic schedule (p, K)."""
    dt = _dt(dtype)
    a, lda = _mat(A, "A", dt)
    b, ldb = _mat(B, "B", dt)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    with _on(stream):
        C = _new_out((m, n), dt, A.device, out, "out")
        ws, nb = _workspace(hs_workspace_size(HS_OP_GEMM, m, n, k, dt, p, K), A.device)
        st = lib().hs_gemm(m, n, k, dt, hs_schedule(p, K), a, lda, b, ldb, C.data_ptr(),
                           row_layout((m, n), C.stride()), ws.data_ptr() if ws is not None else None, nb,
                           _stream(stream))
    _check(st, "hs_gemm")
    return C


def hs_gemm_noalloc(A, B, out, dtype="f32", p=1, K=0, stream=None):
    """C = A . B into ``out`` without any device allocation (the library's
    static scratch array is the workspace)."""
    dt = _dt(dtype)
    a, lda = _mat(A, "A", dt)
    b, ldb = _mat(B, "B", dt)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    C = _new_out((m, n), dt, A.device, out, "out")
    st = lib().hs_gemm_noalloc(m, n, k, dt, hs_schedule(p, K), a, lda, b, ldb, C.data_ptr(),
                               row_layout((m, n), C.stride()), _stream(stream))
    _check(st, "hs_gemm_noalloc")
    return C


def hs_gemm_tn(A, B, dtype="f32", p=1, K=0, out=None, stream=None):
    """C = A^T . B with A stored k x m."""
    dt = _dt(dtype)
    a, lda = _mat(A, "A", dt)
    b, ldb = _mat(B, "B", dt)
    k, m = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("contraction dimensions differ: %d vs %d" % (k, k2))
    with _on(stream):
        C = _new_out((m, n), dt, A.device, out, "out")
        ws, nb = _workspace(hs_workspace_size(HS_OP_GEMM_TN, m, n, k, dt, p, K), A.device)
        st = lib().hs_gemm_tn(m, n, k, dt, hs_schedule(p, K), a, lda, b, ldb, C.data_ptr(),
                              row_layout((m, n), C.stride()), ws.data_ptr() if ws is not None else None, nb,
                              _stream(stream))
    _check(st, "hs_gemm_tn")
    return C


def hs_gemv(A, x, dtype="f32", p=1, K=0, out=None, stream=None):
    """y = A . x."""
    torch = _torch()
    dt = _dt(dtype)
    a, lda = _mat(A, "A", dt)
    m, n = A.shape
    if x.dim() != 1 or x.shape[0] != n or x.dtype != A.dtype or x.device != A.device:
        raise ValueError("x must be a length-%d vector of A's dtype on A's device" % n)
    with _on(stream):
        x = x.contiguous()
        y = torch.empty(m, dtype=A.dtype, device=A.device) if out is None else out
        if y.shape != (m,) or y.dtype != A.dtype or (m and y.stride(0) != 1):
            raise ValueError("out must be a contiguous length-%d vector" % m)
        st = lib().hs_gemv(m, n, dt, hs_schedule(p, K), a, lda, x.data_ptr(), y.data_ptr(),
                           None, 0, _stream(stream))
    _check(st, "hs_gemv")
    return y


def hs_gemm_backward(A, B, G, dtype="f32", p=1, K=0, need_a=True, need_b=True, stream=None):
    """dA = G . B^T and dB = A^T . G (either may be skipped)."""
    torch = _torch()
    dt = _dt(dtype)
    a, lda = _mat(A, "A", dt)
    b, ldb = _mat(B, "B", dt)
    g, ldg = _mat(G, "G", dt)
    m, k = A.shape
    k2, n = B.shape
    if k != k2 or tuple(G.shape) != (m, n):
        raise ValueError("shape mismatch: A %s, B %s, G %s" % (tuple(A.shape), tuple(B.shape), tuple(G.shape)))
    ot = getattr(torch, _out_type(dt))
    with _on(stream):
        dA = torch.empty((m, k), dtype=ot, device=A.device) if need_a else None
        dB = torch.empty((k, n), dtype=ot, device=A.device) if need_b else None
        ws, nb = _workspace(hs_workspace_size(HS_OP_BACKWARD, m, n, k, dt, p, K), A.device)
        st = lib().hs_gemm_backward(m, n, k, dt, hs_schedule(p, K), a, lda, b, ldb, g, ldg,
                                    dA.data_ptr() if dA is not None else None, max(k, 1),
                                    dB.data_ptr() if dB is not None else None, max(n, 1),
                                    ws.data_ptr() if ws is not None else None, nb, _stream(stream))
    _check(st, "hs_gemm_backward")
    return dA, dB


def hs_nbody(bodies, eps2=0.0, dtype=None, p=1, K=0, out=None, stream=None):
    """(ax, ay, az, phi) of every body of ``bodies`` (n x 4: x, y, z, m), the
    all-pairs gravitational interaction on the two-array schedule (p, K).
    dtype: "f32" or "f64" (default: the tensor's)."""
    torch = _torch()
    if not isinstance(bodies, torch.Tensor) or bodies.device.type != "cuda":
        raise TypeError("bodies must be a GPU tensor")
    if bodies.dim() != 2 or bodies.shape[1] != 4:
        raise ValueError("bodies must be n x 4 (x, y, z, m)")
    if dtype is None:
        dtype = {torch.float32: "f32", torch.float64: "f64"}.get(bodies.dtype)
        if dtype is None:
            raise TypeError("bodies must be float32 or float64")
    dt = _dt(dtype)
    if bodies.dtype != getattr(torch, IN_TYPES[dt]) or dt not in (HS_F32, HS_F64):
        raise TypeError("bodies must be float32 (f32) or float64 (f64)")
    n = bodies.shape[0]
    with _on(stream):
        bodies = bodies.contiguous()
        o = torch.empty((n, 4), dtype=bodies.dtype, device=bodies.device) if out is None else out
        if tuple(o.shape) != (n, 4) or o.dtype != bodies.dtype or (n and not o.is_contiguous()):
            raise ValueError("out must be a contiguous n x 4 tensor of the bodies' dtype")
        ws, nb = _workspace(hs_workspace_size(HS_OP_NBODY, n, 0, 0, dt, p, K), bodies.device)
        st = lib().hs_nbody(n, dt, hs_schedule(p, K), bodies.data_ptr(), float(eps2), o.data_ptr(),
                            ws.data_ptr() if ws is not None else None, nb, _stream(stream))
    _check(st, "hs_nbody")
    return o
