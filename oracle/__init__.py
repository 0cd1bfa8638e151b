"""FP64 oracle for the hyper-systolic matrix product -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The product path (the HIP library and its Python
binding) never touches it, and the two share no code.

What it computes is the plain definition the method reaches exactly
(Sec. 3.1, Eq. PRODUCT): c_ij = sum_k a_ik b_kj in double precision, ascending
k, plus the transposed product, the matrix-vector product and the gradient of
L = sum(C * G), and the complex product (``complex_gemm``, by its real
and imaginary parts).  ``nbody`` is the all-pairs gravitational sum, the
prototype n^2-problem (Sec. 2.2) of the two-array recipe (Sec. 4.1).  See
``hs_oracle.c``.  ``ring`` holds a ring simulator of the systolic and
hyper-systolic products (Sec. 5), driven by the three bases and the circular
shift alone, and ``bases`` the regular hyper-systolic bases (Sec. 4.4,
Sec. 5.2.1); both pin the schedule.

Parity pins: see tests/test_oracle.py (identity, permutation, small-integer
exactness, explicit transpose, associativity, central differences, exactly
rounded brute force) and tests/test_oracle_nbody.py (a = -grad phi, momentum
conservation, the virial identity, the field of a Plummer sphere, symmetry).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        i64 = ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.hs_oracle_gemm.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.hs_oracle_gemm_tn.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
        lib.hs_oracle_gemv.argtypes = [i64, i64, dp, i64, dp, dp]
        lib.hs_oracle_backward.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64,
                                           dp, i64, dp, i64]
        lib.hs_oracle_gemm_rows.argtypes = [i64, i64, dp, i64, dp, i64, ip, i64, dp, i64]
        lib.hs_oracle_gemm_tn_rows.argtypes = [i64, i64, dp, i64, dp, i64, ip, i64, dp, i64]
        lib.hs_oracle_grad_a_rows.argtypes = [i64, i64, dp, i64, dp, i64, ip, i64, dp, i64]
        lib.hs_oracle_nbody.argtypes = [i64, dp, ctypes.c_double, dp, dp]
        lib.hs_oracle_nbody_rows.argtypes = [i64, dp, ctypes.c_double, ip, i64, dp, dp]
        lib.hs_oracle_set_threads.argtypes = [ctypes.c_int]
        lib.hs_oracle_set_threads.restype = None
        for f in ("hs_oracle_gemm", "hs_oracle_gemm_tn", "hs_oracle_gemv",
                  "hs_oracle_backward", "hs_oracle_gemm_rows", "hs_oracle_gemm_tn_rows",
                  "hs_oracle_grad_a_rows", "hs_oracle_nbody", "hs_oracle_nbody_rows"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def set_threads(n):
    """Threads of the oracle's loops (n <= 0: all); for timing only."""
    _load().hs_oracle_set_threads(int(n))


def _d(x):
    """Promote to a C-contiguous float64 array (the stored values, exactly)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gemm(A, B):
    """C = A . B  (A m x k, B k x n), Eq. PRODUCT."""
    A, B = _d(A), _d(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n), np.float64)
    _load().hs_oracle_gemm(m, n, k, _p(A), k, _p(B), n, _p(C), n)
    return C


def gemm_tn(A, B):
    """C = A^T . B with A stored k x m (transposed product of the abstract)."""
    A, B = _d(A), _d(B)
    k, m = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n), np.float64)
    _load().hs_oracle_gemm_tn(m, n, k, _p(A), m, _p(B), n, _p(C), n)
    return C


def gemv(A, x):
    """y = A . x (matrix-vector product of the abstract)."""
    A, x = _d(A), _d(x)
    m, n = A.shape
    assert x.shape == (n,)
    y = np.empty(m, np.float64)
    _load().hs_oracle_gemv(m, n, _p(A), n, _p(x), _p(y))
    return y


def backward(A, B, G, need_a=True, need_b=True):
    """Gradient of L = sum(C * G), C = A . B:  dA = G . B^T, dB = A^T . G."""
    A, B, G = _d(A), _d(B), _d(G)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2 and G.shape == (m, n)
    dA = np.empty((m, k), np.float64) if need_a else None
    dB = np.empty((k, n), np.float64) if need_b else None
    null = ctypes.POINTER(ctypes.c_double)()
    _load().hs_oracle_backward(m, n, k, _p(A), k, _p(B), n, _p(G), n,
                               _p(dA) if need_a else null, k,
                               _p(dB) if need_b else null, n)
    return dA, dB


def _rows(rows):
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    return r, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def gemm_rows(A, B, rows):
    """Rows ``rows`` of A . B (for sizes where the full product is too slow)."""
    A, B = _d(A), _d(B)
    m, k = A.shape
    n = B.shape[1]
    r, rp = _rows(rows)
    out = np.empty((len(r), n), np.float64)
    _load().hs_oracle_gemm_rows(n, k, _p(A), k, _p(B), n, rp, len(r), _p(out), n)
    return out


def gemm_tn_rows(A, B, rows):
    """Rows ``rows`` of A^T . B with A stored k x m."""
    A, B = _d(A), _d(B)
    k, m = A.shape
    n = B.shape[1]
    r, rp = _rows(rows)
    out = np.empty((len(r), n), np.float64)
    _load().hs_oracle_gemm_tn_rows(n, k, _p(A), m, _p(B), n, rp, len(r), _p(out), n)
    return out


def grad_a_rows(G, B, rows):
    """Rows ``rows`` of dA = G . B^T (G m x n, B k x n)."""
    G, B = _d(G), _d(B)
    m, n = G.shape
    k = B.shape[0]
    r, rp = _rows(rows)
    out = np.empty((len(r), k), np.float64)
    _load().hs_oracle_grad_a_rows(n, k, _p(G), n, _p(B), n, rp, len(r), _p(out), k)
    return out


def grad_b_rows(A, G, rows):
    """Rows ``rows`` of dB = A^T . G (A m x k, G m x n)."""
    return gemm_tn_rows(A, G, rows)


# ---------------------------------------------------------------------------
# complex data (the complex workload of Sec. 7): the same definition,
# c_ij = sum_k a_ik b_kj, in complex arithmetic, written with real products:
# re c = re a re b - im a im b, im c = re a im b + im a re b.
# ---------------------------------------------------------------------------
def complex_gemm(A, B):
    """C = A . B for complex A (m x k), B (k x n), in FP64 parts."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    Ar, Ai, Br, Bi = A.real, A.imag, B.real, B.imag
    return (gemm(Ar, Br) - gemm(Ai, Bi)) + 1j * (gemm(Ar, Bi) + gemm(Ai, Br))


def complex_gemv(A, x):
    """y = A . x for complex A (m x n) and x (n), in FP64 parts."""
    A = np.asarray(A, np.complex128)
    x = np.asarray(x, np.complex128)
    Ar, Ai, xr, xi = A.real, A.imag, x.real, x.imag
    return (gemv(Ar, xr) - gemv(Ai, xi)) + 1j * (gemv(Ar, xi) + gemv(Ai, xr))


def complex_gemm_rows(A, B, rows):
    """Rows ``rows`` of the complex product A . B."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    Ar, Ai, Br, Bi = A.real, A.imag, B.real, B.imag
    return ((gemm_rows(Ar, Br, rows) - gemm_rows(Ai, Bi, rows))
            + 1j * (gemm_rows(Ar, Bi, rows) + gemm_rows(Ai, Br, rows)))


# ---------------------------------------------------------------------------
# all-pairs n-body interaction (Sec. 2.2 prototype n^2-problem; Sec. 4.1)
# ---------------------------------------------------------------------------
def nbody(bodies, eps2, with_scale=False):
    """(ax, ay, az, phi) of every body; bodies is n x 4 (x, y, z, m).

    a_i = sum_{j != i} m_j d_ij / (|d_ij|^2 + eps2)^(3/2), d_ij = r_j - r_i;
    phi_i = -sum_{j != i} m_j / (|d_ij|^2 + eps2)^(1/2).  With ``with_scale``
    also returns sum_{j != i} |m_j d_ij| / (|d_ij|^2 + eps2)^(3/2)."""
    X = _d(bodies)
    n = X.shape[0]
    assert X.shape == (n, 4)
    out = np.empty((n, 4), np.float64)
    sc = np.empty(n, np.float64)
    _load().hs_oracle_nbody(n, _p(X), float(eps2), _p(out), _p(sc))
    return (out, sc) if with_scale else out


def nbody_rows(bodies, eps2, rows):
    """(out, scale) of ``nbody`` for the bodies ``rows`` only."""
    X = _d(bodies)
    n = X.shape[0]
    r, rp = _rows(rows)
    out = np.empty((len(r), 4), np.float64)
    sc = np.empty(len(r), np.float64)
    _load().hs_oracle_nbody_rows(n, _p(X), float(eps2), rp, len(r), _p(out), _p(sc))
    return out, sc


# ---------------------------------------------------------------------------
# sums of absolute products: the scale of the element-wise error bounds
# (every rounding-error bound of a dot product is a multiple of
# sum_k |a_ik| |b_kj|)
# ---------------------------------------------------------------------------
def absprod(A, B):
    """(|A| |B|)_ij = sum_k |a_ik| |b_kj| (A m x k, B k x n)."""
    return gemm(np.abs(_d(A)), np.abs(_d(B)))


def absprod_rows(A, B, rows):
    """Rows ``rows`` of |A| |B|."""
    return gemm_rows(np.abs(_d(A)), np.abs(_d(B)), rows)


def complex_absprod(A, B):
    """Sums of absolute real products of the complex product A . B, as
    re + 1j im: the real part of c_ij is sum_k (re a re b - im a im b), so
    its scale is sum_k (|re a||re b| + |im a||im b|); the imaginary part's
    is sum_k (|re a||im b| + |im a||re b|)."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    Ar, Ai, Br, Bi = np.abs(A.real), np.abs(A.imag), np.abs(B.real), np.abs(B.imag)
    return (gemm(Ar, Br) + gemm(Ai, Bi)) + 1j * (gemm(Ar, Bi) + gemm(Ai, Br))


def complex_absprod_rows(A, B, rows):
    """Rows ``rows`` of complex_absprod(A, B)."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    Ar, Ai, Br, Bi = np.abs(A.real), np.abs(A.imag), np.abs(B.real), np.abs(B.imag)
    return ((gemm_rows(Ar, Br, rows) + gemm_rows(Ai, Bi, rows))
            + 1j * (gemm_rows(Ar, Bi, rows) + gemm_rows(Ai, Br, rows)))


def sqprod(A, B):
    """sum_k a_ik^2 b_kj^2 (the squared 2-norm of the terms of each dot
    product; the scale of err_term)."""
    A, B = _d(A), _d(B)
    return gemm(A * A, B * B)


def complex_sqprod(A, B):
    """sum of squared real terms of each part of the complex product, as
    re + 1j im (terms as in complex_absprod)."""
    A = np.asarray(A, np.complex128)
    B = np.asarray(B, np.complex128)
    Ar, Ai, Br, Bi = A.real ** 2, A.imag ** 2, B.real ** 2, B.imag ** 2
    return (gemm(Ar, Br) + gemm(Ai, Bi)) + 1j * (gemm(Ar, Bi) + gemm(Ai, Br))
