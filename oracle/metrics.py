"""Error metrics against the FP64 oracle (test infrastructure).

err_row  = max_r ||C_r - Chat_r||_2 / ||Chat_r||_2
           (relative error per output row; insensitive to per-row scales)
err_term = max_ij |C_ij - Chat_ij| / sqrt(k sum_t a_it^2 b_tj^2)
           (each element's error over the statistical scale of the rounding
           errors of its k-term dot product: the sum of the rounding errors
           of the partial sums S_t behaves like u sqrt(sum_t S_t^2), and
           sum_t S_t^2 is of the order of k sum_t (a_it b_tj)^2; unlike a
           per-row norm, it sees a lone wrong element at its own scale.
           sqprod holds sum_t a_it^2 b_tj^2; complex results as for err_elem)
err_elem = max_ij |C_ij - Chat_ij| / (|A| |B|)_ij
           (error relative to the sum of absolute products, the scale of
           every rounding-error bound of a dot product; for complex results
           the real and imaginary parts are taken separately, each against
           its own sum of absolute products, given as absprod.real and
           absprod.imag)

A row whose reference is all zeros is measured in absolute terms (its
denominator is taken as 1), and so is an element whose absprod or sqprod
is zero.
"""
import numpy as np


def _promote(C, ref):
    """float64, or complex128 when either side is complex (the imaginary
    parts must count)."""
    dt = np.complex128 if (np.iscomplexobj(C) or np.iscomplexobj(ref)) else np.float64
    return np.asarray(C, dt), np.asarray(ref, dt)


def _rows(C, ref):
    C, ref = _promote(C, ref)
    if C.ndim == 1:
        C, ref = C[None, :], ref[None, :]
    return C, ref


def err_row(C, ref):
    C, ref = _rows(C, ref)
    num = np.linalg.norm(C - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den)) if C.size else 0.0


def err_term(C, ref, sqprod, k):
    C, ref = _promote(C, ref)
    if not C.size:
        return 0.0
    if np.iscomplexobj(C):
        sq = np.asarray(sqprod, np.complex128)
        return max(err_term(C.real, ref.real, sq.real, k), err_term(C.imag, ref.imag, sq.imag, k))
    den = np.sqrt(max(int(k), 1) * np.asarray(sqprod, np.float64))
    den = np.where(den == 0, 1.0, den)
    return float(np.max(np.abs(C - ref) / den))


def err_elem(C, ref, absprod):
    C, ref = _promote(C, ref)
    if not C.size:
        return 0.0
    if np.iscomplexobj(C):
        ap = np.asarray(absprod, np.complex128)
        return max(err_elem(C.real, ref.real, ap.real), err_elem(C.imag, ref.imag, ap.imag))
    ap = np.asarray(absprod, np.float64)
    den = np.where(ap == 0, 1.0, ap)
    return float(np.max(np.abs(C - ref) / den))
