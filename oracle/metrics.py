"""Error metrics against the FP64 oracle (test infrastructure).

err_row  = max_r ||C_r - Chat_r||_2 / ||Chat_r||_2
           (relative error per output row; insensitive to per-row scales)
err_elem = max_ij |C_ij - Chat_ij| / (|A| |B|)_ij
           (error relative to the sum of absolute products, the natural
           scale of a rounding error in a dot product)
"""
import numpy as np


def _promote(C, ref):
    """float64, or complex128 when either side is complex (the imaginary
    parts must count)."""
    dt = np.complex128 if (np.iscomplexobj(C) or np.iscomplexobj(ref)) else np.float64
    return np.asarray(C, dt), np.asarray(ref, dt)


def err_row(C, ref):
    C, ref = _promote(C, ref)
    if C.ndim == 1:
        C, ref = C[None, :], ref[None, :]
    num = np.linalg.norm(C - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den)) if C.size else 0.0


def err_elem(C, ref, absprod):
    C, ref = _promote(C, ref)
    den = np.where(absprod == 0, 1.0, absprod)
    return float(np.max(np.abs(C - ref) / den)) if C.size else 0.0
