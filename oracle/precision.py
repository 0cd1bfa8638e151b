"""Operand splitting and FP8 quantisation of the precision forms -- TEST
INFRASTRUCTURE (imported only by the tests).

The precision forms approximate the plain product (Sec. 3.1, Eq. PRODUCT)
by replacing each FP32 operand with pieces in a narrow format.  This module
states those pieces from their definitions, in numpy float64, with no code
shared with the HIP path:

* bf16(x): round to nearest, ties to even, to 8 significant bits.
* 3-piece split: a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16(a - a0 - a1).
* e4m3 (OCP FP8): 1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits;
  largest finite value 448, no infinities; round to nearest, ties to the
  even code, saturating at 448.  Found here by searching the table of all
  127 non-negative finite values, not by bit manipulation.
* Per 128 x 128 tile of an operand (rows x contraction index, aligned to
  the matrix origin): e = the largest integer with amax * 2^e <= 448 (0 for
  a tile of zeros), q0 = e4m3(a 2^e), and for the refined form e1 = the same
  exponent for the residuals a 2^e - q0, q1 = e4m3((a 2^e - q0) 2^e1).
  Dequantised: q0 2^-e, refined q0 2^-e + q1 2^-(e + e1).
* f16(x): IEEE binary16, round to nearest, ties to even: 11 significant
  bits, smallest normal 2^-14, subnormal spacing 2^-24, largest finite 65504.
* 2-piece FP16 split with a power-of-two scale per operand row (row = the
  non-contraction index): e = the largest integer with amax * 2^e < 2^15
  (15 for a row of zeros), x' = x 2^e, a0 = f16(x'), a1 = f16(x' - a0).
  The element stands for (a0 + a1) 2^-e; a product keeps a0 b0 + a0 b1 +
  a1 b0 and scales the sum by 2^-(e_row + e_col).

Pins: tests/test_oracle_precision.py (torch's own bfloat16 and float8_e4m3fn
conversions, the table's structure, tie cases, error bounds).
"""
import numpy as np

E4M3_MAX = 448.0
TILE = 128


def e4m3_table():
    """All non-negative finite e4m3 values, indexed by their code 0..126."""
    vals = []
    for code in range(127):                       # 127 = 0x7f is NaN
        e, m = code >> 3, code & 7
        vals.append(m * 2.0 ** -9 if e == 0 else (8 + m) * 2.0 ** (e - 10))
    return np.array(vals)


_TABLE = e4m3_table()


def e4m3_code(x):
    """Code (0..126, magnitude only) of the nearest e4m3 value to |x|, ties to
    the even code, saturating at 448."""
    ax = np.minimum(np.abs(np.asarray(x, np.float64)), E4M3_MAX)
    hi = np.clip(np.searchsorted(_TABLE, ax, side="left"), 0, 126)   # first value >= ax
    lo = np.maximum(hi - 1, 0)
    d_lo = ax - _TABLE[lo]
    d_hi = _TABLE[hi] - ax
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (hi % 2 == 0))
    return np.where(pick_hi, hi, lo)


def e4m3(x):
    """Round x to e4m3 (value, in float64)."""
    x = np.asarray(x, np.float64)
    return np.sign(x) * _TABLE[e4m3_code(x)]


def tile_exponent(amax):
    """Largest integer e with amax * 2^e <= 448; 0 when amax == 0."""
    if amax == 0.0:
        return 0
    e = int(np.floor(np.log2(E4M3_MAX / amax)))
    while amax * 2.0 ** (e + 1) <= E4M3_MAX:       # settle log2 rounding
        e += 1
    while amax * 2.0 ** e > E4M3_MAX:
        e -= 1
    return e


def fp8_dequantized(X, refine, row_axis=0):
    """The value each element of operand X stands for in the FP8 forms.

    X is the operand with its rows along ``row_axis`` and its contraction
    index along the other axis; tiles are 128 x 128 from the origin."""
    X = np.asarray(X, np.float64)
    Xr = X if row_axis == 0 else X.T
    out = np.zeros_like(Xr)
    R, Kd = Xr.shape
    for r0 in range(0, R, TILE):
        for k0 in range(0, Kd, TILE):
            t = Xr[r0:r0 + TILE, k0:k0 + TILE]
            e = tile_exponent(float(np.max(np.abs(t))) if t.size else 0.0)
            xs = t * 2.0 ** e                      # exact: a power of two
            q0 = e4m3(xs)
            v = q0 * 2.0 ** -e
            if refine:
                res = xs - q0                      # exact in float64
                e1 = tile_exponent(float(np.max(np.abs(res))))
                q1 = e4m3(res * 2.0 ** e1)
                v = v + q1 * 2.0 ** -(e + e1)
            out[r0:r0 + TILE, k0:k0 + TILE] = v
    return out if row_axis == 0 else out.T


def bf16(x):
    """Round to bfloat16 (8 significant bits), ties to even, as float64.

    Written from the definition: scale |x| so its leading bit sits at 2^7,
    round to an integer with ties to even (numpy's rint), scale back."""
    x = np.asarray(x, np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        E = np.where(ax > 0, np.floor(np.log2(np.where(ax > 0, ax, 1.0))), 0.0)
    # settle floor(log2) against rounding in log2
    E = np.where(ax >= 2.0 ** (E + 1), E + 1, E)
    E = np.where(ax < 2.0 ** E, E - 1, E)
    E = np.maximum(E, -126.0)                      # bf16 subnormals share FP32's floor
    q = np.rint(ax * 2.0 ** (7 - E)) * 2.0 ** (E - 7)
    return np.sign(x) * q


def split3(a):
    """a0 = bf16(a), a1 = bf16(a - a0), a2 = bf16(a - a0 - a1); a is FP32."""
    a = np.asarray(a, np.float32).astype(np.float64)
    a0 = bf16(a)
    r1 = a - a0
    a1 = bf16(r1)
    a2 = bf16(r1 - a1)
    return a0, a1, a2


def f16(x):
    """Round to IEEE binary16 (11 significant bits), ties to even, as float64.

    From the definition, as bf16 above: the leading bit of |x| scaled to 2^10,
    rounded to an integer with ties to even, scaled back; exponents below -14
    share the subnormal spacing 2^-24; results past the largest finite value
    65504 (from 65520 on, the rounding boundary) become infinite."""
    x = np.asarray(x, np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        E = np.where(ax > 0, np.floor(np.log2(np.where(ax > 0, ax, 1.0))), 0.0)
    E = np.where(ax >= 2.0 ** (E + 1), E + 1, E)
    E = np.where(ax < 2.0 ** E, E - 1, E)
    E = np.maximum(E, -14.0)
    q = np.rint(ax * 2.0 ** (10 - E)) * 2.0 ** (E - 10)
    q = np.where(q >= 65520.0, np.inf, q)
    return np.sign(x) * q


def row_exponent(amax):
    """Largest integer e with amax * 2^e < 2^15; 15 when amax == 0."""
    amax = float(amax)
    if amax == 0.0:
        return 15
    e = int(np.floor(15 - np.log2(amax)))
    while amax * 2.0 ** e >= 2.0 ** 15:            # settle log2 rounding
        e -= 1
    while amax * 2.0 ** (e + 1) < 2.0 ** 15:
        e += 1
    return e


def split2_f16(X, row_axis=0):
    """Pieces of the 2-piece FP16 split: (a0, a1, e) with a0, a1 in the
    scaled domain (float64 arrays shaped like X) and e the exponent of each
    row (rows along ``row_axis``, the contraction along the other axis)."""
    X = np.asarray(X, np.float32).astype(np.float64)
    Xr = X if row_axis == 0 else X.T
    e = np.array([row_exponent(np.max(np.abs(r)) if r.size else 0.0) for r in Xr], dtype=np.int64)
    xs = Xr * np.ldexp(1.0, e)[:, None]            # exact: a power of two
    a0 = f16(xs)
    a1 = f16(xs - a0)                              # the residual is exact in float64
    if row_axis != 0:
        a0, a1 = a0.T, a1.T
    return a0, a1, e


def split2_f16_value(X, row_axis=0):
    """The value each element of X stands for in the 2-piece FP16 form."""
    a0, a1, e = split2_f16(X, row_axis)
    scale = np.ldexp(1.0, -e)
    return (a0 + a1) * (scale[:, None] if row_axis == 0 else scale[None, :])
