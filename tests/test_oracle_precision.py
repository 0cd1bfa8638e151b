"""Pins of oracle.precision (CPU): the BF16 split and the e4m3 quantisation
that the precision forms are defined by, checked against torch's own
conversions, the format's structure and exact special cases."""
import numpy as np
import pytest
import torch

from oracle import precision as P


def test_e4m3_table_structure():
    t = P.e4m3_table()
    assert len(t) == 127 and t[0] == 0.0
    assert np.all(np.diff(t) > 0)                   # codes are ordered by value
    assert t[1] == 2.0 ** -9 and t[8] == 2.0 ** -6  # smallest subnormal, smallest normal
    assert t[-1] == 448.0 and t[-2] == 416.0
    for e in range(1, 16):                          # 8 values per binade
        assert t[e * 8] == 2.0 ** (e - 7)


def test_e4m3_matches_torch_float8_within_range():
    rng = np.random.default_rng(11)
    t = P.e4m3_table()
    mids = (t[:-1] + t[1:]) / 2                     # every tie between neighbours
    x = np.concatenate([rng.uniform(-448, 448, 50000), rng.uniform(-0.03, 0.03, 50000),
                        mids, -mids, t, -t])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).double().numpy()
    assert np.array_equal(P.e4m3(x), ref)


def test_e4m3_ties_to_even_and_saturation():
    assert P.e4m3(1.0625) == 1.0          # between 1 (code 56) and 1.125 (57)
    assert P.e4m3(1.1875) == 1.25         # between 1.125 (57) and 1.25 (58)
    assert P.e4m3(2.0 ** -10) == 0.0      # between 0 and 2^-9
    assert P.e4m3(3 * 2.0 ** -10) == 2 * 2.0 ** -9
    assert P.e4m3(1e6) == 448.0 and P.e4m3(-500.0) == -448.0


def test_tile_exponent_definition():
    rng = np.random.default_rng(12)
    for amax in np.concatenate([10.0 ** rng.uniform(-30, 30, 2000), [448.0, 224.0, 1.0, 2.0 ** -20]]):
        e = P.tile_exponent(float(amax))
        assert amax * 2.0 ** e <= 448.0 < amax * 2.0 ** (e + 1)
    assert P.tile_exponent(0.0) == 0
    assert P.tile_exponent(1.0) == 8 and P.tile_exponent(448.0) == 0


def test_fp8_dequantised_error_bounds():
    """|deq(a) - a| <= u |a| + half a subnormal step (plain, u = 2^-4), and
    <= u^2 |a| + u half-step + half a subnormal step of the residual scale
    (refined), per 128 x 128 tile with its own exponents."""
    rng = np.random.default_rng(13)
    X = rng.uniform(-1, 1, (256, 384)) * 10.0 ** rng.uniform(-3, 3, (256, 1))
    u, half_sub = 2.0 ** -4, 2.0 ** -10
    D0 = P.fp8_dequantized(X, False)
    D1 = P.fp8_dequantized(X, True)
    for r0 in range(0, 256, 128):
        for k0 in range(0, 384, 128):
            t = X[r0:r0 + 128, k0:k0 + 128]
            e = P.tile_exponent(float(np.max(np.abs(t))))
            e1 = P.tile_exponent(float(np.max(np.abs(t * 2.0 ** e - P.e4m3(t * 2.0 ** e)))))
            err0 = np.abs(D0[r0:r0 + 128, k0:k0 + 128] - t)
            err1 = np.abs(D1[r0:r0 + 128, k0:k0 + 128] - t)
            assert np.all(err0 <= u * np.abs(t) + half_sub * 2.0 ** -e)
            assert np.all(err1 <= u * u * np.abs(t) + u * half_sub * 2.0 ** -e + half_sub * 2.0 ** -(e + e1))
            assert np.mean(err1) < np.mean(err0) * 2.0 ** -3
    # powers of two times small integers are exact in both forms
    Z = rng.integers(-8, 9, (128, 128)).astype(np.float64) * 0.25
    assert np.array_equal(P.fp8_dequantized(Z, False), Z)
    assert np.array_equal(P.fp8_dequantized(Z, True), Z)


def test_bf16_matches_torch_bfloat16():
    rng = np.random.default_rng(14)
    y = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-30, 30, 100000)).astype(np.float32)
    # exact ties: 8 significant bits plus a half
    ties = ((rng.integers(128, 256, 2000) * 2 + 1) * 2.0 ** rng.integers(-40, 40, 2000)).astype(np.float32)
    for x in (y, ties, -ties):
        ref = torch.from_numpy(x).to(torch.bfloat16).double().numpy()
        assert np.array_equal(P.bf16(x.astype(np.float64)), ref)


def test_split3_reconstructs_exactly_in_normal_range():
    rng = np.random.default_rng(15)
    a = (rng.standard_normal(200000) * 10.0 ** rng.uniform(-20, 20, 200000)).astype(np.float32)
    a0, a1, a2 = P.split3(a)
    for q in (a0, a1, a2):                          # each piece is a bf16 value
        assert np.array_equal(P.bf16(q), q)
    assert np.array_equal(a0 + a1 + a2, a.astype(np.float64))
    nz = a1 != 0
    assert np.all(np.abs(a1[nz]) <= np.abs(a0[nz]) * 2.0 ** -8)


def test_f16_matches_numpy_and_torch_float16():
    rng = np.random.default_rng(16)
    y = (rng.standard_normal(100000) * 2.0 ** rng.uniform(-30, 17, 100000)).astype(np.float32)
    # exact ties of 11 significant bits, normal and subnormal
    ties = ((rng.integers(1024, 2048, 2000) * 2 + 1) * 2.0 ** rng.integers(-25, 5, 2000))
    sub = (rng.integers(0, 2048, 2000) * 2 + 1) * 2.0 ** -25
    for x in (y.astype(np.float64), ties, -ties, sub):
        with np.errstate(over="ignore"):            # past 65520: infinity on both sides
            ref = x.astype(np.float16).astype(np.float64)
        assert np.array_equal(P.f16(x), ref)
        assert np.array_equal(P.f16(x), torch.from_numpy(x).to(torch.float16).double().numpy())
    assert P.f16(65519.0) == 65504.0 and P.f16(65520.0) == np.inf and P.f16(2.0 ** -25) == 0.0
    assert P.f16(3 * 2.0 ** -26) == 2.0 ** -24


def test_row_exponent_definition():
    rng = np.random.default_rng(17)
    for amax in np.concatenate([2.0 ** rng.uniform(-140, 120, 2000), [1.0, 2.0 ** 15, 3.0, 2.0 ** -149]]):
        e = P.row_exponent(amax)
        assert 2.0 ** 14 <= amax * 2.0 ** e < 2.0 ** 15, amax
    assert P.row_exponent(0.0) == 15
    assert P.row_exponent(1.0) == 14 and P.row_exponent(1.5) == 14 and P.row_exponent(0.5) == 15


def test_split2_f16_hand_value():
    # float32(1/3) = 11184811 * 2^-25, row max 1/3: e = 16 (2^16/3 lies in
    # [2^14, 2^15)), x' = 11184811 / 512 = 21845.333984375; binary16 spacing
    # at 2^14 is 16: a0 = 21840; the residual 2731/512 = 5.333984375 has
    # spacing 2^-8 and sits exactly halfway between 1365 and 1366 units: the
    # tie goes to the even one, a1 = 1366/256
    a0, a1, e = P.split2_f16(np.array([[np.float32(1.0 / 3.0)]]))
    assert e.tolist() == [16]
    assert a0[0, 0] == 21840.0 and a1[0, 0] == 1366.0 / 256.0
    v = P.split2_f16_value(np.array([[np.float32(1.0 / 3.0)]]))
    assert v[0, 0] == (21840.0 + 1366.0 / 256.0) * 2.0 ** -16


def test_split2_f16_error_bound_and_structure():
    rng = np.random.default_rng(18)
    X = (rng.standard_normal((64, 300)) * 10.0 ** rng.uniform(-30, 30, (64, 1))).astype(np.float32)
    X[3, :] = 0.0
    X[5, 7] = 0.0
    for axis in (0, 1):
        Y = X if axis == 0 else X.T
        a0, a1, e = P.split2_f16(Y, row_axis=axis)
        xs = X * np.ldexp(1.0, e)[:, None]
        A0 = a0 if axis == 0 else a0.T
        A1 = a1 if axis == 0 else a1.T
        for q in (A0, A1):                          # each piece is a binary16 value
            assert np.array_equal(P.f16(q), q)
        amax = np.max(np.abs(xs), axis=1)
        nz = amax > 0
        assert np.all((amax[nz] >= 2.0 ** 14) & (amax[nz] < 2.0 ** 15))
        # |x' - a0 - a1| <= 2^-22 |x'| + 2^-25 (the last term: subnormal a1)
        err = np.abs(xs - A0 - A1)
        assert np.all(err <= 2.0 ** -22 * np.abs(xs) + 2.0 ** -25)
        assert np.all(np.abs(xs - A0) <= 2.0 ** -11 * np.abs(xs) + 2.0 ** -25)
        val = P.split2_f16_value(Y, row_axis=axis)
        V = val if axis == 0 else val.T
        assert np.all(np.abs(V - X) <= (2.0 ** -22 * np.abs(xs) + 2.0 ** -25) * np.ldexp(1.0, -e)[:, None])
    # small integers and powers of two are exact
    Z = rng.integers(-8, 9, (32, 40)).astype(np.float32) * np.float32(2.0 ** -3)
    assert np.array_equal(P.split2_f16_value(Z), Z.astype(np.float64))
    assert np.array_equal(P.split2_f16_value(Z, row_axis=1), Z.astype(np.float64))
