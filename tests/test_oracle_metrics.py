"""Pins for the oracle's error metrics and absolute-product sums (CPU only).

Every parity gate goes through these functions, so they are pinned by values
worked out by hand below (not by retyping their formulas), and by planted
mistakes: each plausible wrong version of a metric is written out here and
must disagree with the hand-computed value on the same fixture.
"""
import numpy as np
import pytest

import oracle
from oracle.metrics import err_elem, err_row, err_term

# ---------------------------------------------------------------------------
# fixtures, with the values worked out by hand
# ---------------------------------------------------------------------------
# three rows of different scale; row 0 errs in one element, row 1 not at all,
# row 2 in both:
#   row 0: error (0, 0.5),      |ref| = 5,  err = 0.1
#   row 1: error (0, 0),        |ref| = 10, err = 0
#   row 2: error (0.12, 0.16),  |ref| = 1,  err = 0.2   <- the maximum
REF = np.array([[3.0, 4.0], [6.0, 8.0], [0.6, 0.8]])
GOT = np.array([[3.0, 4.5], [6.0, 8.0], [0.72, 0.96]])
ERR_ROW = 0.2
# err_term: errors |GOT3 - REF3| = [[0, 0.5], [0.3, 0]] over sqrt(k SQP) with
# k = 4, SQP = [[4, 1], [9, 16]], i.e. over [[4, 2], [6, 8]]:
# [[0, 0.25], [0.05, 0]] -> 0.25
REF3 = np.array([[1.0, 2.5], [3.0, 4.0]])
GOT3 = np.array([[1.0, 3.0], [3.3, 4.0]])
SQP, K3 = np.array([[4.0, 1.0], [9.0, 16.0]]), 4
ERR_TERM = 0.25

# element errors |GOT2 - REF2| = [[0.5, 0], [0, 0.25]] over ABSP = [[4, 4], [5, 1]]
# -> [[0.125, 0], [0, 0.25]]: err_elem = 0.25
REF2 = np.array([[1.0, -2.0], [3.0, 0.5]])
GOT2 = np.array([[1.5, -2.0], [3.0, 0.25]])
ABSP = np.array([[4.0, 4.0], [5.0, 1.0]])
ERR_ELEM = 0.25

# |A| |B| by hand: A = [[1, -2], [3, 4]], B = [[-1, 2], [0.5, -3]]
#   (0,0) 1*1 + 2*0.5 = 2    (0,1) 1*2 + 2*3 = 8
#   (1,0) 3*1 + 4*0.5 = 5    (1,1) 3*2 + 4*3 = 18
ABS_A = np.array([[1.0, -2.0], [3.0, 4.0]])
ABS_B = np.array([[-1.0, 2.0], [0.5, -3.0]])
ABSPROD = np.array([[2.0, 8.0], [5.0, 18.0]])
# sum_k a^2 b^2 by hand: A^2 = [[1, 4], [9, 16]], B^2 = [[1, 4], [0.25, 9]]
#   (0,0) 1 + 4*0.25 = 2   (0,1) 4 + 4*9 = 40   (1,0) 9 + 16*0.25 = 13   (1,1) 36 + 144 = 180
SQPROD = np.array([[2.0, 40.0], [13.0, 180.0]])


def test_err_row_hand_value():
    assert err_row(GOT, REF) == pytest.approx(ERR_ROW, rel=1e-12)
    assert err_row(REF, REF) == 0.0
    # one row given as a vector
    assert err_row(GOT[2], REF[2]) == pytest.approx(0.2, rel=1e-12)
    # an all-zero reference row is measured in absolute terms
    assert err_row(np.array([[3.0, 4.0]]), np.zeros((1, 2))) == pytest.approx(5.0)
    # the imaginary part counts: error (0, 1i) against |ref| = 2
    assert err_row(np.array([[2.0 + 1j]]), np.array([[2.0]])) == pytest.approx(0.5)
    assert err_row(np.zeros((0, 3)), np.zeros((0, 3))) == 0.0


def test_err_term_hand_value():
    assert err_term(GOT3, REF3, SQP, K3) == pytest.approx(ERR_TERM, rel=1e-12)
    assert err_term(REF3, REF3, SQP, K3) == 0.0
    # a lone wrong element of a wide row is seen at its own scale: a row
    # gate dilutes it by sqrt(n)
    n, k = 1024, 64
    ref = np.ones((1, n))
    sq = np.full((1, n), 1.0 / k)          # k terms of size 1/k summing to 1
    got = ref.copy()
    got[0, 17] += 1e-3
    assert err_term(got, ref, sq, k) == pytest.approx(1e-3, rel=1e-9)
    assert err_row(got, ref) == pytest.approx(1e-3 / np.sqrt(n), rel=1e-9)
    # complex: parts against their own scales (re 0.5 / sqrt(1 * 4), im 0.3 / sqrt(1 * 1))
    assert err_term(np.array([[1.5 + 0.3j]]), np.array([[1.0 + 0j]]), np.array([[4.0 + 1.0j]]), 1) == \
        pytest.approx(0.3, rel=1e-12)


def test_err_elem_hand_value():
    assert err_elem(GOT2, REF2, ABSP) == pytest.approx(ERR_ELEM, rel=1e-12)
    assert err_elem(REF2, REF2, ABSP) == 0.0
    # a zero absprod element is measured in absolute terms
    assert err_elem(np.array([[0.5]]), np.array([[0.0]]), np.array([[0.0]])) == 0.5


def test_err_elem_complex_parts_separately():
    # re error 0.5 against re scale 2 (0.25), im error 0.3 against im scale
    # 0.5 (0.6): the maximum is the imaginary part's
    got = np.array([[1.5 + 0.3j]])
    ref = np.array([[1.0 + 0.0j]])
    ap = np.array([[2.0 + 0.5j]])
    assert err_elem(got, ref, ap) == pytest.approx(0.6, rel=1e-12)


def test_absprod_hand_value():
    got = oracle.absprod(ABS_A, ABS_B)
    assert np.array_equal(got, ABSPROD)
    assert np.array_equal(oracle.absprod_rows(ABS_A, ABS_B, [1]), ABSPROD[1:2])
    # the bound it scales: |A B| <= |A| |B| element by element
    C = oracle.gemm(ABS_A, ABS_B)
    assert (np.abs(C) <= got).all() and not np.array_equal(np.abs(C), got)


def test_sqprod_hand_value():
    got = oracle.sqprod(ABS_A, ABS_B)
    assert np.array_equal(got, SQPROD)
    # Cauchy-Schwarz and its converse: |A||B|^2 / k <= sum a^2 b^2 <= |A||B|^2
    k = ABS_A.shape[1]
    assert (ABSPROD ** 2 / k <= got).all() and (got <= ABSPROD ** 2).all()
    # planted mistakes: the square of the product, the product of squares
    # of one operand only
    assert not np.array_equal(oracle.gemm(ABS_A, ABS_B) ** 2, SQPROD)
    assert not np.array_equal(oracle.gemm(ABS_A * ABS_A, np.abs(ABS_B)), SQPROD)


def test_complex_absprod_hand_value():
    # a = 1 - 2i, b = 3 + 0.5i:
    #   re c = 3 + 1 = 4, its scale |1||3| + |-2||0.5| = 4
    #   im c = 0.5 - 6 = -5.5, its scale |1||0.5| + |-2||3| = 6.5
    A = np.array([[1.0 - 2.0j]])
    B = np.array([[3.0 + 0.5j]])
    assert np.array_equal(oracle.complex_gemm(A, B), np.array([[4.0 - 5.5j]]))
    assert np.array_equal(oracle.complex_absprod(A, B), np.array([[4.0 + 6.5j]]))
    assert np.array_equal(oracle.complex_absprod_rows(A, B, [0]), np.array([[4.0 + 6.5j]]))
    # squared terms: re 3^2 + (-2 * 0.5)^2 = 10, im 0.5^2 + (-2 * 3)^2 = 36.25
    assert np.array_equal(oracle.complex_sqprod(A, B), np.array([[10.0 + 36.25j]]))


# ---------------------------------------------------------------------------
# planted mistakes: each must disagree with the hand-computed value
# ---------------------------------------------------------------------------
def _row_mean(C, ref):            # mean instead of max over rows
    return float(np.mean(np.linalg.norm(C - ref, axis=1) / np.linalg.norm(ref, axis=1)))


def _row_by_got(C, ref):          # ||C_r|| instead of ||Chat_r|| as denominator
    return float(np.max(np.linalg.norm(C - ref, axis=1) / np.linalg.norm(C, axis=1)))


def _row_axis_swapped(C, ref):    # norms over columns instead of rows
    return float(np.max(np.linalg.norm(C - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def _row_maxabs(C, ref):          # max-abs instead of 2-norm in the numerator
    return float(np.max(np.abs(C - ref).max(axis=1) / np.linalg.norm(ref, axis=1)))


def _row_squared(C, ref):         # squared norms
    return float(np.max((np.linalg.norm(C - ref, axis=1) / np.linalg.norm(ref, axis=1)) ** 2))


@pytest.mark.parametrize("mutant", [_row_mean, _row_by_got, _row_axis_swapped, _row_maxabs, _row_squared])
def test_err_row_mutants_caught(mutant):
    assert abs(mutant(GOT, REF) - ERR_ROW) > 1e-3


def _term_no_sqrt(C, ref, sq, k):    # k sum a^2 b^2 without the square root
    return float(np.max(np.abs(C - ref) / (k * sq)))


def _term_no_k(C, ref, sq, k):       # the terms' 2-norm without sqrt(k)
    return float(np.max(np.abs(C - ref) / np.sqrt(sq)))


def _term_by_ref(C, ref, sq, k):     # |Chat| as the scale
    return float(np.max(np.abs(C - ref) / np.abs(ref)))


def _term_mean(C, ref, sq, k):       # mean instead of max
    return float(np.mean(np.abs(C - ref) / np.sqrt(k * sq)))


@pytest.mark.parametrize("mutant", [_term_no_sqrt, _term_no_k, _term_by_ref, _term_mean])
def test_err_term_mutants_caught(mutant):
    assert abs(mutant(GOT3, REF3, SQP, K3) - ERR_TERM) > 1e-3


def _elem_mean(C, ref, ap):       # mean instead of max
    return float(np.mean(np.abs(C - ref) / ap))


def _elem_signed(C, ref, ap):     # missing abs of the difference
    return float(np.max((C - ref) / ap))


def _elem_by_ref(C, ref, ap):     # |Chat| instead of |A||B| as the scale
    den = np.where(ref == 0, 1.0, np.abs(ref))
    return float(np.max(np.abs(C - ref) / den))


@pytest.mark.parametrize("mutant", [_elem_mean, _elem_signed, _elem_by_ref])
def test_err_elem_mutants_caught(mutant):
    assert abs(mutant(GOT2, REF2, ABSP) - ERR_ELEM) > 1e-3


def test_absprod_mutant_missing_abs_caught():
    # |A B| (abs taken after the product) or A B itself are not |A| |B|
    assert not np.array_equal(np.abs(oracle.gemm(ABS_A, ABS_B)), ABSPROD)
    assert not np.array_equal(oracle.gemm(ABS_A, ABS_B), ABSPROD)
    # |A| B (one abs dropped)
    assert not np.array_equal(oracle.gemm(np.abs(ABS_A), ABS_B), ABSPROD)


# ---------------------------------------------------------------------------
# the element-wise bound of the parity gates, on the oracle's own rounding
# ---------------------------------------------------------------------------
def test_elem_bound_holds_for_float32_accumulation():
    """A sequential FP32 dot product (round to nearest) stays within
    k u sum|a||b| (u = 2^-24) of the FP64 oracle, far inside the
    3 k u of the FP32 gate; a wrong contraction block does not."""
    g = np.random.default_rng(5)
    m, k, n = 6, 300, 5
    A = g.standard_normal((m, k)).astype(np.float32)
    B = g.standard_normal((k, n)).astype(np.float32)
    acc = np.zeros((m, n), np.float32)
    for t in range(k):
        acc = (acc + np.outer(A[:, t], B[t, :]).astype(np.float32)).astype(np.float32)
    ref = oracle.gemm(A, B)
    ap = oracle.absprod(A, B)
    u = 2.0 ** -24
    assert err_elem(acc, ref, ap) <= k * u
    # a missing block of 10 contraction terms is far outside 3 k u
    bad = acc - (A[:, :10].astype(np.float64) @ B[:10, :].astype(np.float64))
    assert err_elem(bad, ref, ap) > 3 * k * u
