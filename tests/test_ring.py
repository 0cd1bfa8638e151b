"""Pins for the ring simulator and the hyper-systolic bases (CPU only).

The simulator runs the systolic and hyper-systolic products (Sec. 5) on a
ring of cells with the shift of Eq. CSHIFT1, driven by the bases of
Sec. 5.2.1.  These tests check it against
the definition of the product (exactly, on small integers and symbolically),
against the counting theorems, and against the facts the text states for the
p = 4, K = 2 worked example (Sec. 3.2.3 and 3.3.3; the figures are missing).
They also show that the alternative readings of the garbled passages fail.
"""
import json
import os

import numpy as np
import pytest

from oracle import bases, ring
from paper_cs_9809105_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _int_obj(shape, seed):
    return inputs.small_int(shape, seed).astype(np.int64).astype(object)


def _divisors(p):
    return [K for K in range(1, p + 1) if p % K == 0]


@pytest.mark.parametrize("p", range(1, 13))
def test_systolic_exact(p):
    A, B = _int_obj((p, p), 100 + p), _int_obj((p, p), 200 + p)
    C, shifts = ring.systolic(A, B, 0)
    assert (C == A.dot(B)).all()
    assert shifts == p          # the p-th shift only restores A


@pytest.mark.parametrize("p", range(1, 17))
def test_hyper_systolic_exact_all_K(p):
    A, B = _int_obj((p, p), 300 + p), _int_obj((p, p), 400 + p)
    for K in _divisors(p):
        C, shifts = ring.hyper_systolic(A, B, K, 0)
        assert (C == A.dot(B)).all(), (p, K)
        # Thm. GAIN3 / Eq. COMPL: one B pre-shift, K~-1 A-shifts, K-1 back-shifts
        assert shifts == bases.shifts_matrix_product(K, p // K)


@pytest.mark.parametrize("p", [1, 2, 4, 6, 8, 9])
def test_hyper_systolic_each_product_exactly_once(p):
    """Symbolic run: every a_ik b_kj reaches c_ij exactly once, nothing else does."""
    A, B = ring.leaves("A", p), ring.leaves("B", p)
    expect = ring.expected_terms(p)
    for K in _divisors(p):
        C, _ = ring.hyper_systolic(A, B, K, ring.Term())
        for i in range(p):
            for j in range(p):
                assert C[i, j] == expect[i, j], (p, K, i, j)


@pytest.mark.parametrize("p,K,bm,bk,bn", [(4, 2, 3, 2, 5), (6, 3, 2, 3, 1), (6, 2, 1, 4, 2),
                                          (8, 4, 2, 2, 3), (9, 3, 2, 1, 2)])
def test_block_mapping_rectangular_blocks(p, K, bm, bk, bn):
    """Sec. 6.1: a p x p system of sub-matrices is handled like scalars."""
    A = inputs.small_int((p * bm, p * bk), 500 + p).astype(np.int64)
    B = inputs.small_int((p * bk, p * bn), 600 + p).astype(np.int64)
    Ab = np.empty((p, p), dtype=object)
    Bb = np.empty((p, p), dtype=object)
    for i in range(p):
        for j in range(p):
            Ab[i, j] = A[i * bm:(i + 1) * bm, j * bk:(j + 1) * bk]
            Bb[i, j] = B[i * bk:(i + 1) * bk, j * bn:(j + 1) * bn]

    class Blk:                       # block with @ as the elementary product
        def __init__(self, x):
            self.x = x

        def __mul__(self, o):
            return Blk(self.x @ o.x)

        def __add__(self, o):
            return Blk(self.x + o.x)

    wrap = np.vectorize(Blk, otypes=[object])
    Cb, _ = ring.hyper_systolic(wrap(Ab), wrap(Bb), K, Blk(np.zeros((bm, bn), np.int64)))
    C = np.block([[Cb[i, j].x for j in range(p)] for i in range(p)])
    assert np.array_equal(C, A @ B)


def test_worked_example_p4_k2():
    """Facts stated in the text for p = 4, K = 2 (golden fixture, cited there)."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example_p4_k2.json")))
    p, K = g["p"], g["K"]
    # pre-shift strides of storage rows j = 1..p (0-based q = j - 1)
    strides = [ring.preshift_stride(j - 1, K) for j in range(1, p + 1)]
    moved = [j for j, s in zip(range(1, p + 1), strides) if abs(s) == 1]
    still = [j for j, s in zip(range(1, p + 1), strides) if s == 0]
    assert moved == g["preshift_rows_moved_by_one_1based"]
    assert still == g["preshift_rows_not_moved_1based"]

    # record the whole-array shifts made after the pre-shift
    calls = []
    orig = ring.cshift_row

    def spy(x, k, counter=None):
        calls.append(k)
        return orig(x, k, counter)

    ring.cshift_row = spy
    try:
        A, B = _int_obj((p, p), 7), _int_obj((p, p), 8)
        C, _ = ring.hyper_systolic(A, B, K, 0)
    finally:
        ring.cshift_row = orig
    assert (C == A.dot(B)).all()
    a_shifts = calls[:p // K - 1]
    c_shifts = calls[p // K - 1:]
    assert a_shifts == [g["a_shift_stride"]] * g["a_shift_count"]
    assert c_shifts == [g["c2_backshift_stride"]] * g["c2_backshift_count"]
    # stride +1 means cell i receives cell i+1: a shift to the left
    x = np.array([[0, 1, 2, 3]], dtype=object)
    assert list(orig(x, 1)[0]) == [1, 2, 3, 0]


def test_floored_mod_reading_fails():
    """Reading the pre-shift with a floored mod breaks the product for 1 < K < p."""
    orig = ring.preshift_stride
    ring.preshift_stride = lambda q, K: (-q) % K      # [(1 - j) mod K], floored
    try:
        failures = 0
        for p in (4, 6, 8, 9):
            A, B = _int_obj((p, p), 900 + p), _int_obj((p, p), 901 + p)
            for K in _divisors(p):
                if 1 < K < p:
                    C, _ = ring.hyper_systolic(A, B, K, 0)
                    failures += int(not (C == A.dot(B)).all())
        assert failures == sum(1 for p in (4, 6, 8, 9) for K in _divisors(p) if 1 < K < p)
    finally:
        ring.preshift_stride = orig


def test_stride_Ktilde_reading_fails_when_K_differs():
    """Sec. 3.3.3 says 'shift by K~ every K-th step'; the listing shifts by K.

    Replacing the A-stride K by K~ breaks the product whenever K != K~."""
    orig = ring.cshift_row
    for p, K in [(6, 2), (6, 3), (8, 2), (8, 4)]:
        Kt = p // K

        def swap(x, k, counter=None, K=K, Kt=Kt):
            return orig(x, Kt if k == K and x.shape[0] == p and k != 1 else k, counter)

        ring.cshift_row = swap
        try:
            A, B = _int_obj((p, p), 31), _int_obj((p, p), 32)
            C, _ = ring.hyper_systolic(A, B, K, 0)
        finally:
            ring.cshift_row = orig
        assert not (C == A.dot(B)).all(), (p, K)


@pytest.mark.parametrize("n", range(1, 65))
def test_regular_bases_complete(n):
    """Thm. (h-range of a regular base is n), checked by brute force."""
    for K in _divisors(n):
        Ab, Bb = bases.regular_bases_two_array(n, K)
        assert len(Ab) - 1 == K - 1 and len(Bb) - 1 == n // K - 1
        assert bases.h_range_complete(Ab, Bb, n)


def test_incomplete_bases_detected():
    """Dropping one element of a regular base leaves some offset unreachable."""
    for n, K in [(16, 4), (12, 3), (64, 8)]:
        Ab, Bb = bases.regular_bases_two_array(n, K)
        assert not bases.h_range_complete(Ab[:-1], Bb, n)
        assert not bases.h_range_complete(Ab, Bb[:-1], n)


def test_min_length_at_sqrt():
    """Thm. (minimal length): K + n/K - 1 is minimal at K = sqrt(n)."""
    for r in range(1, 12):
        n = r * r
        best = min(_divisors(n), key=lambda K: (K + n // K - 1, K))
        assert best == r


def _shortest_complete(n, complete, max_len):
    """Smallest k + k' over all base pairs with strides 1..n-1 that
    ``complete`` accepts (None if none up to max_len)."""
    import itertools
    for L in range(0, max_len + 1):
        for k in range(L + 1):
            for sa in itertools.product(range(1, n), repeat=k):
                for sb in itertools.product(range(1, n), repeat=L - k):
                    if complete([0] + list(sa), [0] + list(sb), n):
                        return L
    return None


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 9, 10, 12])
def test_two_array_minimum_length_brute_force(n):
    """Thm. MINIMUM2 by exhaustive search: over every pair of bases with
    strides 1..n-1, the shortest pair the recipe makes complete has k + k'
    equal to the best regular pair's (K - 1) + (n/K - 1), and at least the
    bound 2 (sqrt(n) - 1) ((k + 1)(k' + 1) offsets must cover n)."""
    best_regular = min((K - 1) + (n // K - 1) for K in _divisors(n))
    for K in _divisors(n):
        assert bases.recipe_complete(*bases.regular_bases_two_array(n, K), n)
    shortest = _shortest_complete(n, bases.recipe_complete, best_regular)
    assert shortest is not None and shortest >= 2 * (n ** 0.5 - 1) - 1e-12
    # the regular pairs are shortest except where a non-divisor split of n
    # into (k + 1)(k' + 1) >= n offsets is shorter (n = 5, 10: prime factors)
    assert shortest == min(k + kp for k in range(n) for kp in range(n) if (k + 1) * (kp + 1) >= n)


def test_literal_definition_admits_pairs_the_recipe_cannot_realise():
    """Def. DEF:OPTI2 read literally (any contiguous runs of both bases)
    accepts A = (0, 1), B = (0, 2, 4) for n = 8: k + k' = 3, below the bound
    2 (sqrt(8) - 1) = 3.66 of Thm. MINIMUM2.  The recipe meets only the
    offsets P_B(j) - P_A(t) mod 8 with P_A = {0, 1}, P_B = {0, 2, 6}, i.e.
    {0, 1, 2, 5, 6, 7}, never 3 or 4, so it is not complete; read as the
    recipe runs, the bound holds."""
    A, Bb = [0, 1], [0, 2, 4]
    assert bases.h_range_complete(A, Bb, 8)
    assert not bases.recipe_complete(A, Bb, 8)
    assert _shortest_complete(8, bases.h_range_complete, 4) == 3 < 2 * (8 ** 0.5 - 1)
    assert _shortest_complete(8, bases.recipe_complete, 4) == 4


def test_gain_factors():
    """Thm. GAIN3: R = (p-1)/(K+K~-1) ~ sqrt(p)/2;  Thm. GAIN2: T = 2K+K~-3."""
    for p in (16, 64, 256, 1024):
        K = int(round(p ** 0.5))
        T = bases.shifts_matrix_product(K, p // K)
        assert T == 2 * K - 1
        R = (p - 1) / T
        assert abs(R / (p ** 0.5 / 2) - 1) < 0.2
    assert bases.shifts_two_array(4, 4) == 9
    # Sec. 5.2.4: Cannon needs 2 sqrt(p) - 2 shifts, the hyper-systolic product 2K - 1
    for K in (2, 4, 8):
        assert bases.shifts_matrix_product(K, K) - (2 * K - 2) == 1


def test_matrix_product_bases_shapes():
    A, B, C = bases.matrix_product_bases(64, 8)
    assert A == [0] + [8] * 7 and B == [0] + [-1] * 7 and C == [0] + [1] * 7
    A, B, C = bases.matrix_product_bases(16, 2)
    assert A == [0] + [2] * 7 and B == [0, -1] and C == [0, 1]
