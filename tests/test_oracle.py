"""Pins for the FP64 oracle (CPU only).

The oracle is the plain definition of the product (Sec. 3.1, Eq. PRODUCT).
These checks tie it to facts that do not come from the oracle itself:
identities and permutations, exact integer arithmetic, the exactly rounded
sum with the standard dot-product error bound, an explicit transpose,
associativity, and central differences for the gradient.  Each check is a
function of the implementation under test, so the last group of tests can
plant plausible mistakes (a transposed operand, a dropped term, a wrong sign,
an off-by-one index) into a copy of the oracle and show that some pin fails.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_cs_9809105_amd import inputs

U = 2.0 ** -53  # unit roundoff of IEEE double


# ---------------------------------------------------------------------------
# pin functions: each takes (gemm, gemm_tn, gemv, backward) implementations
# ---------------------------------------------------------------------------
def pin_identity(gemm):
    A = inputs.uniform((13, 7), seed=1)
    ok = np.array_equal(gemm(A, np.eye(7)), A) and np.array_equal(gemm(np.eye(13), A), A)
    return ok


def pin_permutation(gemm):
    A = inputs.uniform((9, 11), seed=2)
    pr = inputs.rng(3).permutation(9)
    pc = inputs.rng(4).permutation(11)
    Pr = np.eye(9)[pr]            # (Pr A)[i] = A[pr[i]]
    Pc = np.eye(11)[:, pc]        # (A Pc)[:, j] = A[:, pc[j]]
    return np.array_equal(gemm(Pr, A), A[pr]) and np.array_equal(gemm(A, Pc), A[:, pc])


def pin_small_int(gemm):
    A = inputs.small_int((37, 29), seed=5)
    B = inputs.small_int((29, 23), seed=6)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    return np.array_equal(gemm(A, B), exact.astype(np.float64))


def pin_error_bound(gemm):
    """|c - exact| <= gamma_k sum|a||b| with exact rational arithmetic (Higham, Thm 3.1)."""
    m, k, n = 5, 17, 4
    A = inputs.normal((m, k), seed=7)
    B = inputs.normal((k, n), seed=8)
    C = gemm(A, B)
    gamma = k * U / (1 - k * U)
    for i in range(m):
        for j in range(n):
            exact = sum(Fraction(A[i, p]) * Fraction(B[p, j]) for p in range(k))
            absum = sum(abs(A[i, p] * B[p, j]) for p in range(k))
            if abs(Fraction(C[i, j]) - exact) > Fraction(gamma * absum * (1 + 1e-12)):
                return False
    return True


def pin_transpose(gemm, gemm_tn):
    A = inputs.normal((19, 12), seed=9)       # stored k x m
    B = inputs.normal((19, 15), seed=10)
    return np.array_equal(gemm_tn(A, B), gemm(np.ascontiguousarray(A.T), B))


def pin_tn_small_int(gemm_tn):
    ok = True
    for (k, m, n), s in (((21, 10, 14), 11), ((16, 16, 16), 12)):
        A = inputs.small_int((k, m), seed=s)
        B = inputs.small_int((k, n), seed=s + 100)
        exact = A.T.astype(np.int64) @ B.astype(np.int64)
        ok = ok and np.array_equal(gemm_tn(A, B), exact.astype(np.float64))
    return ok


def pin_associativity(gemm, gemv):
    A = inputs.small_int((17, 13), seed=13)
    B = inputs.small_int((13, 11), seed=14)
    x = inputs.small_int((11,), seed=15)
    return np.array_equal(gemv(gemm(A, B), x), gemv(A, gemv(B, x)))


def pin_gemv_small_int(gemv):
    A = inputs.small_int((31, 27), seed=16)
    x = inputs.small_int((27,), seed=17)
    return np.array_equal(gemv(A, x), (A.astype(np.int64) @ x.astype(np.int64)).astype(np.float64))


def pin_backward_fd(gemm, backward, size=(64, 64, 64), h=2.0 ** -4, ndir=24):
    """Central differences of L(A, B) = sum((A B) * G).

    L is linear in A for fixed B (and in B for fixed A), so the central
    difference equals the directional derivative up to rounding only.
    """
    m, k, n = size
    A = inputs.normal((m, k), seed=18)
    B = inputs.normal((k, n), seed=19)
    G = inputs.normal((m, n), seed=20)
    dA, dB = backward(A, B, G)

    def L(Ax, Bx):
        return float(np.sum(gemm(Ax, Bx) * G))

    g = inputs.rng(21)
    for t in range(ndir):
        if t < ndir // 2:
            D = g.standard_normal((m, k))
            fd = (L(A + h * D, B) - L(A - h * D, B)) / (2 * h)
            an = float(np.sum(dA * D))
        else:
            D = g.standard_normal((k, n))
            fd = (L(A, B + h * D) - L(A, B - h * D)) / (2 * h)
            an = float(np.sum(dB * D))
        if abs(fd - an) > 1e-9 * max(1.0, abs(an)):
            return False
    # unit directions: single entries of dA and dB
    for (i, p) in [(0, 0), (m - 1, k - 1), (3, k // 2)]:
        E = np.zeros((m, k))
        E[i, p] = 1.0
        fd = (L(A + h * E, B) - L(A - h * E, B)) / (2 * h)
        if abs(fd - dA[i, p]) > 1e-9 * max(1.0, abs(dA[i, p])):
            return False
    for (p, j) in [(0, 0), (k - 1, n - 1), (k // 3, 5)]:
        E = np.zeros((k, n))
        E[p, j] = 1.0
        fd = (L(A, B + h * E) - L(A, B - h * E)) / (2 * h)
        if abs(fd - dB[p, j]) > 1e-9 * max(1.0, abs(dB[p, j])):
            return False
    return True


def pin_backward_small_int(backward):
    A = inputs.small_int((12, 9), seed=22)
    B = inputs.small_int((9, 14), seed=23)
    G = inputs.small_int((12, 14), seed=24)
    dA, dB = backward(A, B, G)
    Ai, Bi, Gi = (x.astype(np.int64) for x in (A, B, G))
    return np.array_equal(dA, (Gi @ Bi.T).astype(np.float64)) and \
        np.array_equal(dB, (Ai.T @ Gi).astype(np.float64))


def all_pins(gemm, gemm_tn, gemv, backward):
    return {
        "identity": pin_identity(gemm),
        "permutation": pin_permutation(gemm),
        "small_int": pin_small_int(gemm),
        "error_bound": pin_error_bound(gemm),
        "transpose": pin_transpose(gemm, gemm_tn),
        "tn_small_int": pin_tn_small_int(gemm_tn),
        "associativity": pin_associativity(gemm, gemv),
        "gemv_small_int": pin_gemv_small_int(gemv),
        "backward_fd": pin_backward_fd(gemm, backward, size=(24, 20, 16), ndir=8),
        "backward_small_int": pin_backward_small_int(backward),
    }


# ---------------------------------------------------------------------------
# the oracle passes every pin
# ---------------------------------------------------------------------------
def test_identity():
    assert pin_identity(oracle.gemm)


def test_permutation():
    assert pin_permutation(oracle.gemm)


def test_small_int_exact():
    assert pin_small_int(oracle.gemm)


def test_exact_rational_error_bound():
    assert pin_error_bound(oracle.gemm)


def test_transposed_product_is_explicit_transpose():
    assert pin_transpose(oracle.gemm, oracle.gemm_tn)
    assert pin_tn_small_int(oracle.gemm_tn)


def test_associativity_and_gemv():
    assert pin_associativity(oracle.gemm, oracle.gemv)
    assert pin_gemv_small_int(oracle.gemv)


def test_backward_central_differences_fp64_64cubed():
    """The FP64 64 x 64 x 64 finite-difference check of the differentiation workload."""
    assert pin_backward_fd(oracle.gemm, oracle.backward)


def test_backward_small_int():
    assert pin_backward_small_int(oracle.backward)


def test_sampled_rows_match_full():
    A = inputs.normal((40, 33), seed=30)
    B = inputs.normal((33, 21), seed=31)
    G = inputs.normal((40, 21), seed=32)
    rows = inputs.sample_rows(40, 7, seed=33)
    assert np.array_equal(oracle.gemm_rows(A, B, rows), oracle.gemm(A, B)[rows])
    At = np.ascontiguousarray(A.T)
    assert np.array_equal(oracle.gemm_tn_rows(At, G[:33], rows[:5] % 33),
                          oracle.gemm_tn(At, G[:33])[rows[:5] % 33])
    dA, dB = oracle.backward(A, B, G)
    assert np.array_equal(oracle.grad_a_rows(G, B, rows), dA[rows])
    rb = rows % 33
    assert np.array_equal(oracle.grad_b_rows(A, G, rb), dB[rb])


def test_empty_shapes():
    assert oracle.gemm(np.zeros((0, 3)), np.zeros((3, 4))).shape == (0, 4)
    C = oracle.gemm(np.zeros((2, 0)), np.zeros((0, 4)))
    assert C.shape == (2, 4) and not C.any()
    assert oracle.gemv(np.zeros((3, 0)), np.zeros(0)).tolist() == [0.0, 0.0, 0.0]


def test_thread_count_does_not_change_bits():
    """Each element is one ascending sum: results are independent of OpenMP threads."""
    import subprocess
    import sys
    code = ("import numpy as np, oracle; from paper_cs_9809105_amd import inputs;"
            "A=inputs.normal((64,300),seed=40);B=inputs.normal((300,50),seed=41);"
            "print(oracle.gemm(A,B).tobytes().hex()[:4000])")
    outs = []
    for t in ("1", "5"):
        env = dict(__import__("os").environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env,
                                            cwd=__import__("os").path.dirname(
                                                __import__("os").path.dirname(__file__))))
    assert outs[0] == outs[1]


# ---------------------------------------------------------------------------
# planted mistakes: a copy of the oracle with one plausible bug fails a pin
# ---------------------------------------------------------------------------
def _np_gemm(A, B):
    return oracle.gemm(A, B)


MUTANTS = {
    # B used transposed where the shapes allow it: square B makes it silent
    "transposed_B": dict(gemm=lambda A, B: oracle.gemm(A, np.ascontiguousarray(B.T))
                         if B.shape[0] == B.shape[1] else oracle.gemm(A, B)),
    # last contraction term dropped
    "dropped_term": dict(gemm=lambda A, B: oracle.gemm(A[:, :-1], B[:-1, :])
                         if A.shape[1] > 1 else oracle.gemm(A, B)),
    # wrong sign on one term
    "sign": dict(gemm=lambda A, B: oracle.gemm(A, B) - 2 * np.outer(A[:, 0], B[0, :])
                 if A.shape[1] > 1 else oracle.gemm(A, B)),
    # off-by-one contraction index (k+1 wraps)
    "index_shift": dict(gemm=lambda A, B: oracle.gemm(A, np.roll(B, 1, axis=0))),
    # transposed product forgets the transpose on square operands
    "tn_no_transpose": dict(gemm_tn=lambda A, B: oracle.gemm(A, B)
                            if A.shape[0] == A.shape[1] else oracle.gemm_tn(A, B)),
    # transposed product reads A with the untransposed index (A[i, p] of the
    # k x m storage reinterpreted as m x k)
    "tn_wrong_index": dict(gemm_tn=lambda A, B: oracle.gemm(
        np.ascontiguousarray(A).reshape(A.shape[1], A.shape[0]), B)),
    # gemv drops the last column
    "gemv_dropped": dict(gemv=lambda A, x: oracle.gemv(A[:, :-1], x[:-1])),
    # gradient of A uses B instead of B^T pattern (roll of columns)
    "grad_a_wrong": dict(backward=lambda A, B, G: (
        np.roll(oracle.backward(A, B, G)[0], 1, axis=1), oracle.backward(A, B, G)[1])),
    # gradient of B with a sign error
    "grad_b_sign": dict(backward=lambda A, B, G: (
        oracle.backward(A, B, G)[0], -oracle.backward(A, B, G)[1])),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    impl = dict(gemm=oracle.gemm, gemm_tn=oracle.gemm_tn, gemv=oracle.gemv,
                backward=oracle.backward)
    impl.update(MUTANTS[name])
    res = all_pins(**impl)
    assert not all(res.values()), "mutant %s passed every pin: %r" % (name, res)


def test_unmutated_oracle_passes_all_pins():
    res = all_pins(oracle.gemm, oracle.gemm_tn, oracle.gemv, oracle.backward)
    assert all(res.values()), res


def test_thread_count_does_not_change_results():
    A = inputs.normal((67, 45), seed=71)
    B = inputs.normal((45, 38), seed=72)
    ref = oracle.gemm(A, B)
    oracle.set_threads(1)
    try:
        one = oracle.gemm(A, B)
    finally:
        oracle.set_threads(0)
    assert np.array_equal(one, ref)
