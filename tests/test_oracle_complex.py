"""Pins of the complex product of the oracle (CPU): numpy's complex matmul,
exact Gaussian-integer products, the unit i, conjugation, real inputs, and
the 2 x 2 real block embedding that the library's complex forms run."""
import numpy as np

import oracle
from paper_cs_9809105_amd import inputs


def _cplx(shape, seed, gen=inputs.normal):
    return gen(shape, seed) + 1j * gen(shape, seed + 1)


def test_matches_numpy_complex_matmul():
    A = _cplx((37, 53), 1)
    B = _cplx((53, 29), 3)
    ref = A @ B
    got = oracle.complex_gemm(A, B)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(A) @ np.abs(B))


def test_gaussian_integers_exact():
    A = _cplx((40, 64), 5, inputs.small_int)
    B = _cplx((64, 24), 7, inputs.small_int)
    ref = A @ B                                  # integers, exact in float64
    assert np.array_equal(oracle.complex_gemm(A, B), ref)


def test_unit_i_and_conjugation():
    A = _cplx((17, 19), 9)
    B = _cplx((19, 11), 11)
    assert np.array_equal(oracle.complex_gemm(A, 1j * np.eye(19)), 1j * A)
    assert np.array_equal(np.conj(oracle.complex_gemm(A, B)), oracle.complex_gemm(np.conj(A), np.conj(B)))


def test_real_inputs_reduce_to_the_real_product():
    A = inputs.normal((21, 33), 13)
    B = inputs.normal((33, 15), 14)
    got = oracle.complex_gemm(A.astype(np.complex128), B.astype(np.complex128))
    assert np.array_equal(got.real, oracle.gemm(A, B)) and not got.imag.any()


def test_rows_agree_with_full_product():
    A = _cplx((30, 20), 15)
    B = _cplx((20, 25), 17)
    rows = [0, 7, 29]
    assert np.array_equal(oracle.complex_gemm_rows(A, B, rows), oracle.complex_gemm(A, B)[rows])


def test_real_block_embedding_identity():
    """A (as m x 2k reals) times the embedding of B (2k x 2n, block (t, j) =
    [[re b, im b], [-im b, re b]]) is C = A . B as m x 2n interleaved reals."""
    A = _cplx((12, 9), 19, inputs.small_int)
    B = _cplx((9, 7), 21, inputs.small_int)
    k, n = B.shape
    E = np.zeros((2 * k, 2 * n))
    E[0::2, 0::2], E[0::2, 1::2] = B.real, B.imag
    E[1::2, 0::2], E[1::2, 1::2] = -B.imag, B.real
    Ar = np.empty((12, 2 * k))
    Ar[:, 0::2], Ar[:, 1::2] = A.real, A.imag
    Cr = oracle.gemm(Ar, E)
    C = oracle.complex_gemm(A, B)
    assert np.array_equal(Cr[:, 0::2], C.real) and np.array_equal(Cr[:, 1::2], C.imag)


def test_error_metric_counts_imaginary_parts():
    from oracle.metrics import err_row
    ref = np.array([[1 + 1j, 2 - 1j]])
    assert err_row(ref, ref) == 0.0
    assert err_row(ref + 1e-3j, ref) > 1e-4        # an error only in the imaginary parts


def _blocks(X):
    """Real 2 x 2 block embedding of X (r x c complex): 2r x 2c reals with
    block (t, j) = [[re x, im x], [-im x, re x]]."""
    r, c = X.shape
    E = np.zeros((2 * r, 2 * c))
    E[0::2, 0::2], E[0::2, 1::2] = X.real, X.imag
    E[1::2, 0::2], E[1::2, 1::2] = -X.imag, X.real
    return E


def _as_reals(X):
    R = np.empty((X.shape[0], 2 * X.shape[1]))
    R[:, 0::2], R[:, 1::2] = X.real, X.imag
    return R


def test_backward_embeddings():
    """The gradients of C = A . B for complex data (G = dL/dC in PyTorch's
    convention): dA = G . B^H and dB = A^H . G, each as one real product of
    (complex as reals) and (block embedding), as the library runs them."""
    import torch
    A = _cplx((6, 5), 23, inputs.small_int)
    B = _cplx((5, 4), 25, inputs.small_int)
    G = _cplx((6, 4), 27, inputs.small_int)
    # PyTorch's own complex autograd fixes the convention
    At = torch.tensor(A, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    (At @ Bt).backward(torch.tensor(G))
    dA = oracle.complex_gemm(G, np.conj(B).T)
    dB = oracle.complex_gemm(np.conj(A).T, G)
    assert np.array_equal(At.grad.numpy(), dA) and np.array_equal(Bt.grad.numpy(), dB)
    # dA: G as reals times the block embedding of B^H
    dA_r = oracle.gemm(_as_reals(G), _blocks(np.conj(B).T))
    assert np.array_equal(dA_r, _as_reals(dA))
    # dB: conj(A)^T as reals times the block embedding of G
    dB_r = oracle.gemm(_as_reals(np.conj(A).T), _blocks(G))
    assert np.array_equal(dB_r, _as_reals(dB))


def test_complex_gemv_brute_force_gaussian_integers():
    """Python's own complex integers, one product at a time (exact)."""
    A = _cplx((13, 21), 21, inputs.small_int)
    x = _cplx((21,), 23, inputs.small_int)
    ref = [sum(complex(A[i, j]) * complex(x[j]) for j in range(21)) for i in range(13)]
    assert np.array_equal(oracle.complex_gemv(A, x), np.array(ref))


def test_complex_gemv_is_a_one_column_product():
    A = _cplx((30, 47), 25)
    x = _cplx((47,), 27)
    got = oracle.complex_gemv(A, x)
    assert np.allclose(got, oracle.complex_gemm(A, x[:, None])[:, 0], rtol=1e-14, atol=0)
    assert np.allclose(got, A @ x, rtol=1e-13, atol=1e-13 * np.abs(A) @ np.abs(x))
