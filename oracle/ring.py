"""Literal simulator of the systolic and hyper-systolic matrix products, and
of the two-array hyper-systolic recipe (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (never imported by the product path).

A ring of p cells, each cell i holding column i of three skew-ordered p x p
arrays a, b, c (Sec. 3.3.1).  The two data movements are exactly the paper's:

* ``cshift_row(x, k)`` -- Sec. 5.1, Eq. CSHIFT1: cell i receives the column of
  cell i+k (1-based: a_{j,(i+k-1+n) mod n + 1}); interprocessor communication.
* ``cshift_col(x, k)`` -- Sec. 5.1: inside every cell, storage row j reads
  storage row j+k (a_{(j+k-1+n) mod n + 1, i}); a local address offset only.

``systolic`` runs Algorithm SYSTOLIC and ``hyper_systolic`` Algorithm
HYPER-SYSTOLIC (Sec. 5.2.2) step by step in the paper's order and notation
(1-based loop variables).  Elements may be numbers, numpy blocks (block
mapping, Sec. 6.1: a p x p system of sub-matrices used like scalars) or the
symbolic terms below, which record which products were formed.

Readings of points the text leaves open (each pinned by brute force in the
tests):
* skew order: storage row r of cell i holds element ((i + r) mod p, i),
  0-based, for all of a, b and c (Figs. TEMPLATE/TEMPLATE2 are missing);
* pre-shift stride ``[(1-j) mod K]`` uses the remainder with the sign of the
  dividend (Fortran MOD / C %), i.e. row j moves by -((j-1) mod K);
* A moves by K (not K~) between the K~ groups, as in the algorithm listing.
"""
from collections import Counter

import numpy as np


# ----------------------------------------------------------------------------
# skew order (Sec. 3.2.1 / 3.3.1)
# ----------------------------------------------------------------------------
def to_skew(M):
    """p x p object array -> storage s[r, i] = M[(i + r) mod p, i]."""
    p = M.shape[0]
    s = np.empty((p, p), dtype=object)
    for i in range(p):
        for r in range(p):
            s[r, i] = M[(i + r) % p, i]
    return s


def from_skew(s):
    p = s.shape[0]
    M = np.empty((p, p), dtype=object)
    for i in range(p):
        for r in range(p):
            M[(i + r) % p, i] = s[r, i]
    return M


# ----------------------------------------------------------------------------
# the two shift primitives (Sec. 5.1)
# ----------------------------------------------------------------------------
class ShiftCounter:
    """Counts interprocessor communication events (cshift-row calls)."""

    def __init__(self):
        self.events = 0


def _fmod(a, b):
    """Remainder with the sign of the dividend (Fortran MOD, C %)."""
    r = abs(a) % abs(b)
    return -r if a < 0 else r


def cshift_row(x, k, counter=None):
    """Eq. CSHIFT1 on the whole array: new[:, i] = old[:, (i + k) mod n]."""
    n = x.shape[1]
    out = np.empty_like(x)
    for i1 in range(1, n + 1):                      # 1-based cell index
        src = (i1 + k - 1 + n) % n + 1
        out[:, i1 - 1] = x[:, src - 1]
    if counter is not None:
        counter.events += 1
    return out


def cshift_row_1(col_values, k, i1, n):
    """Value arriving at cell i1 (1-based) when one storage row moves by k."""
    return col_values[(i1 + k - 1 + n) % n]


def cshift_col(x, k, j1, i1):
    """Element (j1, i1) (1-based) of cshift-col^k(x): x_{(j+k-1+n) mod n + 1, i}."""
    n = x.shape[0]
    return x[(j1 + k - 1 + n) % n, i1 - 1]


# ----------------------------------------------------------------------------
# Algorithm SYSTOLIC (Sec. 5.1)
# ----------------------------------------------------------------------------
def systolic(A, B, zero, trace=None):
    """C = A B on a ring of p cells, p steps, A travels by one each step."""
    p = A.shape[0]
    a, b = to_skew(A), to_skew(B)
    c = np.empty((p, p), dtype=object)
    c[:, :] = [[zero for _ in range(p)] for _ in range(p)]
    cnt = ShiftCounter()
    for j in range(1, p + 1):
        for i in range(1, p + 1):                   # foreach processor (SIMD)
            for l in range(1, p + 1):
                ae = cshift_col(a, 1 - j, l, i)
                be = b[j - 1, i - 1]
                c[l - 1, i - 1] = c[l - 1, i - 1] + ae * be
                if trace is not None:
                    trace.append((i, j, l, ae, be))
        a = cshift_row(a, 1, cnt)
    return from_skew(c), cnt.events


# ----------------------------------------------------------------------------
# Algorithm HYPER-SYSTOLIC (Sec. 5.2.2)
# ----------------------------------------------------------------------------
def hyper_systolic(A, B, K, zero, trace=None):
    """C = A B with the regular bases A=(0,K,..,K), B=(0,-1,..,-1), C=(0,1,..,1).

    Returns (C, shift_count).  ``trace`` (a list) receives one record
    (i, j, l, n, a_elem, b_elem) per block product formed, with 1-based cell
    i, step j, auxiliary array l and storage row n.
    """
    p = A.shape[0]
    assert p % K == 0
    Kt = p // K
    a, b = to_skew(A), to_skew(B)
    cnt = ShiftCounter()

    # pre-shift of B: storage row j moves by [(1-j) mod K]; all rows move at
    # once, which the complexity count treats as one communication event.
    nb = np.empty_like(b)
    for j in range(1, p + 1):
        stride = _fmod(1 - j, K)
        for i in range(1, p + 1):
            nb[j - 1, i - 1] = cshift_row_1(b[j - 1, :], stride, i, p)
    b = nb
    cnt.events += 1

    # K auxiliary result arrays C^1..C^K
    c = {}
    for l in range(1, K + 1):
        c[l] = np.empty((p, p), dtype=object)
        c[l][:, :] = [[zero for _ in range(p)] for _ in range(p)]

    def multiply(j):
        for i in range(1, p + 1):
            for l in range(1, K + 1):
                for n in range(1, p + 1):
                    ae = cshift_col(a, 1 - (j - 1) * K - l, n, i)
                    be = b[(j - 1) * K + l - 1, i - 1]
                    c[l][n - 1, i - 1] = c[l][n - 1, i - 1] + ae * be
                    if trace is not None:
                        trace.append((i, j, l, n, ae, be))

    for j in range(1, Kt):                          # multiplication and shift of A
        multiply(j)
        a = cshift_row(a, K, cnt)
    multiply(Kt)

    for j in range(1, K):                           # back shift and accumulation
        shifted = cshift_row(c[K - j + 1], 1, cnt)
        c[K - j] = c[K - j] + shifted

    return from_skew(c[1]), cnt.events


# ----------------------------------------------------------------------------
# symbolic elements: record which products reach which result element
# ----------------------------------------------------------------------------
class Leaf:
    """An input element identified by (matrix name, row, column)."""

    __slots__ = ("name", "r", "c")

    def __init__(self, name, r, c):
        self.name, self.r, self.c = name, r, c

    def key(self):
        return (self.name, self.r, self.c)

    def __mul__(self, other):
        return Term(Counter({(self.key(), other.key()): 1}))

    def __repr__(self):
        return "%s[%d,%d]" % (self.name, self.r, self.c)


class Term:
    """A multiset of products (sum of products with multiplicities)."""

    __slots__ = ("prods",)

    def __init__(self, prods=None):
        self.prods = prods if prods is not None else Counter()

    def __add__(self, other):
        return Term(self.prods + other.prods)

    def __eq__(self, other):
        return isinstance(other, Term) and self.prods == other.prods

    def __repr__(self):
        return "Term(%r)" % (dict(self.prods),)


def leaves(name, p):
    M = np.empty((p, p), dtype=object)
    for r in range(p):
        for c in range(p):
            M[r, c] = Leaf(name, r, c)
    return M


def expected_terms(p, a_name="A", b_name="B"):
    """c_ij = sum_k a_ik b_kj as multisets, each product exactly once."""
    C = np.empty((p, p), dtype=object)
    for i in range(p):
        for j in range(p):
            C[i, j] = Term(Counter({((a_name, i, k), (b_name, k, j)): 1 for k in range(p)}))
    return C


# ----------------------------------------------------------------------------
# the two-array recipe (Sec. 4.1) on the regular bases (Def. REGULARBASE2)
# ----------------------------------------------------------------------------
def cshift_1d(x, k, counter=None):
    """One row of Eq. CSHIFT1: cell i receives the element of cell i + k."""
    n = len(x)
    out = np.empty(n, dtype=object)
    for i in range(n):
        out[i] = x[(i + k) % n]
    if counter is not None:
        counter.events += 1
    return out


def _cells(x):
    """1D object array holding x's elements one per cell (blocks stay whole)."""
    out = np.empty(len(x), dtype=object)
    for i in range(len(x)):
        out[i] = x[i]
    return out


def two_array(x, z, K, f, zero):
    """F_i = sum_j f(x_i, z_j) on a ring of p = len(x) cells (Sec. 4.1).

    Step by step as the recipe states it, with A = (0, 1, .., 1) (K - 1
    ones) and B = (0, K, .., K) (K~ - 1 entries K), K K~ = p:
      1. K replicas x^_t of x, each made from the previous one by a shift of
         stride a_t (x^_0 = x);
      2. z visits its K~ positions, moved by the strides b_t;
      3. after each move of z, every cell adds f(x^_t, z) into the
         intermediate result y^_t, t = 0..K-1;
      4. a collector starts as y^_{K-1} and is moved by the inverse strides
         -a_t, adding y^_{t-1} after each move.
    Elements may be numbers or numpy blocks (one block of bodies per cell);
    ``zero()`` makes a fresh zero result.  Returns (y, shift_count)."""
    p = len(x)
    assert len(z) == p and p % K == 0
    Kt = p // K
    a = [0] + [1] * (K - 1)
    b = [0] + [K] * (Kt - 1)
    cnt = ShiftCounter()
    xh = [_cells(x)]
    for t in range(1, K):
        xh.append(cshift_1d(xh[-1], a[t], cnt))
    yh = []
    for t in range(K):
        yt = np.empty(p, dtype=object)
        for i in range(p):
            yt[i] = zero()
        yh.append(yt)
    zc = _cells(z)
    for j in range(Kt):
        if j > 0:
            zc = cshift_1d(zc, b[j], cnt)
        for t in range(K):
            for i in range(p):
                yh[t][i] = yh[t][i] + f(xh[t][i], zc[i])
    y = yh[K - 1]
    for t in range(K - 1, 0, -1):
        y = cshift_1d(y, -a[t], cnt)
        for i in range(p):
            y[i] = y[i] + yh[t - 1][i]
    return y, cnt.events
