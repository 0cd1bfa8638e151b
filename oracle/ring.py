"""Literal simulator of the systolic and hyper-systolic matrix products.

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
