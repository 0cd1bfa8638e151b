"""Ring simulator of the systolic and hyper-systolic matrix products, and of
the two-array hyper-systolic recipe (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (never imported by the product path).

The machine: a ring of p cells; cell i holds column i of three skew-ordered
p x p arrays a, b, c (Sec. 3.3.1), i.e. storage row r of cell i holds the
element ((i + r) mod p, i) (0-based).  It has one communication primitive,
the circular shift of Sec. 5.1, Eq. CSHIFT1: after a shift by s, cell i holds
what cell i + s held.  Reading a neighbouring storage row of the own column
(cshift-col) is a local address offset, not communication.

The product is driven by the three bases of Sec. 5.2.1 alone (0-based
indices, K * K~ = p):

* base B = (0, -1, .., -1), K entries: storage rows of b fall into K classes
  q mod K; class t is moved once, before any product, to the position
  P_B(t) = b_0 + .. + b_t = -t of the base (a right shift by t);
* base A = (0, K, .., K), K~ entries: a is moved by a_j before step j, so
  during step j it sits at P_A(j) = j K;
* base C = (0, 1, .., 1), K entries: the K auxiliary arrays c^0 .. c^{K-1}
  (Sec. 5.2.2) are combined by a collector that starts as c^{K-1}, is moved
  by c_t and then absorbs c^{t-1}, for t = K-1 .. 1.

During step j, class t of b contributes storage row q = P_A(j) - P_B(t)
(= j K + t), and each cell multiplies it with the a element whose storage
row lies P_A(j) - P_B(t) rows above the c^t row it updates.  Derivation:
after the moves, cell i holds a column (i + jK) of A and b column (i - t) of
B, and both share the contraction index (i + jK) mod p; the product belongs
to C column i - t, which the collector brings to cell i - t after t moves
by +1, at the storage row that the skew order gives it.

Elements may be numbers, numpy blocks (block mapping, Sec. 6.1: a p x p
system of sub-matrices used like scalars) or the symbolic terms below,
which record which products were formed.

Readings of points the text leaves open (each pinned by brute force in the
tests):
* skew order: the same for a, b and c (Figs. TEMPLATE/TEMPLATE2 are missing);
* the pre-shift stride of storage row q is -(q mod K): the remainder taken
  with the sign of the dividend (``preshift_stride``);
* a moves by K (not K~) between steps, as base A states.
"""
from collections import Counter

import numpy as np

from . import bases as _bases


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
# communication (Sec. 5.1, Eq. CSHIFT1)
# ----------------------------------------------------------------------------
class ShiftCounter:
    """Counts interprocessor communication events (whole-array shifts)."""

    def __init__(self):
        self.events = 0


def cshift_row(x, k, counter=None):
    """Shift a whole skew-ordered array along the ring: cell i receives the
    column of cell i + k (Eq. CSHIFT1)."""
    p = x.shape[1]
    src = [(i + k) % p for i in range(p)]
    out = x[:, src]
    if counter is not None:
        counter.events += 1
    return out


def preshift_stride(q, K):
    """Stride by which storage row q of b is moved before the first product:
    -(q mod K), the position P_B(q mod K) of base B = (0, -1, .., -1).  The
    printed stride [(1 - j) mod K] (1-based row j = q + 1) gives the same
    value when the remainder keeps the sign of the dividend."""
    return -(q % K)


def _zeros(p, zero):
    c = np.empty((p, p), dtype=object)
    for r in range(p):
        for i in range(p):
            c[r, i] = zero
    return c


# ----------------------------------------------------------------------------
# the systolic product (Sec. 5.1): base A = (0, 1, .., 1), one array c
# ----------------------------------------------------------------------------
def systolic(A, B, zero, trace=None):
    """C = A B on a ring of p cells in p steps: step j multiplies storage row
    j of b with a, read j rows up, and a then moves by one cell.  The last
    move only returns a to where it started.  Returns (C, shift_count)."""
    p = A.shape[0]
    a, b = to_skew(A), to_skew(B)
    c = _zeros(p, zero)
    cnt = ShiftCounter()
    for j in range(p):
        for i in range(p):
            for n in range(p):
                ae = a[(n - j) % p, i]
                be = b[j, i]
                c[n, i] = c[n, i] + ae * be
                if trace is not None:
                    trace.append((i, j, 0, n, ae, be))
        a = cshift_row(a, 1, cnt)
    return from_skew(c), cnt.events


# ----------------------------------------------------------------------------
# the hyper-systolic product (Sec. 5.2.2) driven by the bases of Sec. 5.2.1
# ----------------------------------------------------------------------------
def _positions(base):
    """Prefix sums of a base: where an array stands after each stride."""
    return _bases.prefix_sums(base)


def hyper_systolic(A, B, K, zero, trace=None):
    """C = A B with the regular bases A=(0,K,..,K), B=(0,-1,..,-1), C=(0,1,..,1).

    Returns (C, shift_count).  ``trace`` (a list) receives one record
    (i, j, t, n, a_elem, b_elem) per product formed: 0-based cell i, step j,
    auxiliary array t and storage row n of c^t.
    """
    p = A.shape[0]
    assert p % K == 0
    base_a, base_b, base_c = _bases.matrix_product_bases(p, K)
    pos_a = _positions(base_a)
    pos_b = _positions(base_b)                      # 0, -1, .., -(K-1)
    a, b = to_skew(A), to_skew(B)
    cnt = ShiftCounter()

    # base B: every storage row of b moves to its class position at once (the
    # printed stride, read by preshift_stride); the complexity count
    # (Thm. GAIN3) takes this as one event
    moved = np.empty_like(b)
    for q in range(p):
        s = preshift_stride(q, K)
        for i in range(p):
            moved[q, i] = b[q, (i + s) % p]
    b = moved
    cnt.events += 1

    c = [_zeros(p, zero) for _ in range(K)]
    for j, stride in enumerate(base_a):
        if j > 0:                                   # base A: a moves by a_j
            a = cshift_row(a, stride, cnt)
        for t in range(K):
            off = pos_a[j] - pos_b[t]               # = j K + t
            q = off % p                             # the storage row of b in use
            for i in range(p):
                be = b[q, i]
                for n in range(p):
                    ae = a[(n - off) % p, i]
                    c[t][n, i] = c[t][n, i] + ae * be
                    if trace is not None:
                        trace.append((i, j, t, n, ae, be))

    # base C: the collector picks up c^{K-1}, .., c^0, moving by c_t before
    # each pick-up
    coll = c[K - 1]
    for t in range(K - 1, 0, -1):
        coll = cshift_row(coll, base_c[t], cnt)
        coll = _add(c[t - 1], coll)
    return from_skew(coll), cnt.events


def _add(x, y):
    """Element-wise x + y of two object arrays (x's element first)."""
    out = np.empty_like(x)
    for r in range(x.shape[0]):
        for i in range(x.shape[1]):
            out[r, i] = x[r, i] + y[r, i]
    return out


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
