"""Hyper-systolic bases (Sec. 4.2-4.4 and Sec. 5.2.1).

TEST INFRASTRUCTURE ONLY.  Written from the definitions; used to pin the
library's schedule generator and the counting theorems.
"""


def regular_bases_two_array(n, K):
    """Def. REGULARBASE2: A=(0,1,..,1) with K-1 ones, B=(0,K,..,K) with K~-1 K's."""
    assert n % K == 0
    Kt = n // K
    return [0] + [1] * (K - 1), [0] + [K] * (Kt - 1)


def matrix_product_bases(p, K):
    """Sec. 5.2.1: A=(0,K,..,K) (K~-1 entries), B=(0,-1,..,-1), C=(0,1,..,1) (K-1)."""
    assert p % K == 0
    Kt = p // K
    return [0] + [K] * (Kt - 1), [0] + [-1] * (K - 1), [0] + [1] * (K - 1)


def ordered_partial_sums(base):
    """All sums a_i + ... + a_{i+j} over contiguous runs of the base (Eq. ADD2)."""
    s = set()
    for i in range(len(base)):
        acc = 0
        for j in range(i, len(base)):
            acc += base[j]
            s.add(acc)
    return s


def h_range_complete(A, B, n):
    """True iff every m in 0..n-1 is a sum of two ordered partial sums (Def. DEF:OPTI2,
    read literally: any contiguous run of each base)."""
    sa, sb = ordered_partial_sums(A), ordered_partial_sums(B)
    reach = {x + y for x in sa for y in sb}
    return all(m in reach for m in range(n))


def shifts_two_array(K, Kt):
    """Thm. GAIN2, Eq. COMPLEXR: (K-1) + (K~-1) forward shifts, (K-1) back-shifts."""
    return 2 * K + Kt - 3


def shifts_matrix_product(K, Kt):
    """Thm. GAIN3, Eq. COMPL: 1 pre-shift of B, K~-1 shifts of A, K-1 of C."""
    return K + Kt - 1


def prefix_sums(base):
    """Positions an array visits when moved by the strides of ``base`` in turn
    (a_0 = 0 first): 0, a_1, a_1 + a_2, ..."""
    out, acc = [], 0
    for a in base:
        acc += a
        out.append(acc)
    return out


def recipe_complete(A, B, n):
    """True iff the two-array recipe (Sec. 4.1) with these bases pairs every
    offset: replica t of x sits at offset P_A(t), the travelling z at P_B(j),
    so the pairs met have offsets (P_B(j) - P_A(t)) mod n, and all n residues
    must occur."""
    pa, pb = prefix_sums(A), prefix_sums(B)
    return len({(y - x) % n for x in pa for y in pb}) == n
