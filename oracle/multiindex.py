"""Multi-index sets for the O(D^p) expansions (section 2, note 1).

An expansion "of order p" keeps every multi-index alpha with |alpha| < p; there
are C(D+p-1, D) of them (section 2).  They are ordered by total degree, and
inside one degree in decreasing lexicographic order, so that for D = 2 the
order-2 set is (0,0), (1,0), (0,1): the coefficients stored for the example of
section 2 are sum w, sum w*x1, sum w*x2, in that order.  Because the order is
graded, the set of order p is a prefix of the set of any larger order, and a
coefficient vector of order PLIMIT holds every lower order as its first
C(D+p-1, D) entries.

The O(p^D) expansions of the DFTO variant (section 2; section 7 compares it)
keep instead every alpha with alpha_d < p in each dimension: p^D of them.  They
are ordered by their largest component, and inside one value of it in
decreasing lexicographic order, so that the set of order p is again a prefix
of the set of any larger order (its first p^D entries).
"""

import math

# PLIMIT per dimension as fixed for the experiments (section 6): 8 for D=2,
# 6 for D=3, 4 for D=5, 2 for D=6, 1 above 6.  D=1 and D=4 are not given; the
# values used for them are this implementation's reading.
_PLIMIT = {1: 10, 2: 8, 3: 6, 4: 5, 5: 4, 6: 2}


def plimit_for(D):
    """Maximum expansion order for dimension D (section 6)."""
    if D < 1:
        raise ValueError("D must be >= 1")
    return _PLIMIT.get(D, 1)


def _degree_block(D, deg):
    """All alpha in N^D with |alpha| = deg, decreasing lexicographic order."""
    if D == 1:
        return [(deg,)]
    out = []
    for first in range(deg, -1, -1):
        for rest in _degree_block(D - 1, deg - first):
            out.append((first,) + rest)
    return out


def multi_indices(D, p):
    """Graded list of all alpha with |alpha| < p (section 2)."""
    out = []
    for deg in range(p):
        out.extend(_degree_block(D, deg))
    return out


def num_terms(D, p):
    """Number of multi-indices with |alpha| < p: C(D+p-1, D) (section 2)."""
    return math.comb(D + p - 1, D)


def index_of(D, p):
    """Map alpha -> position in multi_indices(D, p)."""
    return {a: i for i, a in enumerate(multi_indices(D, p))}


def mi_factorial(alpha):
    """alpha! = alpha_1! ... alpha_D! (note 1)."""
    out = 1
    for a in alpha:
        out *= math.factorial(a)
    return out


def mi_degree(alpha):
    """|alpha| = alpha_1 + ... + alpha_D (note 1)."""
    return sum(alpha)


# Families of index sets: "graded" (|alpha| < p, the O(D^p) expansions) and
# "tensor" (every alpha_d < p, the O(p^D) expansions).
FAMILIES = ("graded", "tensor")

# Largest number of terms an expansion may have (the library's coefficient
# arrays hold at most this many).
MAX_TERMS = 286


def plimit_tensor(D):
    """Maximum order of the O(p^D) expansions: the O(D^p) limit of the same
    dimension, lowered until p^D <= MAX_TERMS (this implementation's reading;
    the paper fixes no limit for them)."""
    p = plimit_for(D)
    while p > 1 and p ** D > MAX_TERMS:
        p -= 1
    return p


def _max_block(D, m):
    """All alpha in N^D with max_d alpha_d = m, decreasing lexicographic order."""
    out = []

    def rec(prefix, left, hit):
        if left == 0:
            if hit:
                out.append(tuple(prefix))
            return
        for v in range(m, -1, -1):
            rec(prefix + [v], left - 1, hit or v == m)

    rec([], D, False)
    return out


def tensor_indices(D, p):
    """All alpha with alpha_d < p for every d, ordered by max component (the
    O(p^D) set of section 2)."""
    out = []
    for m in range(p):
        out.extend(_max_block(D, m))
    return out


def index_set(D, p, family="graded"):
    """The multi-indices of an expansion of order p in the given family."""
    if family == "graded":
        return multi_indices(D, p)
    if family == "tensor":
        return tensor_indices(D, p)
    raise ValueError(family)


def set_size(D, p, family="graded"):
    """C(D+p-1, D) for the graded family, p^D for the tensor family."""
    if family == "graded":
        return num_terms(D, p)
    if family == "tensor":
        return p ** D
    raise ValueError(family)
