"""Pins of the oracle's Runge--Kutta tableaux (Appendix A) against the
order conditions, computed in exact rational arithmetic."""
from fractions import Fraction as F

import pytest

from oracle import tableaux


def rooted_trees(order):
    """All rooted trees with `order` nodes; a tree is a sorted tuple of
    its children (each a tree)."""
    if order == 1:
        return [()]
    out = set()
    # children multisets whose node counts sum to order - 1
    def parts(remaining, max_first):
        if remaining == 0:
            yield []
            return
        for first in range(min(remaining, max_first), 0, -1):
            for rest in parts(remaining - first, first):
                yield [first] + rest
    for p in parts(order - 1, order - 1):
        combos = [[]]
        for size in p:
            combos = [c + [t] for c in combos for t in rooted_trees(size)]
        for c in combos:
            out.add(tuple(sorted(c)))
    return sorted(out)


def size(t):
    return 1 + sum(size(c) for c in t)


def gamma(t):
    g = size(t)
    for c in t:
        g *= gamma(c)
    return g


def g_vec(t, A):
    """Internal elementary weight vector: 1 for a leaf, else the
    elementwise product over children of A g(child)."""
    s = len(A)
    v = [F(1)] * s
    for c in t:
        gc = g_vec(c, A)
        Agc = [sum(A[i][j] * gc[j] for j in range(s)) for i in range(s)]
        v = [v[i] * Agc[i] for i in range(s)]
    return v


def satisfies(b, A, t):
    return sum(bi * gi for bi, gi in zip(b, g_vec(t, A))) == F(1, gamma(t))


def test_tree_counts():
    # number of rooted trees of order 1..6 (OEIS A000081)
    assert [len(rooted_trees(k)) for k in range(1, 7)] == [1, 1, 2, 4, 9, 20]


@pytest.mark.parametrize("tab,name", [(tableaux.RK4, "rk4"), (tableaux.BS5, "bs5"),
                                      (tableaux.DP5, "dp5")])
def test_row_sums_equal_c(tab, name):
    for row, c in zip(tab["A"], tab["c"]):
        assert sum(row) == c
    for i, row in enumerate(tab["A"]):
        assert all(x == 0 for x in row[i:]), "explicit: strictly lower triangular"


@pytest.mark.parametrize("tab,order", [(tableaux.RK4, 4), (tableaux.BS5, 5), (tableaux.DP5, 5)])
def test_main_weights_order(tab, order):
    for p in range(1, order + 1):
        for t in rooted_trees(p):
            assert satisfies(tab["b"], tab["A"], t), (p, t)
    # and not one order higher
    assert not all(satisfies(tab["b"], tab["A"], t) for t in rooted_trees(order + 1))


@pytest.mark.parametrize("tab", [tableaux.BS5, tableaux.DP5])
def test_embedded_weights_order4(tab):
    for p in range(1, 5):
        for t in rooted_trees(p):
            assert satisfies(tab["bhat"], tab["A"], t), (p, t)
    assert not all(satisfies(tab["bhat"], tab["A"], t) for t in rooted_trees(5))


@pytest.mark.parametrize("tab", [tableaux.BS5, tableaux.DP5])
def test_fsal(tab):
    assert tab["A"][-1] == tab["b"]
    assert tab["c"][-1] == 1


def stability_coeffs(tab, b):
    A = tab["A"]
    s = len(A)
    v = [F(1)] * s
    out = [F(1)]
    for _ in range(s):
        out.append(sum(bi * vi for bi, vi in zip(b, v)))
        v = [sum(A[i][j] * v[j] for j in range(s)) for i in range(s)]
    return out


def test_bs5_stability_polynomials():
    """R(z) = 1 + sum_j b^T A^(j-1) 1 z^j: Taylor through z^5 for b,
    through z^4 for b_hat, then the pair's own tail coefficients."""
    from math import factorial
    R = stability_coeffs(tableaux.BS5, tableaux.BS5["b"])
    Rh = stability_coeffs(tableaux.BS5, tableaux.BS5["bhat"])
    assert R[:6] == [F(1, factorial(j)) for j in range(6)]
    assert R[6:] == [F(17291, 12418560), F(269, 1379840), F(0)]
    assert Rh[:5] == [F(1, factorial(j)) for j in range(5)]
    assert Rh[5] != F(1, 120)
    assert Rh[5:] == [F(269672, 32164209), F(2349047, 1715424480),
                      F(1309661503, 6916591503360), F(885817, 768510167040)]
