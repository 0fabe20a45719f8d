"""Pin P1: the oracle's Runge-Kutta tableaux satisfy the order conditions.

The order of an explicit Runge-Kutta method is fixed by Butcher's rooted-tree
conditions sum_j b_j Phi_j(t) = 1/gamma(t) (Hairer, Norsett & Wanner I,
Sec. II.2).  The trees are generated here from scratch and the conditions are
evaluated in 40-digit arithmetic, so a mistyped coefficient shows up as a
residual far above the ~1e-14 left by 16-digit published values.
Tsit5 is Tsitouras' 5(4) pair and Vern7 Verner's 7(6) pair (paper,
Sections 2.1 and 3.2).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np
import pytest

import oracle as O

mp.mp.dps = 40


@lru_cache(None)
def _trees(n):
    """Rooted trees with n nodes, each a sorted tuple of child subtrees."""
    if n == 1:
        return ((),)
    out = set()

    def forests(k, maxt):
        if k == 0:
            yield ()
            return
        for m in range(1, k + 1):
            for t in _trees(m):
                if maxt is not None and t > maxt:
                    continue
                for rest in forests(k - m, t):
                    yield (t,) + rest

    for f in forests(n - 1, None):
        out.add(tuple(sorted(f)))
    return tuple(sorted(out))


def _nodes(t):
    return 1 + sum(_nodes(c) for c in t)


def _gamma(t):
    g = _nodes(t)
    for c in t:
        g *= _gamma(c)
    return g


def _phi(t, A):
    s = len(A)
    v = [mp.mpf(1)] * s
    for ch in t:
        w = _phi(ch, A)
        Aw = [mp.fsum(A[i][j] * w[j] for j in range(s)) for i in range(s)]
        v = [v[i] * Aw[i] for i in range(s)]
    return v


def _residuals(A, b, order, rhs_one=True):
    res = []
    for o in range(1, order + 1):
        for t in _trees(o):
            lhs = mp.fsum(bi * x for bi, x in zip(b, _phi(t, A)))
            res.append(abs(lhs - (mp.mpf(1) / _gamma(t) if rhs_one else 0)))
    return res


def test_tree_counts():
    # number of rooted trees of order 1..8 (OEIS A000081)
    assert [len(_trees(k)) for k in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]


def _mp_tab(method):
    tb = O.erk_tableau(method)
    A = [[mp.mpf(float(x)) for x in row] for row in tb["A"]]
    b = [mp.mpf(float(x)) for x in tb["b"]]
    ew = [mp.mpf(float(x)) for x in tb["ew"]]
    return tb, A, b, ew


@pytest.mark.parametrize("method,p,q,ncond", [(O.TSIT5, 5, 4, 17), (O.VERN7, 7, 6, 85)])
def test_order_conditions(method, p, q, ncond):
    tb, A, b, ew = _mp_tab(method)
    assert tb["order"] == p and tb["q_emb"] == q
    rb = _residuals(A, b, p)
    assert len(rb) == ncond
    assert max(rb) < 2e-14, max(rb)
    # the method is not of order p+1 (the tableau is the intended one, not a
    # degenerate higher-order accident)
    assert max(_residuals(A, b, p + 1)) > 1e-6
    # embedded weights bhat = b - ew reach order q exactly
    bh = [x - y for x, y in zip(b, ew)]
    assert max(_residuals(A, bh, q)) < 2e-14
    assert max(_residuals(A, bh, q + 1)) > 1e-6
    # row sums: c_i = sum_j a_ij
    for i in range(tb["s"]):
        assert abs(mp.fsum(A[i]) - mp.mpf(float(tb["c"][i]))) < 1e-13
    # explicit: strictly lower triangular
    assert np.all(np.triu(tb["A"]) == 0.0)


def test_tsit5_structure():
    tb = O.erk_tableau(O.TSIT5)
    assert tb["s"] == 7
    # first-same-as-last: last row of A equals b, c_7 = 1, b_7 = 0
    assert np.array_equal(tb["A"][6, :6], tb["b"][:6])
    assert tb["b"][6] == 0.0 and tb["c"][6] == 1.0
    # nodes that identify Tsitouras' table
    assert np.allclose(tb["c"][:4], [0.0, 0.161, 0.327, 0.9])


def test_vern7_structure():
    tb = O.erk_tableau(O.VERN7)
    assert tb["s"] == 10
    # b uses stages 1,4..9; bhat uses 1,4..7 and 10
    assert tb["b"][1] == tb["b"][2] == tb["b"][9] == 0.0
    bh = tb["b"] - tb["ew"]
    assert np.all(bh[[1, 2, 7, 8]] == 0.0)
