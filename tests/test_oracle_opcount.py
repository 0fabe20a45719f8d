"""Pins for the algorithmic work figures that set every roofline fraction.

The per-unit operation counts in the package's flops table must equal the
counts of the oracle's own step routines run on its operation-counting scalar
(fma 2; +, -, *, /, min, max, sqrt, tanh and the controller's root 1;
negation, abs and comparisons 0).  The counter itself is pinned by counting
by hand: the explicit pairs' trial and reverse steps follow from the nonzero
pattern of the tableau and the per-evaluation counts of the right-hand side
and its vector-Jacobian product, and those from the formulas of Appendix A.
"""
import numpy as np
import pytest

import oracle as O
from paper_2609_02876_amd import flops as F

SYS = {O.LORENZ: "lorenz", O.VDP: "vdp", O.ROBERTSON: "robertson", O.HIRES: "hires",
       O.LINEAR: "linear", O.LV_UDE: "ude"}
METH = {O.TSIT5: "tsit5", O.VERN7: "vern7", O.RODAS: "rodas4", O.ROS23: "ros23"}
PAIRS = [(m, s) for (m, s) in [(O.TSIT5, O.LORENZ), (O.VERN7, O.LORENZ), (O.TSIT5, O.VDP),
                               (O.VERN7, O.VDP), (O.TSIT5, O.LINEAR), (O.VERN7, O.LINEAR),
                               (O.TSIT5, O.LV_UDE), (O.RODAS, O.ROBERTSON),
                               (O.RODAS, O.HIRES), (O.RODAS, O.LINEAR),
                               (O.ROS23, O.ROBERTSON), (O.ROS23, O.HIRES),
                               (O.ROS23, O.LINEAR)]]


@pytest.mark.parametrize("method,system", PAIRS)
def test_flops_table_equals_oracle_count(method, system):
    got = F.per_unit(METH[method], SYS[system])
    assert got == O.count_ops(method, system)


@pytest.mark.parametrize("system", list(SYS))
def test_system_counts_equal_oracle_count(system):
    assert F.SYSTEMS[SYS[system]][1:] == O.count_system(system)


def test_counter_on_the_printed_fields():
    # Lorenz: sigma (y1 - y0) is 2; fma(y0, rho - y2, -y1) 3; fma(y0, y1, -(beta y2)) 3
    assert O.count_system(O.LORENZ)[0] == 8
    # Van der Pol: f0 = y1 is free; mu * fma(fma(-y0, y0, 1), y1, -y0) is 5
    assert O.count_system(O.VDP)[0] == 5
    # damped rotation: -fma(a, y0, w y1) 3, fma(w, y0, -(a y1)) 3
    assert O.count_system(O.LINEAR)[0] == 6


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
@pytest.mark.parametrize("system", [O.LORENZ, O.VDP, O.LINEAR])
def test_explicit_counts_from_the_tableau_pattern(method, system):
    """Count by hand from the nonzero pattern: a combination of m terms is a
    product then m - 1 fmas (2m - 1), and a stage input or y_new adds
    fma(h, acc, y) (2)."""
    tb = O.erk_tableau(method)
    A, b, ew, s = tb["A"], tb["b"], tb["ew"], tb["s"]
    d, _ = O.dims(system)
    f, v = O.count_system(system)[:2]
    fsal = bool(np.all(A[s - 1, : s - 1] == b[: s - 1]) and b[s - 1] == 0)
    su = int(np.nonzero(b)[0].max()) + 1  # stages that enter y_new
    combo = lambda m: 2 * m + 1
    rows = [int(np.count_nonzero(A[i, :i])) for i in range(s)]
    stages_all = sum(combo(rows[i]) for i in range(1, s)) * d
    stages_su = sum(combo(rows[i]) for i in range(1, su)) * d
    update = combo(int(np.count_nonzero(b))) * d
    err = (2 * int(np.count_nonzero(ew)) - 1) * d + d + 3 * d + (d + 1 + 2 * (d - 1) + 1 + 1)
    trial = stages_all + (s - 1) * f + (0 if fsal else update) + err + 2 + 2
    c = O.count_ops(method, system)
    assert c["trial"] == trial
    assert c["accept"] == 1 + (0 if fsal else f)
    assert c["side_fwd"] == stages_su + (su - 1) * f + update
    # reverse: stage j's cotangent combines [b_j != 0] + #{l > j: a_lj != 0}
    # terms (a product then fmas, then the product by h: 2 terms + ... = 2t),
    # a VJP per stage and the addition of each stage's cotangent into lambda
    rev = 0
    for j in range(su):
        t = int(b[j] != 0) + sum(1 for l in range(j + 1, su) if A[l, j] != 0)
        rev += (2 * t if t else 1) * d
    adj = f + stages_su + (su - 1) * f + rev + su * v + su * d
    assert c["adj_step"] == adj
    assert c["adj_side"] == adj + update + 3 * d + d
    assert c["adj_zero"] == 3 * d + d
    # dense save: the two end slopes, then per component the four weighted
    # terms and their three additions plus the product by h (8); its reverse
    # adds the cotangent (3d), the two weighted cotangents (2d), two VJPs,
    # lo and hi (a product and an addition each: 4d) and their additions (2d)
    assert c["dense_fwd"] == 2 * f + 8 * d
    assert c["dense_adj"] == c["dense_fwd"] + 3 * d + 2 * d + 2 * v + 4 * d + 2 * d


def _structural_lu_count(P):
    """Hand count of the LU of a matrix with nonzero pattern P (diagonal
    included), no interchanges: per column a reciprocal, per row below with a
    nonzero in the column a multiplier and an fma (2) per nonzero right of
    the column in the pivot row (a product alone (1) where the row held a
    zero, which fills in); a solve is 2 per off-diagonal nonzero of L and U
    plus d products by the diagonal's reciprocals."""
    P = P.copy()
    d = len(P)
    fac = 0
    for k in range(d):
        fac += 1
        for i in range(k + 1, d):
            if not P[i, k]:
                continue
            fac += 1
            for j in range(k + 1, d):
                if P[k, j]:
                    fac += 2 if P[i, j] else 1
                    P[i, j] = True
    solve = 2 * int(np.tril(P, -1).sum() + np.triu(P, 1).sum()) + d
    return fac, solve


@pytest.mark.parametrize("system", [O.ROBERTSON, O.HIRES, O.LINEAR])
def test_lu_count_is_the_structural_count(system):
    """The counter leaves out the operations on W's structural zeros (the
    pattern taken from the oracle's Jacobian at a generic point, so from the
    formulas of Appendix A): its LU counts equal the hand count of the sparse
    factorisation, and no rows are interchanged at the counting point."""
    d, npar = O.dims(system)
    rng = np.random.default_rng(5)
    J = O.jac(system, rng.uniform(0.2, 1.0, d), rng.uniform(0.2, 1.0, npar))
    P = (J != 0) | np.eye(d, dtype=bool)
    fac, solve = _structural_lu_count(P)
    assert O.count_lu(system) == (fac, solve, solve, 0)


def test_hires_dense_lu_would_count_more():
    """The dense count for d = 8 (316 for the factorisation, 120 a solve)
    against the sparse one: the structural zeros are a large part of it."""
    dense_fac, dense_solve = _structural_lu_count(np.ones((8, 8), dtype=bool))
    assert (dense_fac, dense_solve) == (316, 120)
    fac, solve, _, _ = O.count_lu(O.HIRES)
    assert fac < dense_fac // 4 and solve < dense_solve // 2


def test_declared_jacobian_patterns_cover_the_jacobian():
    """The device systems declare their Jacobian's pattern (JAC_ROWS), from
    which the factorisation's skipped operations are found at compile time:
    every entry that the oracle's Jacobian makes nonzero at random points
    must be declared (a declared zero that is not one would drop a term)."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2609_02876_amd", "csrc",
                            "systems.h")).read()
    rng = np.random.default_rng(6)
    for name, system in (("Robertson", O.ROBERTSON), ("Hires", O.HIRES)):
        body = src[src.index(f"struct {name} {{"):]
        rows = re.search(r"JAC_ROWS\[\d+\] = \{([^}]*)\}", body).group(1)
        rows = [int(v.strip().rstrip("u"), 16) for v in rows.split(",")]
        d, npar = O.dims(system)
        seen = np.zeros((d, d), dtype=bool)
        for _ in range(20):
            seen |= O.jac(system, rng.uniform(0.1, 2.0, d), rng.uniform(0.1, 2.0, npar)) != 0
        declared = np.array([[(rows[i] >> j) & 1 for j in range(d)] for i in range(d)], bool)
        assert np.all(declared | ~seen), name
        assert np.array_equal(declared, seen), name  # and no more than that
