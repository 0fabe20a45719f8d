"""Pins for the oracle's right-hand sides and their vector-Jacobian products.

The right-hand sides (paper, Appendix A) are pinned by facts of the
mathematics, not by retyping them: equilibria, the constant divergence of the
Lorenz flow, its (x, y) -> (-x, -y) symmetry, the linearisation of Van der Pol
at the origin, and the damped rotation's eigen-structure.  The VJPs are pinned
against central differences of the right-hand side itself.
"""
import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(0)


def _jac_fd(system, y, p, wrt="y", eps=1e-6):
    y = np.array(y, float); p = np.array(p, float)
    x = y if wrt == "y" else p
    cols = []
    for i in range(len(x)):
        e = np.zeros_like(x); e[i] = eps * max(1.0, abs(x[i]))
        if wrt == "y":
            fp, fm = O.rhs(system, y + e, p), O.rhs(system, y - e, p)
        else:
            fp, fm = O.rhs(system, y, p + e), O.rhs(system, y, p - e)
        cols.append((fp - fm) / (2 * e[i]))
    return np.stack(cols, 1)


def _jac_from_vjp(system, y, p):
    d, npar = O.dims(system)
    Jy = np.zeros((d, d)); Jp = np.zeros((d, npar))
    for r in range(d):
        w = np.zeros(d); w[r] = 1.0
        gy, gp = O.vjp(system, y, p, w)
        Jy[r] = gy; Jp[r] = gp
    return Jy, Jp


def test_lorenz_equilibria_divergence_symmetry():
    for _ in range(5):
        s, r, b = 9 + 2 * RNG.random(), 1.5 + 30 * RNG.random(), 2.5 + 0.5 * RNG.random()
        p = [s, r, b]
        q = np.sqrt(b * (r - 1))
        for eq in ([0, 0, 0], [q, q, r - 1], [-q, -q, r - 1]):
            assert np.max(np.abs(O.rhs(O.LORENZ, eq, p))) < 1e-12 * (1 + r)
        y = RNG.normal(size=3) * 5
        Jy, _ = _jac_from_vjp(O.LORENZ, y, p)
        assert abs(np.trace(Jy) + (s + 1 + b)) < 1e-12
        f = O.rhs(O.LORENZ, y, p)
        fm = O.rhs(O.LORENZ, [-y[0], -y[1], y[2]], p)
        assert np.allclose(fm, [-f[0], -f[1], f[2]], rtol=0, atol=1e-12)


def test_vdp_linearisation_and_axis():
    for mu in (0.5, 1.3, 2.0):
        Jy, Jp = _jac_from_vjp(O.VDP, [0.0, 0.0], [mu])
        assert np.allclose(Jy, [[0, 1], [-mu, mu]], atol=0)
        # on the x axis the velocity vanishes and the acceleration is -mu x
        for x in (-2.0, 0.7, 3.0):
            assert np.allclose(O.rhs(O.VDP, [x, 0.0], [mu]), [0.0, -mu * x])
        # a limit-cycle fact: divergence mu (1 - x^2)
        y = RNG.normal(size=2)
        Jy, _ = _jac_from_vjp(O.VDP, y, [mu])
        assert abs(np.trace(Jy) - mu * (1 - y[0] ** 2)) < 1e-12


def test_linear_rotation_eigen():
    a, w = 0.3, 1.7
    Jy, _ = _jac_from_vjp(O.LINEAR, [0.2, -0.4], [a, w])
    ev = np.linalg.eigvals(Jy)
    assert np.allclose(sorted(ev, key=lambda z: z.imag), [complex(-a, -w), complex(-a, w)])
    # f is linear: f(y) = J y
    y = RNG.normal(size=2)
    assert np.allclose(O.rhs(O.LINEAR, y, [a, w]), Jy @ y, atol=1e-14)


@pytest.mark.parametrize("system,ymk,pmk", [
    (O.LORENZ, lambda: RNG.normal(size=3) * 4, lambda: [9 + 2 * RNG.random(), 27 + 2 * RNG.random(), 2.5 + 0.5 * RNG.random()]),
    (O.VDP, lambda: RNG.normal(size=2) * 2, lambda: [0.5 + 1.5 * RNG.random()]),
    (O.LINEAR, lambda: RNG.normal(size=2), lambda: [RNG.random(), 2 * RNG.random()]),
])
def test_vjp_matches_finite_differences(system, ymk, pmk):
    for _ in range(5):
        y, p = ymk(), pmk()
        Jy, Jp = _jac_from_vjp(system, y, p)
        Jy_fd = _jac_fd(system, y, p, "y")
        Jp_fd = _jac_fd(system, y, p, "p")
        sc = 1 + np.max(np.abs(Jy_fd))
        assert np.max(np.abs(Jy - Jy_fd)) < 1e-7 * sc
        assert np.max(np.abs(Jp - Jp_fd)) < 1e-7 * (1 + np.max(np.abs(Jp_fd)))
        # vjp accumulates into gp
        w = RNG.normal(size=len(y))
        gy, gp = O.vjp(system, y, p, w)
        assert np.allclose(gy, Jy.T @ w, rtol=1e-13, atol=1e-13)
        assert np.allclose(gp, Jp.T @ w, rtol=1e-13, atol=1e-13)
