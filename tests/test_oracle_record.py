"""Pins for the oracle's adaptive record (paper, Section 2.1, Appendix A/B).

* P4: the adaptive solve of y' = A y against exp(A t), and the gradient of
  ||y(t1)||^2 against its closed form -2 t1 e^(-2 a t1) ||y0||^2, each within
  the solver's own error;
* the paper's linear family y' = 1.01 y takes the same step count on every
  trajectory (Table dispersion) and reaches y0 e^(1.01 t);
* P11 (soft): the step-count statistics of the paper's Lorenz dispersion
  ensemble (Table dispersion);
* P12: the replay gradient against central differences of an independent
  tight scipy DOP853 solve (Table gradacc protocol);
* per-lane failure statuses.
"""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle as O
from oracle_helpers import lorenz_params, rot_matrix

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


@pytest.mark.parametrize("method,rtol,tol", [(O.TSIT5, 1e-6, 1e-5), (O.TSIT5, 1e-9, 1e-8),
                                             (O.VERN7, 1e-6, 1e-5), (O.VERN7, 1e-10, 1e-9)])
def test_adaptive_vs_matrix_exponential(method, rtol, tol):
    rng = np.random.default_rng(4)
    n = 32
    prm = np.stack([0.05 + 0.3 * rng.random(n), 0.5 + 3 * rng.random(n)], 1)
    y0 = rng.normal(size=(n, 2))
    t1 = 5.0
    rec = O.record(O.LINEAR, method, y0, prm, 0.0, t1, rtol, rtol * 1e-2)
    gp, gy, _ = O.adjoint(O.LINEAR, method, y0, prm, rec)
    for l in range(n):
        a, w = prm[l]
        ex = expm(rot_matrix(a, w) * t1) @ y0[l]
        assert np.linalg.norm(rec["y_save"][l, 0] - ex) <= tol * np.linalg.norm(ex)
        ref_da = -2 * t1 * np.exp(-2 * a * t1) * (y0[l] @ y0[l])
        assert abs(gp[l, 0] - ref_da) <= 10 * tol * abs(ref_da)
        # exact d|y|^2/dw = 0 and d|y|^2/dy0 = 2 e^(-2 a t1) y0
        assert abs(gp[l, 1]) <= 10 * tol * abs(ref_da)
        assert np.allclose(gy[l], 2 * np.exp(-2 * a * t1) * y0[l], rtol=10 * tol)


def test_linear_family_equal_steps():
    g = GOLD["linear_family_equal_steps"]
    rng = np.random.default_rng(0)
    n = 64
    y0 = rng.random((n, 2))
    prm = np.tile([-g["rate"], 0.0], (n, 1))   # damped rotation with a = -1.01, w = 0
    rec = O.record(O.LINEAR, O.TSIT5, y0, prm, 0.0, g["t1"], 1e-6, 1e-9)
    assert np.all(rec["status"] == O.ST_OK)
    # the error norm is scale-relative, so every trajectory meets the same
    # sequence of decisions up to the absolute-tolerance floor
    assert rec["S"].max() - rec["S"].min() <= 1
    ex = y0 * np.exp(g["rate"] * g["t1"])
    assert np.max(np.abs(rec["y_save"][:, 0] / ex - 1)) < 1e-4


def test_dispersion_soft_pin():
    g = GOLD["dispersion_lorenz"]
    n = 2048
    rho = 21.0 * np.random.default_rng(0).random(n)
    prm = np.stack([np.full(n, 10.0), rho, np.full(n, 8.0 / 3.0)], 1)
    y0 = np.tile([1.0, 0.0, 0.0], (n, 1))
    rec = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 1e-6, 1e-9)
    S = rec["S"]
    mean, mx = S.mean(), S.max()
    ref = g["fused_recorder"]
    assert abs(mean / ref["mean"] - 1) < 0.15
    assert abs(mx / mean - ref["max_over_mean"]) < 0.1


def test_independent_sensitivity_scipy():
    g = GOLD["independent_sensitivity_lorenz"]
    n = 3
    prm = lorenz_params(n, seed=7)
    y0 = np.tile([1.0, 0.0, 0.0], (n, 1))
    rec = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 1e-8, 1e-10)
    gp, _, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec)

    def final_sq(p):
        f = lambda t, y: [p[0] * (y[1] - y[0]), y[0] * (p[1] - y[2]) - y[1], y[0] * y[1] - p[2] * y[2]]
        sol = solve_ivp(f, (0, 1), [1.0, 0, 0], method="DOP853", rtol=g["reference_rtol"],
                        atol=g["reference_atol"])
        return float(np.sum(sol.y[:, -1] ** 2))

    for l in range(n):
        fd = []
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-5 * prm[l, k]
            fd.append((final_sq(prm[l] + e) - final_sq(prm[l] - e)) / (2 * e[k]))
        fd = np.array(fd)
        assert np.linalg.norm(gp[l] - fd) / np.linalg.norm(fd) < 1e-5


def test_failure_statuses():
    y0 = np.tile([1.0, 0.0, 0.0], (4, 1))
    prm = lorenz_params(4)
    r = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 1e-6, 1e-8, max_steps=5)
    assert np.all(r["status"] == O.ST_MAX_STEPS) and np.all(r["n_trial"] == 5)
    r = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 1e-6, 1e-8, cap=8)
    assert np.all(r["status"] == O.ST_NOSPACE) and np.all(r["S"] == 8)
    bad = prm.copy(); bad[1, 1] = np.nan
    r = O.record(O.LORENZ, O.TSIT5, y0, bad, 0.0, 1.0, 1e-6, 1e-8)
    assert r["status"][1] == O.ST_NONFINITE and np.all(r["status"][[0, 2, 3]] == O.ST_OK)
    r = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 0.0, 1e-300)
    assert np.all(r["status"] == O.ST_DT_UNDERFLOW)
    # unreached save times stay NaN on a failed lane
    r = O.record(O.LORENZ, O.TSIT5, y0, prm, 0.0, 1.0, 1e-6, 1e-8, save_t=[0.5, 1.0], max_steps=5)
    assert np.all(np.isnan(r["y_save"][:, 1]))


def test_controller_root_is_accurate():
    """The controller's x^(-1/k) (frexp/ldexp + Newton) against 40 digits."""
    import mpmath as mp
    mp.mp.dps = 40
    rng = np.random.default_rng(0)
    xs = np.concatenate([np.exp(rng.uniform(-690, 690, 400)), [1.0, 0.5, 2.0, 1e-300, 1.7e300]])
    for k in (3, 4, 5, 6, 7, 8):
        for x in xs:
            r = O.root_inv(x, k)
            ref = float(mp.power(mp.mpf(float(x)), mp.mpf(-1) / k))
            assert abs(r - ref) <= 2 * np.spacing(ref), (x, k, r, ref)
    # below 1e-300 the argument is raised to 1e-300; 0 -> that bound, inf -> 0
    assert O.root_inv(0.0, 5) == O.root_inv(1e-300, 5)
    assert O.root_inv(np.inf, 5) == 0.0 and np.isnan(O.root_inv(np.nan, 5))
    assert np.isnan(O.root_inv(-1.0, 5))
    # only the roots the methods need are defined (k = 3: Rosenbrock23)
    assert np.isnan(O.root_inv(2.0, 2)) and np.isnan(O.root_inv(2.0, 9))
