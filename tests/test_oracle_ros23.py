"""Pins for the oracle's Rosenbrock23 (the paper's default stiff method for
fields in the fused kernels' form, Section 3.2; Shampine & Reichelt 1997).

The oracle writes the method in the transformed form it shares with Rodas4.
What fixes it independently of that form:

* the transformed coefficients against their exact values in d = 1/(2+sqrt 2)
  and e32 = 6 + sqrt 2, and, after undoing the transformation, the
  Rosenbrock order conditions on rooted trees: order 2 for y_new, order 3 for
  y_new plus the error estimate (the pair the controller's cube root assumes);
* one trial step against Shampine's original slope form (the ode23s
  formulas, written out here in numpy with an explicit Jacobian) on the
  damped rotation and on Robertson, for y_new and for the error estimate;
* L-stability (a very stiff linear step is damped to nothing), convergence
  order 2 on fixed meshes, the adaptive solve against exp(A t);
* Robertson mass conservation and the adjoint consequences of the invariant;
  forward-mode duals and complex steps against the reverse sweep (they
  differentiate the factorisation and J, so they pin the transposed solves
  and the d(J)/d(y, p) terms); central differences on the frozen mesh.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from paper_2609_02876_amd import workloads as W
from oracle_helpers import make_mesh, rot_matrix
from test_oracle_rosenbrock import _res

mp.mp.dps = 40


def _exact():
    s2 = mp.sqrt(2)
    d = 1 / (2 + s2)
    e32 = 6 + s2
    return d, e32


def test_ros23_coefficients_are_the_exact_numbers():
    tb = O.ros_tableau(O.ROS23)
    d, e32 = _exact()
    assert (tb["s"], tb["su"], tb["order"], tb["q_emb"]) == (3, 2, 2, 2)
    want = {
        "gamma": d,
        ("a", 1, 0): 1 / (2 * d), ("a", 2, 0): 1 / d, ("a", 2, 1): 1 / d,
        ("c", 1, 0): -1 / d, ("c", 2, 0): -2 / d, ("c", 2, 1): -e32 / d,
        ("m", 0): 1 / d, ("m", 1): 1 / d, ("m", 2): 0,
        ("e", 0): 1 / (6 * d), ("e", 1): (e32 - 2) / (6 * d), ("e", 2): 1 / (6 * d),
    }
    for key, v in want.items():
        got = tb["gamma"] if key == "gamma" else tb[key[0]][key[1:]]
        assert abs(got - float(v)) <= 0.5 * np.spacing(abs(float(v))) or got == float(v), key
    # nothing else is nonzero
    assert np.count_nonzero(tb["a"]) == 3 and np.count_nonzero(tb["c"]) == 3


def test_ros23_order_conditions():
    tb = O.ros_tableau(O.ROS23)
    s = tb["s"]
    M = mp.mpf
    A = mp.matrix([[M(float(x)) for x in r] for r in tb["a"]])
    Cc = mp.matrix([[M(float(x)) for x in r] for r in tb["c"]])
    G = (mp.eye(s) / M(float(tb["gamma"])) - Cc) ** -1   # Gamma (d on the diagonal)
    alpha = A * G
    beta = alpha + G
    m = [M(float(x)) for x in tb["m"]]
    e = [M(float(x)) for x in tb["e"]]
    b = [mp.fsum(m[i] * G[i, j] for i in range(s)) for j in range(s)]
    bh = [b[j] + mp.fsum(e[i] * G[i, j] for i in range(s)) for j in range(s)]
    # the standard-form coefficients of the published method
    d, e32 = _exact()
    assert abs(alpha[1, 0] - 0.5) < 1e-15 and abs(alpha[2, 1] - 1) < 1e-15
    assert abs(G[1, 0] + d) < 1e-15 and abs(G[2, 0] - (e32 - 2) * d) < 1e-15
    assert abs(G[2, 1] + e32 * d) < 1e-15
    assert np.allclose([float(x) for x in b], [0, 1, 0], atol=1e-15)
    assert np.allclose([float(x) for x in bh], [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    assert max(_res(b, 2, alpha, beta, s)) < 1e-15
    assert max(_res(b, 3, alpha, beta, s)) > 1e-3
    assert max(_res(bh, 3, alpha, beta, s)) < 1e-15
    assert max(_res(bh, 4, alpha, beta, s)) > 1e-3


# ------------------------------------------- Shampine's original form ---
def _ode23s_step(f, J, y, h):
    """One step of ode23s in slope form (Shampine & Reichelt 1997, Sec. 4)."""
    d = 1.0 / (2.0 + math.sqrt(2.0))
    e32 = 6.0 + math.sqrt(2.0)
    Wm = np.eye(len(y)) - h * d * J(y)
    F0 = f(y)
    k1 = np.linalg.solve(Wm, F0)
    F1 = f(y + 0.5 * h * k1)
    k2 = np.linalg.solve(Wm, F1 - k1) + k1
    ynew = y + h * k2
    F2 = f(ynew)
    k3 = np.linalg.solve(Wm, F2 - e32 * (k2 - F1) - 2.0 * (k1 - F0))
    return ynew, h / 6.0 * (k1 - 2.0 * k2 + k3)


def _robertson_fJ(k):
    k1, k2, k3 = k
    f = lambda y: np.array([-k1 * y[0] + k3 * y[1] * y[2],
                            k1 * y[0] - k3 * y[1] * y[2] - k2 * y[1] ** 2,
                            k2 * y[1] ** 2])
    J = lambda y: np.array([[-k1, k3 * y[2], k3 * y[1]],
                            [k1, -k3 * y[2] - 2 * k2 * y[1], -k3 * y[1]],
                            [0.0, 2 * k2 * y[1], 0.0]])
    return f, J


def test_ros23_step_equals_shampine_slope_form():
    rng = np.random.default_rng(11)
    # damped rotation, J = A exactly
    for _ in range(5):
        a, w = 0.05 + rng.random(), 0.5 + 3 * rng.random()
        A = rot_matrix(a, w)
        y = rng.normal(size=2)
        h = 10 ** rng.uniform(-3, 1)
        yn, e = O.ros_trial(O.ROS23, O.LINEAR, y, np.array([a, w]), h)
        yr, er = _ode23s_step(lambda v: A @ v, lambda v: A, y, h)
        assert np.linalg.norm(yn - yr) <= 1e-14 * np.linalg.norm(yr)
        assert np.linalg.norm(e - er) <= 1e-11 * np.linalg.norm(er) + 1e-16 * np.linalg.norm(y)
    # Robertson at stiff step sizes
    _, kk = W.robertson(4, 3)
    for l in range(4):
        f, J = _robertson_fJ(kk[l])
        y = np.array([0.9, 2e-5, 0.1])
        for h in (1e-4, 1e-2, 1.0, 1e2):
            yn, e = O.ros_trial(O.ROS23, O.ROBERTSON, y, kk[l], h)
            yr, er = _ode23s_step(f, J, y, h)
            assert np.allclose(yn, yr, rtol=1e-12, atol=1e-15), (h, yn, yr)
            assert np.allclose(e, er, rtol=1e-8, atol=1e-14), (h, e, er)


def test_ros23_l_stability():
    # y' = A y with eigenvalues -1e8 +- i: one step of size 1 is damped to
    # about |R(z)| ~ 1/|z|; an A-stable but not L-stable method would not be
    y = np.array([1.0, 0.5])
    yn, _ = O.ros_trial(O.ROS23, O.LINEAR, y, np.array([1e8, 1.0]), 1.0)
    assert np.linalg.norm(yn) < 1e-7 * np.linalg.norm(y)
    # and a mildly stiff step stays bounded by the exact decay factor's order
    yn, _ = O.ros_trial(O.ROS23, O.LINEAR, y, np.array([10.0, 1.0]), 1.0)
    assert np.linalg.norm(yn) < np.linalg.norm(y)


def test_ros23_convergence_order_two():
    a, w, T = 0.1, 1.0, 10.0
    y0 = np.array([[1.0, 0.5]])
    errs = []
    for n_steps in (400, 800, 1600):
        m = make_mesh([[T / n_steps] * n_steps], [T], 0.0, T)
        ys = O.replay(O.LINEAR, O.ROS23, y0, np.array([[a, w]]), m)[0, -1]
        errs.append(np.linalg.norm(ys - expm(rot_matrix(a, w) * T) @ y0[0]))
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(r - 2) < 0.1), (errs, r)


def test_ros23_adaptive_linear_vs_expm():
    # order 2 under a per-step bound on an O(h^3) local error estimate: the
    # global error is a few hundred local errors, and shrinks about like
    # rtol^(2/3) while the step count grows like rtol^(-1/3)
    rng = np.random.default_rng(5)
    n = 8
    prm = np.stack([0.05 + 0.3 * rng.random(n), 0.5 + 2 * rng.random(n)], 1)
    y0 = rng.normal(size=(n, 2))
    errs, steps = [], []
    for rtol in (1e-6, 1e-9):
        rec = O.record(O.LINEAR, O.ROS23, y0, prm, 0.0, 5.0, rtol, rtol * 1e-2, cap=20000)
        assert np.all(rec["status"] == O.ST_OK)
        e = [np.linalg.norm(rec["y_save"][l, 0] - expm(rot_matrix(*prm[l]) * 5.0) @ y0[l])
             / np.linalg.norm(y0[l]) for l in range(n)]
        errs.append(max(e))
        steps.append(rec["S"].mean())
        assert errs[-1] < 5 * rtol ** (2 / 3), (rtol, errs[-1])
    assert 5 < steps[1] / steps[0] < 20, steps
    assert 30 < errs[0] / errs[1] < 300, errs


def test_ros23_robertson_mass_and_invariant_adjoint():
    n = 32
    y0, k = W.robertson(n, 1)
    st = [1e-3, 1.0, 1e2, 1e4, 1e5]
    rec = O.record(O.ROBERTSON, O.ROS23, y0, k, 0.0, 1e5, 1e-6, 1e-10, save_t=st, cap=20000)
    assert np.all(rec["status"] == O.ST_OK)
    assert np.abs(rec["y_save"].sum(-1) - 1.0).max() < 1e-13
    gp, gy, _ = O.adjoint(O.ROBERTSON, O.ROS23, y0, k, rec, O.LOSS_COTANGENT,
                          np.ones((n, len(st), 3)))
    gref, _, _ = O.adjoint(O.ROBERTSON, O.ROS23, y0, k, rec)
    assert np.abs(gp / np.abs(gref).max(axis=1, keepdims=True)).max() < 1e-11
    assert np.abs(gy - len(st)).max() < 1e-11


@pytest.mark.parametrize("system", [O.ROBERTSON, O.HIRES])
def test_ros23_dual_and_complex_step_match_adjoint(system):
    n = 3
    if system == O.ROBERTSON:
        y0, p = W.robertson(n, 6); t1, st = 100.0, [1.0, 10.0, 100.0]
    else:
        y0, p = W.hires(n, 6); t1, st = 50.0, [5.0, 50.0]
    d, npar = O.dims(system)
    rec = O.record(system, O.ROS23, y0, p, 0.0, t1, 1e-6, 1e-10, save_t=st, cap=20000)
    assert np.all(rec["status"] == O.ST_OK)
    gp, gy, _ = O.adjoint(system, O.ROS23, y0, p, rec)
    scale = np.max(np.abs(np.concatenate([gp * p, gy], 1)), axis=1)
    for k in range(npar + d):
        dp = np.zeros_like(p); dy = np.zeros_like(y0)
        if k < npar:
            dp[:, k] = p[:, k]
            ref = gp[:, k] * p[:, k]
        else:
            dy[:, k - npar] = 1.0
            ref = gy[:, k - npar]
        ys, dys = O.replay_dual(system, O.ROS23, y0, p, dy, dp, rec)
        fwd = np.sum(2 * ys * dys, axis=(1, 2))
        assert np.all(np.abs(fwd - ref) <= 1e-11 * scale), (k, fwd, ref)
        re, im = O.replay_complex(system, O.ROS23, y0, p, dy, dp, 1e-30, rec)
        cs = np.sum(2 * re * (im / 1e-30), axis=(1, 2))
        assert np.all(np.abs(cs - ref) <= 1e-11 * scale), (k, cs, ref)


def test_ros23_frozen_mesh_finite_differences():
    n = 3
    y0, k = W.robertson(n, 7)
    rec = O.record(O.ROBERTSON, O.ROS23, y0, k, 0.0, 1e4, 1e-6, 1e-10, cap=20000)
    gp, _, _ = O.adjoint(O.ROBERTSON, O.ROS23, y0, k, rec)
    rng = np.random.default_rng(0)
    for l in range(n):
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        dlog = 1e-6
        sl = slice(l, l + 1)
        m = {key: rec[key][sl] for key in ("h", "S", "save_idx", "save_dt")}
        lp = np.sum(O.replay(O.ROBERTSON, O.ROS23, y0[sl], k[sl] * np.exp(dlog * v), m) ** 2)
        lm = np.sum(O.replay(O.ROBERTSON, O.ROS23, y0[sl], k[sl] * np.exp(-dlog * v), m) ** 2)
        fd = (lp - lm) / (2 * dlog)
        ad = np.sum(gp[l] * k[l] * v)
        assert abs(fd - ad) <= 1e-6 * np.linalg.norm(gp[l] * k[l]), (fd, ad)
