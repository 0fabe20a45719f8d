"""Pins for the oracle's Rosenbrock path (Rodas4; paper Section 3.2 and
Appendix A: Robertson, HIRES).

* the tableau satisfies the Rosenbrock order conditions (order 4, embedded 3),
  evaluated on rooted trees after undoing the transformed form;
* Jacobians, VJPs and Jacobian-VJPs against finite differences; the linear
  invariants of Robertson (sum of species) and HIRES (y7 + y8);
* convergence order 4 and the matrix exponential on the damped rotation;
* mass conservation along Robertson solutions and the adjoint consequences
  of the invariants (zero parameter gradient, unit initial-state gradient);
* forward-mode duals and complex steps against the reverse sweep (these
  differentiate the LU factorisation and J itself, so they pin the transposed
  solves and the d(J)/d(y, p) terms);
* central differences on the frozen mesh and an independent tight scipy
  Radau sensitivity (Table gradacc protocol).
"""
from functools import lru_cache

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle as O
from paper_2609_02876_amd import workloads as W
from oracle_helpers import make_mesh, rot_matrix
from test_oracle_tableaux import _gamma, _trees

mp.mp.dps = 40
HIRES_THETA = np.array(W.HIRES_THETA)
HIRES_Y0 = np.array(W.HIRES_Y0)
_robertson = W.robertson
_hires = W.hires


# ------------------------------------------------------------- tableau ---
def _ros_weights():
    tb = O.ros_tableau()
    s = tb["s"]
    M = mp.mpf
    A = mp.matrix([[M(float(x)) for x in row] for row in tb["a"]])
    Cc = mp.matrix([[M(float(x)) for x in row] for row in tb["c"]])
    g = M(float(tb["gamma"]))
    Ginv = mp.eye(s) / g - Cc          # transformed form: C = diag(1/g) - Gamma^{-1}
    G = Ginv ** -1
    alpha = A * G
    beta = alpha + G                   # includes the diagonal gamma
    m = [M(float(x)) for x in tb["m"]]
    mh = [M(float(x)) for x in tb["a"][s - 1]]  # embedded: the last stage input
    b = [mp.fsum(m[i] * G[i, j] for i in range(s)) for j in range(s)]
    bh = [mp.fsum(mh[i] * G[i, j] for i in range(s)) for j in range(s)]
    return tb, s, alpha, beta, b, bh


def _phi_ros(t, alpha, beta, s):
    """Elementary weights of a Rosenbrock method (Hairer & Wanner II, IV.7):
    a node with one child multiplies by beta (J times the child), a node with
    several children by alpha (f'' on the children)."""
    if len(t) == 0:
        return [mp.mpf(1)] * s
    if len(t) == 1:
        c = _phi_ros(t[0], alpha, beta, s)
        return [mp.fsum(beta[j, k] * c[k] for k in range(s)) for j in range(s)]
    v = [mp.mpf(1)] * s
    for ch in t:
        c = _phi_ros(ch, alpha, beta, s)
        w = [mp.fsum(alpha[j, k] * c[k] for k in range(s)) for j in range(s)]
        v = [v[j] * w[j] for j in range(s)]
    return v


def _res(wts, order, alpha, beta, s):
    return [abs(mp.fsum(wts[j] * x for j, x in enumerate(_phi_ros(t, alpha, beta, s)))
                - mp.mpf(1) / _gamma(t))
            for o in range(1, order + 1) for t in _trees(o)]


def test_rodas4_order_conditions():
    tb, s, alpha, beta, b, bh = _ros_weights()
    assert tb["order"] == 4 and tb["q_emb"] == 3 and s == 6
    assert max(_res(b, 4, alpha, beta, s)) < 1e-14
    assert max(_res(b, 5, alpha, beta, s)) > 1e-6
    assert max(_res(bh, 3, alpha, beta, s)) < 1e-14
    assert max(_res(bh, 4, alpha, beta, s)) > 1e-6
    # the published nodes alpha_i = (0, 0.386, 0.21, 0.63, 1, 1)
    c = [float(mp.fsum(alpha[i, j] for j in range(s))) for i in range(s)]
    assert np.allclose(c, [0, 0.386, 0.21, 0.63, 1, 1], atol=1e-14)


# ------------------------------------------------------------- systems ---
def _fd_jac(system, y, p, eps=1e-3):
    # these fields are at most quadratic in y, so central differences are
    # exact up to rounding and a large step beats cancellation
    y = np.asarray(y, float)
    J = np.zeros((len(y), len(y)))
    for k in range(len(y)):
        e = np.zeros_like(y); e[k] = eps * max(1.0, abs(y[k]))
        J[:, k] = (O.rhs(system, y + e, p) - O.rhs(system, y - e, p)) / (2 * e[k])
    return J


@pytest.mark.parametrize("system", [O.ROBERTSON, O.HIRES, O.LINEAR])
def test_jacobian_vjp_and_jac_vjp(system):
    rng = np.random.default_rng(3)
    d, npar = O.dims(system)
    for _ in range(4):
        if system == O.ROBERTSON:
            y = rng.random(3) * [1, 1e-4, 1]; p = _robertson(1, rng.integers(99))[1][0]
        elif system == O.HIRES:
            y = rng.random(8); p = _hires(1, rng.integers(99))[1][0]
        else:
            y = rng.normal(size=2); p = rng.random(2)
        J = O.jac(system, y, p)
        Jfd = _fd_jac(system, y, p)
        assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-7 * np.abs(J).max())
        w = rng.normal(size=d)
        gy, gp = O.vjp(system, y, p, w)
        assert np.allclose(gy, J.T @ w, rtol=1e-12, atol=1e-12 * np.abs(J).max())
        # d/dp of f against FD
        for k in range(npar):
            e = np.zeros(npar); e[k] = 1e-2 * abs(p[k])   # f is linear in p
            fd = (O.rhs(system, y, p + e) - O.rhs(system, y, p - e)) / (2 * e[k])
            assert np.isclose(gp[k], fd @ w, rtol=1e-6, atol=1e-9 * (1 + np.abs(fd @ w)))
        # d/d(y, p) of u^T J v against FD of the Jacobian itself
        u, v = rng.normal(size=d), rng.normal(size=d)
        gyj, gpj = O.jac_vjp(system, y, p, u, v)
        for k in range(d):
            e = np.zeros(d); e[k] = 1e-2 * max(1.0, abs(y[k]))   # J is linear in y
            fd = (u @ O.jac(system, y + e, p) @ v - u @ O.jac(system, y - e, p) @ v) / (2 * e[k])
            assert np.isclose(gyj[k], fd, rtol=1e-6, atol=1e-8 * (1 + abs(fd)))
        for k in range(npar):
            e = np.zeros(npar); e[k] = 1e-2 * abs(p[k])   # and linear in p
            fd = (u @ O.jac(system, y, p + e) @ v - u @ O.jac(system, y, p - e) @ v) / (2 * e[k])
            assert np.isclose(gpj[k], fd, rtol=1e-6, atol=1e-8 * (1 + abs(fd)))


def test_linear_invariants_of_the_fields():
    rng = np.random.default_rng(4)
    for _ in range(10):
        y = rng.random(3); p = _robertson(1, rng.integers(99))[1][0]
        f = O.rhs(O.ROBERTSON, y, p)
        assert abs(f.sum()) <= 1e-15 * np.abs(f).max() * 8
        assert np.allclose(O.jac(O.ROBERTSON, y, p).sum(axis=0), 0, atol=1e-9 * p.max())
        yh = rng.random(8); ph = _hires(1, rng.integers(99))[1][0]
        fh = O.rhs(O.HIRES, yh, ph)
        assert fh[6] + fh[7] == 0.0


# ------------------------------------------------------------- replays ---
def test_convergence_order_four():
    a, w, T = 0.1, 1.0, 10.0
    y0 = np.array([[1.0, 0.5]])
    errs = []
    for n_steps in (160, 320):
        m = make_mesh([[T / n_steps] * n_steps], [T], 0.0, T)
        ys = O.replay(O.LINEAR, O.RODAS, y0, np.array([[a, w]]), m)[0, -1]
        errs.append(np.linalg.norm(ys - expm(rot_matrix(a, w) * T) @ y0[0]))
    assert abs(np.log2(errs[0] / errs[1]) - 4) < 0.25, errs


def test_adaptive_linear_vs_expm():
    rng = np.random.default_rng(5)
    n = 16
    prm = np.stack([0.05 + 0.3 * rng.random(n), 0.5 + 2 * rng.random(n)], 1)
    y0 = rng.normal(size=(n, 2))
    rec = O.record(O.LINEAR, O.RODAS, y0, prm, 0.0, 5.0, 1e-8, 1e-10)
    for l in range(n):
        ex = expm(rot_matrix(*prm[l]) * 5.0) @ y0[l]
        assert np.linalg.norm(rec["y_save"][l, 0] - ex) <= 1e-6 * np.linalg.norm(ex)


def test_robertson_mass_and_invariant_adjoint():
    n = 64
    y0, k = _robertson(n, 1)
    st = [1e-3, 1.0, 1e2, 1e4, 1e5]
    rec = O.record(O.ROBERTSON, O.RODAS, y0, k, 0.0, 1e5, 1e-6, 1e-10, save_t=st)
    assert np.all(rec["status"] == O.ST_OK)
    assert np.abs(rec["y_save"].sum(-1) - 1.0).max() < 1e-13
    # cotangent (1,1,1) at every save: the loss is the conserved mass, so its
    # parameter gradient vanishes and its y0-gradient is n_save * (1,1,1)
    gp, gy, _ = O.adjoint(O.ROBERTSON, O.RODAS, y0, k, rec, O.LOSS_COTANGENT,
                          np.ones((n, len(st), 3)))
    gref, _, _ = O.adjoint(O.ROBERTSON, O.RODAS, y0, k, rec)
    assert np.abs(gp / np.abs(gref).max(axis=1, keepdims=True)).max() < 1e-11
    assert np.abs(gy - len(st)).max() < 1e-11


def test_hires_invariant_and_adjoint():
    n = 16
    y0, th = _hires(n, 2)
    rec = O.record(O.HIRES, O.RODAS, y0, th, 0.0, 321.8122, 1e-6, 1e-10)
    assert np.all(rec["status"] == O.ST_OK)
    assert np.abs(rec["y_save"][:, 0, 6] + rec["y_save"][:, 0, 7] - 0.0057).max() < 1e-15
    e67 = np.zeros((n, 1, 8)); e67[..., 6] = e67[..., 7] = 1.0
    gp, gy, _ = O.adjoint(O.HIRES, O.RODAS, y0, th, rec, O.LOSS_COTANGENT, e67)
    gref, _, _ = O.adjoint(O.HIRES, O.RODAS, y0, th, rec)
    # some trajectories barely react to the rates (|grad| ~ 1e-8), so the
    # roundoff floor is measured against the ensemble's gradient scale
    assert np.abs(gp).max() < 1e-12 * np.abs(gref).max()
    assert np.allclose(gy[:, 6], 1.0, atol=1e-12) and np.allclose(gy[:, 7], 1.0, atol=1e-12)
    assert np.abs(gy[:, :6]).max() < 1e-12


@pytest.mark.parametrize("system", [O.ROBERTSON, O.HIRES])
def test_dual_and_complex_step_match_adjoint(system):
    n = 4
    if system == O.ROBERTSON:
        y0, p = _robertson(n, 6); t1, st = 100.0, [1.0, 10.0, 100.0]
    else:
        y0, p = _hires(n, 6); t1, st = 50.0, [5.0, 50.0]
    d, npar = O.dims(system)
    rec = O.record(system, O.RODAS, y0, p, 0.0, t1, 1e-7, 1e-10, save_t=st)
    gp, gy, _ = O.adjoint(system, O.RODAS, y0, p, rec)
    for k in range(npar + d):
        dp = np.zeros_like(p); dy = np.zeros_like(y0)
        if k < npar:
            dp[:, k] = p[:, k]        # relative direction: d/dlog(p_k)
            ref = gp[:, k] * p[:, k]
        else:
            dy[:, k - npar] = 1.0
            ref = gy[:, k - npar]
        ys, dys = O.replay_dual(system, O.RODAS, y0, p, dy, dp, rec)
        fwd = np.sum(2 * ys * dys, axis=(1, 2))
        scale = np.max(np.abs(np.concatenate([gp * p, gy], 1)), axis=1)
        assert np.all(np.abs(fwd - ref) <= 1e-11 * scale), (k, fwd, ref)
        re, im = O.replay_complex(system, O.RODAS, y0, p, dy, dp, 1e-30, rec)
        cs = np.sum(2 * re * (im / 1e-30), axis=(1, 2))
        assert np.all(np.abs(cs - ref) <= 1e-11 * scale), (k, cs, ref)


def test_frozen_mesh_finite_differences():
    n = 4
    y0, k = _robertson(n, 7)
    rec = O.record(O.ROBERTSON, O.RODAS, y0, k, 0.0, 1e4, 1e-6, 1e-10)
    gp, _, _ = O.adjoint(O.ROBERTSON, O.RODAS, y0, k, rec)
    rng = np.random.default_rng(0)
    for l in range(n):
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        dlog = 1e-6
        sl = slice(l, l + 1)
        m = {key: rec[key][sl] for key in ("h", "S", "save_idx", "save_dt")}
        kp = k[sl] * np.exp(dlog * v); km = k[sl] * np.exp(-dlog * v)
        lp = np.sum(O.replay(O.ROBERTSON, O.RODAS, y0[sl], kp, m) ** 2)
        lm = np.sum(O.replay(O.ROBERTSON, O.RODAS, y0[sl], km, m) ** 2)
        fd = (lp - lm) / (2 * dlog)
        ad = np.sum(gp[l] * k[l] * v)
        assert abs(fd - ad) <= 1e-6 * np.linalg.norm(gp[l] * k[l]), (fd, ad)


def test_independent_radau_sensitivity():
    n = 3
    y0, k = _robertson(n, 8)
    rec = O.record(O.ROBERTSON, O.RODAS, y0, k, 0.0, 1e3, 1e-9, 1e-13)
    gp, _, _ = O.adjoint(O.ROBERTSON, O.RODAS, y0, k, rec)

    def final_sq(kk):
        f = lambda t, y: [-kk[0] * y[0] + kk[2] * y[1] * y[2],
                          kk[0] * y[0] - kk[2] * y[1] * y[2] - kk[1] * y[1] ** 2,
                          kk[1] * y[1] ** 2]
        sol = solve_ivp(f, (0, 1e3), [1.0, 0, 0], method="Radau", rtol=1e-11, atol=1e-14)
        return float(np.sum(sol.y[:, -1] ** 2))

    for l in range(n):
        fd = []
        for j in range(3):
            e = np.zeros(3); e[j] = 1e-4 * k[l, j]
            fd.append((final_sq(k[l] + e) - final_sq(k[l] - e)) / (2 * e[j]) * k[l, j])
        fd = np.array(fd)
        assert np.linalg.norm(gp[l] * k[l] - fd) / np.linalg.norm(fd) < 1e-4
