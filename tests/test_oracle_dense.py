"""Pins for the oracle's dense output: save states from the continuous
extension of the accepted step (the cubic Hermite interpolant of the step's
end states and slopes) and their discrete adjoint.

* the interpolant takes the step's end states exactly (theta = 0 and 1);
* on a uniform mesh its error against the exact solution of the damped
  rotation (the matrix exponential) falls like h^4 at the step midpoints
  (the local order of a cubic Hermite interpolant; the steps themselves are
  of order 5, so the interpolant's error dominates);
* the adaptive mesh's dense states are within the record's tolerance of the
  exact solution, and agree with the extra-step save states to the same
  order;
* the hand-written adjoint of the dense loss equals dual numbers, complex
  steps and central differences on the frozen mesh, and an independent torch
  autograd replay written here.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle as O
from oracle_helpers import make_mesh, rot_matrix
from paper_2609_02876_amd import workloads as W


def _uniform_mesh(n_steps, t1, save_t):
    return make_mesh([[t1 / n_steps] * n_steps], save_t, 0.0, t1)


def test_end_states_exactly():
    y0, p = W.lorenz(2, seed=3)
    rec = O.record(O.LORENZ, O.TSIT5, y0, p, 0.0, 1.0, 1e-6, 1e-8)
    l = 0
    S = int(rec["S"][l])
    # states at the mesh points, then saves placed on them with theta = 0
    # (save_idx i, offset 0) and theta = 1 (save_idx i - 1, offset h_{i-1})
    pts = [1, 5, S - 1]
    m = dict(h=rec["h"][l:l + 1], S=rec["S"][l:l + 1],
             save_idx=np.array([pts], np.int32), save_dt=np.zeros((1, len(pts))))
    at0 = O.replay(O.LORENZ, O.TSIT5, y0[:1], p[:1], m, dense=True)
    ref = O.replay(O.LORENZ, O.TSIT5, y0[:1], p[:1], m)          # a step of size 0
    assert np.array_equal(at0, ref)
    m1 = dict(m, save_idx=np.array([[i - 1 for i in pts]], np.int32),
              save_dt=np.array([[rec["h"][l, i - 1] for i in pts]]))
    at1 = O.replay(O.LORENZ, O.TSIT5, y0[:1], p[:1], m1, dense=True)
    assert np.array_equal(at1, ref)


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7, O.RODAS])
def test_interpolation_order_four(method):
    a, w = 0.3, 1.7
    p = np.array([[a, w]])
    y0 = np.array([[1.0, 0.5]])
    t1 = 2.0
    errs = []
    for n_steps in (8, 16, 32):
        h = t1 / n_steps
        mids = [(k + 0.5) * h for k in range(n_steps)]
        m = _uniform_mesh(n_steps, t1, mids)
        ys = O.replay(O.LINEAR, method, y0, p, m, dense=True)[0]
        ex = np.array([scipy.linalg.expm(t * rot_matrix(a, w)) @ y0[0] for t in mids])
        errs.append(np.max(np.linalg.norm(ys - ex, axis=1)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.0 < r1 < 18.5 and 14.0 < r2 < 18.5, (errs, r1, r2)


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7, O.RODAS, O.ROS23])
def test_adaptive_dense_states_within_tolerance(method):
    a, w = 0.2, 1.3
    p = np.tile([a, w], (4, 1))
    y0 = np.random.default_rng(4).normal(size=(4, 2))
    st = list(np.linspace(0.3, 8.0, 17))
    rec = O.record(O.LINEAR, method, y0, p, 0.0, 8.0, 1e-7, 1e-9, save_t=st)
    dense = O.replay(O.LINEAR, method, y0, p, rec, dense=True)
    ex = np.array([[scipy.linalg.expm(t * rot_matrix(a, w)) @ y0[l] for t in st]
                   for l in range(4)])
    scale = np.max(np.abs(ex))
    # the interpolant is of order 3 whatever the method, so its error depends
    # on how long the method's steps are: measured at rtol 1e-7, 1.7e-6
    # (Tsit5, ~69 steps), 8.8e-5 (Vern7, 25 steps), 3.4e-8 (Rodas4, ~195
    # steps), 1.2e-5 (Rosenbrock23, ~1100 steps, its own error)
    bound = {O.TSIT5: 5e-6, O.VERN7: 3e-4, O.RODAS: 2e-7, O.ROS23: 5e-5}[method]
    assert np.max(np.abs(dense - ex)) <= bound * scale
    # and the extra-step save states, of the method's own order, are closer
    assert np.max(np.abs(rec["y_save"] - ex)) <= np.max(np.abs(dense - ex)) + 1e-9 * scale


@pytest.mark.parametrize("system,method", [(O.LORENZ, O.TSIT5), (O.LORENZ, O.VERN7),
                                           (O.VDP, O.TSIT5), (O.ROBERTSON, O.RODAS),
                                           (O.ROBERTSON, O.ROS23)])
def test_dense_adjoint_matches_duals_and_complex_steps(system, method):
    n = 4
    if system == O.LORENZ:
        y0, p = W.lorenz(n, seed=7); t1 = 10.0
    elif system == O.VDP:
        y0, p = W.vdp(n, seed=7); t1 = 6.3
    else:
        y0, p = W.robertson(n, seed=7); t1 = 1e3
    st = list(W.save_times(0.0, t1, 20))
    rtol, atol = (1e-6, 1e-10) if system == O.ROBERTSON else (1e-6, 1e-8)
    rec = O.record(system, method, y0, p, 0.0, t1, rtol, atol, save_t=st)
    gp, gy, ll = O.adjoint(system, method, y0, p, rec, dense=True)
    d, npar = O.dims(system)
    ys = O.replay(system, method, y0, p, rec, dense=True)
    assert np.allclose(np.sum(ys ** 2, axis=(1, 2)), ll, rtol=1e-14)
    for k in range(npar + d):
        dp = np.zeros_like(p); dy = np.zeros_like(y0)
        if k < npar:
            dp[:, k] = 1.0
        else:
            dy[:, k - npar] = 1.0
        ref = gp[:, k] if k < npar else gy[:, k - npar]
        yv, dys = O.replay_dual(system, method, y0, p, dy, dp, rec, dense=True)
        fwd = np.sum(2 * yv * dys, axis=(1, 2))
        assert np.allclose(fwd, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
        re, im = O.replay_complex(system, method, y0, p, dy, dp, 1e-30, rec, dense=True)
        cs = np.sum(2 * re * (im / 1e-30), axis=(1, 2))
        assert np.allclose(cs, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))


def test_dense_adjoint_central_differences_frozen_mesh():
    y0, p = W.lorenz(3, seed=8)
    st = list(W.save_times(0.0, 2.0, 20))
    rec = O.record(O.LORENZ, O.TSIT5, y0, p, 0.0, 2.0, 1e-6, 1e-8, save_t=st)
    gp, _, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, p, rec, dense=True)
    rng = np.random.default_rng(0)
    for l in range(3):
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        eps = 1e-6 * np.linalg.norm(p[l])
        sl = slice(l, l + 1)
        m = {k: rec[k][sl] for k in ("h", "S", "save_idx", "save_dt")}
        f = lambda q: np.sum(O.replay(O.LORENZ, O.TSIT5, y0[sl], q, m, dense=True) ** 2)
        fd = (f(p[sl] + eps * v) - f(p[sl] - eps * v)) / (2 * eps)
        assert abs(fd - gp[l] @ v) <= 1e-8 * np.linalg.norm(gp[l])


def test_dense_adjoint_against_torch_autograd():
    """Independent: torch float64 autograd of a Tsit5 replay with the Hermite
    interpolant written here (natural order, no fma)."""
    tb = O.erk_tableau(O.TSIT5)
    A, b, s = tb["A"], tb["b"], tb["s"]
    y0, p = W.lorenz(2, seed=9)
    st = [0.13, 0.37, 0.5, 0.71, 1.0]
    rec = O.record(O.LORENZ, O.TSIT5, y0, p, 0.0, 1.0, 1e-6, 1e-8, save_t=st)
    gp, gy, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, p, rec, dense=True)
    for l in range(2):
        yt = torch.tensor(y0[l], requires_grad=True)
        pt = torch.tensor(p[l], requires_grad=True)
        f = lambda y: torch.stack([pt[0] * (y[1] - y[0]), y[0] * (pt[1] - y[2]) - y[1],
                                   y[0] * y[1] - pt[2] * y[2]])

        def step(y, h):
            ks = []
            for i in range(s):
                acc = torch.zeros(3, dtype=torch.float64)
                for j in range(i):
                    acc = acc + float(A[i, j]) * ks[j]
                ks.append(f(y + h * acc))
            return y + h * sum(float(b[j]) * ks[j] for j in range(s))

        S = int(rec["S"][l])
        states = [yt]
        for i in range(S):
            states.append(step(states[-1], float(rec["h"][l, i])))
        L = 0
        for k in range(len(st)):
            i = int(rec["save_idx"][l, k])
            if i == S:
                v = states[S]
            else:
                h = float(rec["h"][l, i]); th = float(rec["save_dt"][l, k]) / h
                a0 = (1 - th) ** 2 * (1 + 2 * th); a1 = th ** 2 * (3 - 2 * th)
                c0 = th * (1 - th) ** 2; c1 = -th ** 2 * (1 - th)
                v = (a0 * states[i] + a1 * states[i + 1]
                     + h * (c0 * f(states[i]) + c1 * f(states[i + 1])))
            L = L + (v ** 2).sum()
        L.backward()
        assert np.allclose(gp[l], pt.grad.numpy(), rtol=1e-12, atol=0)
        assert np.allclose(gy[l], yt.grad.numpy(), rtol=1e-12, atol=1e-12 * np.abs(gy[l]).max())
