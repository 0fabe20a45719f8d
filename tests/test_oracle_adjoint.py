"""Pins for the oracle's discrete adjoint (paper, Section 3.1 and App. B.6).

The gradient target is d L(Psi(theta, y0; sg[h])) / d(theta, y0): the exact
derivative of the replay with the mesh frozen.  It is pinned by
  * P3: the closed form of the linear system's replay, differentiated by a
        complex step on prod_i R(h_i A) (no stage loop involved);
  * P5: central finite differences on the frozen mesh (relative step 1e-6,
        seeded unit direction, seed 0 -- the paper's protocol) and complex
        steps through the templated replay;
  * P6: forward-mode dual numbers, which agree with reverse mode to ~1e-13
        (the paper reports 1e-13 for its forward placements);
  * P8: brute force on a tiny ensemble: an independent torch float64 autograd
        replay (code written in this file) against the hand-written sweep.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from oracle_helpers import (lorenz_params, make_mesh, rot_matrix, stability_coeffs,
                            stability_matrix)

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
LOR_SAVE = [0.5 * s for s in range(1, 21)]


def _lorenz_case(n=8, t1=1.0, save_t=None, method=O.TSIT5, seed=0):
    y0 = np.tile([1.0, 0.0, 0.0], (n, 1))
    prm = lorenz_params(n, seed)
    rec = O.record(O.LORENZ, method, y0, prm, 0.0, t1, 1e-6, 1e-8, save_t=save_t)
    assert np.all(rec["status"] == O.ST_OK)
    return y0, prm, rec


def _loss(system, method, y0, prm, mesh):
    return np.sum(O.replay(system, method, y0, prm, mesh) ** 2, axis=(1, 2))


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
def test_closed_form_gradient_linear(method):
    g = stability_coeffs(method)
    rng = np.random.default_rng(1)
    n = 4
    prm = np.stack([0.05 + 0.3 * rng.random(n), 0.5 + 2 * rng.random(n)], 1)
    y0 = rng.normal(size=(n, 2))
    st = np.linspace(1.0, 6.0, 6)
    rec = O.record(O.LINEAR, method, y0, prm, 0.0, 6.0, 1e-7, 1e-9, save_t=st)
    gp, gy, ll = O.adjoint(O.LINEAR, method, y0, prm, rec)

    def loss_cf(a, w, y):
        A = rot_matrix(a, w)
        states = [y]
        for i in range(rec["S"][l]):
            states.append(stability_matrix(g, rec["h"][l, i] * A) @ states[-1])
        tot = 0
        for s in range(len(st)):
            v = stability_matrix(g, rec["save_dt"][l, s] * A) @ states[rec["save_idx"][l, s]]
            tot = tot + v @ v
        return tot

    e = 1e-30
    for l in range(n):
        a, w = prm[l]
        y = y0[l].astype(complex)
        da = loss_cf(a + 1j * e, w, y).imag / e
        dw = loss_cf(a, w + 1j * e, y).imag / e
        dy = [loss_cf(a, w, y + 1j * e * np.eye(2)[c]).imag / e for c in range(2)]
        # d/dw of |y|^2 is a pure discretisation effect (~1e-8): compare
        # componentwise against the size of the whole gradient
        ref = np.array([da, dw, *dy])
        got = np.concatenate([gp[l], gy[l]])
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), (got, ref)
        assert np.isclose(ll[l], loss_cf(a, w, y).real, rtol=1e-13)


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
@pytest.mark.parametrize("t1,save", [(1.0, None), (10.0, LOR_SAVE)])
def test_finite_differences_frozen_mesh(method, t1, save):
    y0, prm, rec = _lorenz_case(n=4, t1=t1, save_t=save, method=method)
    gp, gy, _ = O.adjoint(O.LORENZ, method, y0, prm, rec)
    rng = np.random.default_rng(0)
    rel = GOLD["fd_check"]["relative_step"]
    for l in range(4):
        v = rng.normal(size=3); v /= np.linalg.norm(v)
        eps = rel * np.linalg.norm(prm[l])
        sl = slice(l, l + 1)
        m = {k: rec[k][sl] for k in ("h", "S", "save_idx", "save_dt")}
        lp = _loss(O.LORENZ, method, y0[sl], prm[sl] + eps * v, m)[0]
        lm = _loss(O.LORENZ, method, y0[sl], prm[sl] - eps * v, m)[0]
        fd = (lp - lm) / (2 * eps)
        ad = gp[l] @ v
        # central differences resolve the chaotic t in [0, 10] case less well
        tol = 1e-8 if t1 == 1.0 else 2e-6
        assert abs(fd - ad) <= tol * np.linalg.norm(gp[l]), (fd, ad)


@pytest.mark.parametrize("system,method", [(O.LORENZ, O.TSIT5), (O.LORENZ, O.VERN7),
                                           (O.VDP, O.TSIT5), (O.VDP, O.VERN7)])
def test_complex_step_and_dual_match_adjoint(system, method):
    n = 6
    rng = np.random.default_rng(2)
    if system == O.LORENZ:
        y0 = np.tile([1.0, 0.0, 0.0], (n, 1)); prm = lorenz_params(n, 2)
        t1, st = 10.0, LOR_SAVE
    else:
        y0 = np.tile([2.0, 0.0], (n, 1)); prm = 0.5 + 1.5 * rng.random((n, 1))
        t1 = 6.3; st = [6.3 * s / 20 for s in range(1, 20)] + [6.3]
    d, npar = O.dims(system)
    rec = O.record(system, method, y0, prm, 0.0, t1, 1e-6, 1e-8, save_t=st)
    gp, gy, ll = O.adjoint(system, method, y0, prm, rec)
    for k in range(npar + d):
        dp = np.zeros_like(prm); dy = np.zeros_like(y0)
        if k < npar:
            dp[:, k] = 1.0
        else:
            dy[:, k - npar] = 1.0
        ref = gp[:, k] if k < npar else gy[:, k - npar]
        ys, dys = O.replay_dual(system, method, y0, prm, dy, dp, rec)
        fwd = np.sum(2 * ys * dys, axis=(1, 2))
        assert np.allclose(fwd, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
        re, im = O.replay_complex(system, method, y0, prm, dy, dp, 1e-30, rec)
        cs = np.sum(2 * re * (im / 1e-30), axis=(1, 2))
        assert np.allclose(cs, ref, rtol=1e-12, atol=1e-13 * np.max(np.abs(ref)))
        assert np.allclose(np.sum(ys ** 2, axis=(1, 2)), ll, rtol=1e-14)


# ------------------------------------------------------- P8: brute force --
def _torch_tsit5_replay(tb, y0, prm, h, S, sidx, sdt):
    """Independent float64 autograd replay of one lane (torch, CPU)."""
    A = torch.tensor(tb["A"]); b = torch.tensor(tb["b"])
    s = tb["s"]

    def f(y):
        sg, rho, beta = prm[0], prm[1], prm[2]
        return torch.stack([sg * (y[1] - y[0]), y[0] * (rho - y[2]) - y[1], y[0] * y[1] - beta * y[2]])

    def step(y, hh):
        ks = []
        for i in range(s):
            Y = y + hh * sum((A[i, j] * ks[j] for j in range(i)), torch.zeros(3, dtype=torch.float64))
            ks.append(f(Y))
        return y + hh * sum(b[j] * ks[j] for j in range(s))

    states = [y0]
    for i in range(S):
        states.append(step(states[-1], float(h[i])))
    return torch.stack([step(states[sidx[k]], float(sdt[k])) for k in range(len(sidx))])


@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
def test_brute_force_torch_autograd(method):
    tb = O.erk_tableau(method)
    y0, prm, rec = _lorenz_case(n=3, t1=0.6, save_t=[0.2, 0.45, 0.6], method=method, seed=5)
    assert rec["S"].max() <= 50
    gp, gy, ll = O.adjoint(O.LORENZ, method, y0, prm, rec)
    for l in range(3):
        yt = torch.tensor(y0[l], requires_grad=True)
        pt = torch.tensor(prm[l], requires_grad=True)
        out = _torch_tsit5_replay(tb, yt, pt, rec["h"][l], rec["S"][l], rec["save_idx"][l],
                                  rec["save_dt"][l])
        L = (out ** 2).sum()
        L.backward()
        assert np.allclose(gp[l], pt.grad.numpy(), rtol=1e-12, atol=0)
        assert np.allclose(gy[l], yt.grad.numpy(), rtol=1e-12, atol=1e-12 * np.abs(gy[l]).max())
        assert np.isclose(ll[l], L.item(), rtol=1e-13)


def test_loss_kinds_consistent():
    y0, prm, rec = _lorenz_case(n=8, t1=2.0, save_t=[0.5, 1.0, 2.0])
    gp, gy, ll = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec)
    ys = O.replay(O.LORENZ, O.TSIT5, y0, prm, rec)
    # cotangent 2 y reproduces the sum-of-squares gradient
    gp2, gy2, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec, O.LOSS_COTANGENT, 2 * ys)
    assert np.array_equal(gp, gp2) and np.array_equal(gy, gy2)
    # MSE against a zero target with scale c is c times the sum of squares
    gp3, gy3, ll3 = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec, O.LOSS_MSE_TARGET,
                              np.zeros_like(ys), 0.25)
    assert np.allclose(gp3, 0.25 * gp, rtol=1e-15) and np.allclose(ll3, 0.25 * ll, rtol=1e-15)
    # a target shift moves the MSE gradient by the cotangent of the shift
    tgt = ys + 0.1
    gp4, _, ll4 = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec, O.LOSS_MSE_TARGET, tgt)
    assert np.allclose(ll4, 0.01 * ys.shape[1] * ys.shape[2], rtol=1e-10)
    gp5, _, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, prm, rec, O.LOSS_COTANGENT, -0.2 * np.ones_like(ys))
    assert np.allclose(gp4, gp5, rtol=1e-9, atol=1e-9 * np.abs(gp5).max())
