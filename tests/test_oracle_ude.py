"""Pins for the oracle's universal differential equation (Lotka-Volterra plus a
2-32-32-2 tanh MLP with weights shared by all trajectories).

* with every MLP parameter zero the field is Lotka-Volterra exactly, and the
  solution keeps the Lotka-Volterra first integral;
* the MLP forward against torch's linear layers and tanh (library routines);
* the hand-written VJP against central differences of the field;
* the discrete adjoint against an independent float64 torch autograd replay
  on the same mesh, and against dual numbers through the oracle's replay.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import oracle as O
from paper_2609_02876_amd import workloads as W

ALPHA, BETA, GAMMA, DELTA = 1.5, 1.0, 3.0, 1.0


def _split(th):
    th = torch.as_tensor(th, dtype=torch.float64)
    W1 = th[0:64].reshape(32, 2); b1 = th[64:96]
    W2 = th[96:1120].reshape(32, 32); b2 = th[1120:1152]
    W3 = th[1152:1216].reshape(2, 32); b3 = th[1216:1218]
    return W1, b1, W2, b2, W3, b3


def _torch_field(y, th):
    W1, b1, W2, b2, W3, b3 = _split(th) if not isinstance(th, tuple) else th
    nn = Fn.linear(torch.tanh(Fn.linear(torch.tanh(Fn.linear(y, W1, b1)), W2, b2)), W3, b3)
    lv = torch.stack([ALPHA * y[0] - BETA * y[0] * y[1], DELTA * y[0] * y[1] - GAMMA * y[1]])
    return nn + lv


def _random_theta(seed):
    th = W.ude_weights(seed, scale=1.0)
    th[64:96] = np.random.default_rng(seed + 100).normal(0, 0.3, 32)      # nonzero biases
    th[1120:1152] = np.random.default_rng(seed + 101).normal(0, 0.3, 32)
    th[1216:1218] = np.random.default_rng(seed + 102).normal(0, 0.3, 2)
    return th


def test_zero_network_is_lotka_volterra():
    th = np.zeros(W.UDE_NP)
    rng = np.random.default_rng(0)
    for _ in range(20):
        x, y = rng.uniform(0.1, 3.0, 2)
        f = O.rhs(O.LV_UDE, [x, y], th)
        assert f[0] == ALPHA * x - BETA * (x * y)
        assert f[1] == DELTA * (x * y) - GAMMA * y


def test_lotka_volterra_first_integral_is_kept():
    """V = delta x - gamma ln x + beta y - alpha ln y is constant along solutions."""
    n = 16
    y0 = np.random.default_rng(1).uniform(0.5, 2.0, (n, 2))
    th = np.zeros(W.UDE_NP)
    st = list(np.arange(1, 21) * 0.5)
    rec = O.record(O.LV_UDE, O.TSIT5, y0, th, 0.0, 10.0, 1e-10, 1e-12, save_t=st,
                   params_shared=True)
    assert np.all(rec["status"] == O.ST_OK)
    V = lambda x, y: DELTA * x - GAMMA * np.log(x) + BETA * y - ALPHA * np.log(y)
    v0 = V(y0[:, 0], y0[:, 1])
    ys = rec["y_save"]
    vs = V(ys[..., 0], ys[..., 1])
    assert np.abs(vs - v0[:, None]).max() < 1e-8 * np.abs(v0).max()


def test_mlp_forward_against_torch_layers():
    rng = np.random.default_rng(2)
    for seed in range(4):
        th = _random_theta(seed)
        y = rng.uniform(0.2, 2.5, 2)
        f = O.rhs(O.LV_UDE, y, th)
        ref = _torch_field(torch.tensor(y), th).numpy()
        assert np.allclose(f, ref, rtol=1e-14, atol=1e-14)


def test_vjp_against_central_differences():
    rng = np.random.default_rng(3)
    for seed in range(3):
        th = _random_theta(seed)
        y = rng.uniform(0.2, 2.5, 2)
        w = rng.normal(size=2)
        gy, gp = O.vjp(O.LV_UDE, y, th, w)
        eps = 1e-6
        for k in range(2):
            e = np.zeros(2); e[k] = eps
            fd = (O.rhs(O.LV_UDE, y + e, th) - O.rhs(O.LV_UDE, y - e, th)) @ w / (2 * eps)
            assert abs(fd - gy[k]) < 1e-8 * max(1.0, abs(gy[k]))
        # a random direction in parameter space, and a few single coordinates
        dth = rng.normal(size=th.size)
        fd = (O.rhs(O.LV_UDE, y, th + eps * dth) - O.rhs(O.LV_UDE, y, th - eps * dth)) @ w / (2 * eps)
        assert abs(fd - gp @ dth) < 1e-7 * max(1.0, abs(gp @ dth))
        for i in (0, 70, 500, 1130, 1200, 1217):
            e = np.zeros(th.size); e[i] = eps
            fd = (O.rhs(O.LV_UDE, y, th + e) - O.rhs(O.LV_UDE, y, th - e)) @ w / (2 * eps)
            assert abs(fd - gp[i]) < 1e-8 * max(1.0, abs(gp[i]))


def _torch_replay(tb, y0, th, h, S, sidx, sdt):
    A = torch.tensor(tb["A"]); b = torch.tensor(tb["b"]); s = tb["s"]
    parts = _split(th) if not isinstance(th, torch.Tensor) else None

    def f(y):
        return _torch_field(y, parts if parts is not None else _split_t(th))

    def step(y, hh):
        ks = []
        for i in range(s):
            Y = y + hh * sum((A[i, j] * ks[j] for j in range(i)), torch.zeros(2, dtype=torch.float64))
            ks.append(f(Y))
        return y + hh * sum(b[j] * ks[j] for j in range(s))

    states = [y0]
    for i in range(S):
        states.append(step(states[-1], float(h[i])))
    return torch.stack([step(states[sidx[k]], float(sdt[k])) for k in range(len(sidx))])


def _split_t(th):
    return (th[0:64].reshape(32, 2), th[64:96], th[96:1120].reshape(32, 32), th[1120:1152],
            th[1152:1216].reshape(2, 32), th[1216:1218])


def test_adjoint_against_torch_autograd_replay():
    """Shared weights: the oracle's per-lane contributions summed over lanes
    equal torch's gradient of the summed loss (same mesh)."""
    n = 2
    y0 = np.random.default_rng(4).uniform(0.5, 2.0, (n, 2))
    th = _random_theta(7) * 0.3
    st = [0.25, 0.6, 1.0]
    rec = O.record(O.LV_UDE, O.TSIT5, y0, th, 0.0, 1.0, 1e-6, 1e-6, save_t=st,
                   params_shared=True)
    assert np.all(rec["status"] == O.ST_OK) and rec["S"].max() <= 60
    gp, gy, ll = O.adjoint(O.LV_UDE, O.TSIT5, y0, th, rec, params_shared=True)
    tb = O.erk_tableau(O.TSIT5)
    tt = torch.tensor(th, requires_grad=True)
    total = 0.0
    gys = []
    for l in range(n):
        yt = torch.tensor(y0[l], requires_grad=True)
        out = _torch_replay(tb, yt, tt, rec["h"][l], rec["S"][l], rec["save_idx"][l],
                            rec["save_dt"][l])
        L = (out ** 2).sum()
        L.backward()
        gys.append(yt.grad.numpy().copy())
        total += L.item()
        assert np.isclose(ll[l], L.item(), rtol=1e-13)
    g_ref = tt.grad.numpy()
    assert np.allclose(gp.sum(axis=0), g_ref, rtol=1e-10, atol=1e-12 * np.abs(g_ref).max())
    assert np.allclose(gy, np.array(gys), rtol=1e-11, atol=1e-13)


def test_adjoint_against_dual_numbers():
    """Forward-mode tangents through the oracle's replay (per-lane copies of
    the weights) against the reverse sweep's directional derivative."""
    n = 3
    y0 = np.random.default_rng(5).uniform(0.5, 2.0, (n, 2))
    th = W.ude_weights(0)
    prm = np.tile(th, (n, 1))
    st = list(np.arange(1, 5) * 0.5)
    rec = O.record(O.LV_UDE, O.TSIT5, y0, prm, 0.0, 2.0, 1e-6, 1e-6, save_t=st)
    gp, gy, _ = O.adjoint(O.LV_UDE, O.TSIT5, y0, prm, rec)
    rng = np.random.default_rng(6)
    dy0 = rng.normal(size=y0.shape)
    dp = rng.normal(size=prm.shape)
    ys, dys = O.replay_dual(O.LV_UDE, O.TSIT5, y0, prm, dy0, dp, rec)
    fwd = np.sum(2 * ys * dys, axis=(1, 2))
    rev = np.sum(gp * dp, axis=1) + np.sum(gy * dy0, axis=1)
    assert np.allclose(fwd, rev, rtol=1e-11, atol=1e-13 * np.abs(rev).max())
