"""An independent replay at the benchmark's shapes, to show that agreement
with the oracle does not rest on a shared rounding order.

The replays below are written here with torch float64 autograd on the CPU,
in natural order: sums left to right with plain multiply-adds (no fused
operations), the Rosenbrock stage solves by torch.linalg.solve (LAPACK's
own LU and pivot order) on W = I/(gamma h) - J with J formed by torch's
autograd of the right-hand side, so that the derivative of J enters the
gradient by the chain rule (the terms Section 3.2 names for the stiff
adjoint).  Only the tableau coefficients come from the oracle; they are
pinned separately by the order conditions.  The mesh is the oracle's
recorded one, held fixed (the sg[h] convention of Section 3.1).

Workloads: Lorenz on t in [0, 10] with the loss summed over 20 save times
(the headline shape), Tsit5 and Vern7; Robertson on t in [0, 1e5] with
Rodas4 and Rosenbrock23, 20 save times.  Bound: 1e-11 relative, normwise per
trajectory, on save states, parameter gradients and initial-state
gradients (the FP64 parity bar).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_02876_amd import workloads as W

TOL = 1e-11


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _lorenz_f(p):
    def f(y):
        return torch.stack([p[0] * (y[1] - y[0]), y[0] * (p[1] - y[2]) - y[1],
                            y[0] * y[1] - p[2] * y[2]])
    return f


def _robertson_f(p):
    def f(y):
        a = p[0] * y[0]
        b = p[2] * y[1] * y[2]
        c = p[1] * y[1] * y[1]
        return torch.stack([b - a, a - b - c, c])
    return f


def _erk_step(tb, f, y, h):
    A, b, s = tb["A"], tb["b"], tb["s"]
    ks = []
    for i in range(s):
        acc = torch.zeros_like(y)
        for j in range(i):
            if A[i, j] != 0.0:
                acc = acc + float(A[i, j]) * ks[j]
        ks.append(f(y + h * acc))
    acc = torch.zeros_like(y)
    for j in range(s):
        if b[j] != 0.0:
            acc = acc + float(b[j]) * ks[j]
    return y + h * acc


def _ros_step(tb, f, y, h):
    if h == 0.0:
        return y
    d = y.shape[0]
    J = torch.autograd.functional.jacobian(f, y, create_graph=True)
    Wm = torch.eye(d, dtype=torch.float64) / (tb["gamma"] * h) - J
    a, c, m, su, s = tb["a"], tb["c"], tb["m"], tb["su"], tb["s"]
    us = []
    for i in range(su):
        Yi = y
        rhs = torch.zeros_like(y)
        for j in range(i):
            if a[i, j] != 0.0:
                Yi = Yi + float(a[i, j]) * us[j]
            if c[i, j] != 0.0:
                rhs = rhs + (float(c[i, j]) / h) * us[j]
        us.append(torch.linalg.solve(Wm, f(Yi) + rhs))
    out = y
    for j in range(su):
        if m[j] != 0.0:
            out = out + float(m[j]) * us[j]
    return out


def _replay_loss(step, rec, lane, y0, p):
    """States y_0..y_S on the frozen mesh, save states by one extra step
    from their base points, loss = sum of squares of the save states."""
    S = int(rec["S"][lane])
    states = [y0]
    for i in range(S):
        states.append(step(states[-1], float(rec["h"][lane, i])))
    saves = [step(states[int(rec["save_idx"][lane, k])], float(rec["save_dt"][lane, k]))
             for k in range(rec["save_idx"].shape[1])]
    ys = torch.stack(saves)
    return ys, (ys ** 2).sum()


def _check(system, method, step_of, y0, prm, rec):
    gp, gy, ll = O.adjoint(system, method, y0, prm, rec)
    for l in range(y0.shape[0]):
        yt = torch.tensor(y0[l], requires_grad=True)
        pt = torch.tensor(prm[l], requires_grad=True)
        ys, L = _replay_loss(step_of(pt), rec, l, yt, pt)
        L.backward()
        assert _rel(ys.detach().numpy(), rec["y_save"][l]) <= TOL
        assert _rel(pt.grad.numpy(), gp[l]) <= TOL, (pt.grad.numpy(), gp[l])
        assert _rel(yt.grad.numpy(), gy[l]) <= TOL, (yt.grad.numpy(), gy[l])
        assert abs(L.item() - ll[l]) <= TOL * abs(ll[l])


@pytest.mark.slow
@pytest.mark.parametrize("method", [O.TSIT5, O.VERN7])
def test_lorenz_headline_shape(method):
    cfg, y0, prm, st = W.make("lorenz_2p20_t10", n=3)
    rec = O.record(O.LORENZ, method, y0, prm, 0.0, 10.0, 1e-6, 1e-8, save_t=st)
    assert np.all(rec["status"] == O.ST_OK) and rec["S"].min() > 100
    tb = O.erk_tableau(method)
    _check(O.LORENZ, method, lambda pt: (lambda y, h: _erk_step(tb, _lorenz_f(pt), y, h)),
           y0, prm, rec)


@pytest.mark.slow
@pytest.mark.parametrize("method", [O.RODAS, O.ROS23])
def test_robertson_rosenbrock(method):
    cfg, y0, prm, st = W.make("robertson_2p18_t1e5", n=2)
    rec = O.record(O.ROBERTSON, method, y0, prm, 0.0, 1e5, 1e-6, 1e-10, save_t=st)
    assert np.all(rec["status"] == O.ST_OK)
    tb = O.ros_tableau(method)
    _check(O.ROBERTSON, method,
           lambda pt: (lambda y, h: _ros_step(tb, _robertson_f(pt), y, h)), y0, prm, rec)
