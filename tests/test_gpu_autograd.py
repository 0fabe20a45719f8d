"""torch.autograd path: gradcheck on the frozen-mesh map, agreement with the
oracle's discrete adjoint, and shared-parameter sums."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import oracle_mesh
from paper_2609_02876_amd import autograd as AG
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64, grad=False):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda", requires_grad=grad)


def test_gradcheck_frozen_mesh():
    """Finite differences of the replayed map (mesh held fixed) match the
    reverse sweep -- the paper's check inside the same recorded replay."""
    y0, p = W.lorenz(4, seed=11)
    st = [0.1, 0.25, 0.4]
    Y0, P = _dev(y0.T, grad=True), _dev(p.T, grad=True)
    mesh = AG.frozen_mesh("lorenz", "tsit5", Y0, P, 0.0, 0.4, save_times=st, steps_hint=64)
    f = lambda a, b: AG.odeint("lorenz", "tsit5", a, b, 0.0, 0.4, save_times=st, mesh=mesh)
    assert torch.autograd.gradcheck(f, (Y0, P), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("system,method,t1", [("lorenz", "tsit5", 10.0), ("vdp", "vern7", 6.3)])
def test_autograd_matches_oracle(system, method, t1):
    n = 500
    gen = {"lorenz": W.lorenz, "vdp": W.vdp}[system]
    y0, p = gen(n, seed=12)
    st = list(W.save_times(0.0, t1, 20))
    Y0, P = _dev(y0.T, grad=True), _dev(p.T, grad=True)
    ys = AG.odeint(system, method, Y0, P, 0.0, t1, 1e-6, 1e-8, save_times=st)
    loss = (ys ** 2).sum()
    loss.backward()
    so = {"lorenz": O.LORENZ, "vdp": O.VDP}[system]
    mo = {"tsit5": O.TSIT5, "vern7": O.VERN7}[method]
    # the oracle's discrete adjoint on the mesh the forward recorded (the
    # record is deterministic: a second record of the same inputs has it)
    hd = B.ensemble_record(system, method, Y0.detach(), P.detach(), 0.0, t1, 1e-6, 1e-8,
                           save_times=st)
    gp_o, gy_o, ll_o = O.adjoint(so, mo, y0, p, oracle_mesh(hd))
    assert np.isclose(loss.item(), ll_o.sum(), rtol=1e-12)
    assert np.array_equal(P.grad.cpu().numpy(), gp_o.T)
    assert np.array_equal(Y0.grad.cpu().numpy(), gy_o.T)


def test_shared_parameters_sum_over_trajectories():
    n = 1000
    rng = np.random.default_rng(13)
    y0 = np.stack([1 + rng.random(n), rng.random(n), rng.random(n)], 1)
    p = np.array([10.0, 28.0, 8.0 / 3.0])
    Y0, P = _dev(y0.T), _dev(p, grad=True)
    ys = AG.odeint("lorenz", "tsit5", Y0, P, 0.0, 2.0, 1e-6, 1e-8, save_times=[1.0, 2.0],
                   params_shared=True)
    (ys ** 2).sum().backward()
    g1 = P.grad.clone()
    # deterministic: a second run gives the same bits
    P.grad = None
    ys = AG.odeint("lorenz", "tsit5", Y0, P, 0.0, 2.0, 1e-6, 1e-8, save_times=[1.0, 2.0],
                   params_shared=True)
    (ys ** 2).sum().backward()
    assert torch.equal(g1, P.grad)
    hd = B.ensemble_record("lorenz", "tsit5", Y0, P.detach(), 0.0, 2.0, 1e-6, 1e-8,
                           save_times=[1.0, 2.0], params_shared=True)
    gp_o, _, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, p, oracle_mesh(hd), params_shared=True)
    ref_sum = gp_o.sum(axis=0)
    assert np.allclose(g1.cpu().numpy(), ref_sum, rtol=1e-12, atol=0)


def test_record_reuse_while_parameters_move():
    """One mesh, parameters moved: the replay differentiates at the new point
    with the old mesh (Section 3.1)."""
    n = 256
    y0, p = W.lorenz(n, seed=14)
    st = [0.5, 1.0]
    Y0, P = _dev(y0.T), _dev(p.T)
    mesh = AG.frozen_mesh("lorenz", "tsit5", Y0, P, 0.0, 1.0, save_times=st, steps_hint=96)
    p2 = p * 1.01
    P2 = _dev(p2.T, grad=True)
    ys = AG.odeint("lorenz", "tsit5", Y0, P2, 0.0, 1.0, save_times=st, mesh=mesh)
    (ys ** 2).sum().backward()
    # the oracle on the same (old) mesh at the new parameters
    hd = B.ensemble_record("lorenz", "tsit5", Y0, P, 0.0, 1.0, 1e-6, 1e-8, save_times=st,
                           steps_hint=96)
    gp_o, _, _ = O.adjoint(O.LORENZ, O.TSIT5, y0, p2, oracle_mesh(hd))
    assert np.array_equal(P2.grad.cpu().numpy(), gp_o.T)


def test_inplace_change_of_inputs_is_refused():
    """The sweep reads y0 and params through their storage: a change in
    place between forward and backward must fail (torch's version check),
    not give a gradient at mixed inputs."""
    y0, p = W.lorenz(64, seed=15)
    Y0, P = _dev(y0.T), _dev(p.T, grad=True)
    ys = AG.odeint("lorenz", "tsit5", Y0, P, 0.0, 0.5, save_times=[0.5])
    with torch.no_grad():
        P.mul_(1.01)
    with pytest.raises(RuntimeError, match="modified by an inplace operation"):
        (ys ** 2).sum().backward()
