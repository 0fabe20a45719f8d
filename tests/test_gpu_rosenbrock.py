"""GPU parity of the Rosenbrock path (Rodas4 and Rosenbrock23) against the
CPU oracle: Robertson and HIRES (paper, Appendix A) and the damped rotation,
FP64.

States and gradients are compared on a shared mesh (the oracle on the GPU's
own mesh, and the oracle's mesh replayed on the GPU) at the FP64 bar
(per-lane normwise relative error <= 1e-11); the two adaptive meshes are
compared by their statistics (equal step counts on >= 99.9 % of
trajectories, step sizes to the controller's noise floor where the counts
agree; gpu_helpers).
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import oracle_mesh, own_mesh_parity
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"robertson": O.ROBERTSON, "hires": O.HIRES, "linear": O.LINEAR}
T1 = {"robertson": 1e5, "hires": 321.8122, "linear": 8.0}
TOL64 = 1e-11
METHODS = [("rodas4", O.RODAS), ("ros23", O.ROS23)]
# taped steps reserved per trajectory (Rosenbrock23, of order 2, takes about
# four times the steps of Rodas4 at rtol 1e-6)
HINT = {"rodas4": 512, "ros23": 2560}


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def _gen(system):
    return W.GENERATORS[system]




CASES = [
    # system, n, rtol, atol, n_save
    ("robertson", 1000, 1e-6, 1e-10, 20),
    ("hires", 600, 1e-6, 1e-10, 20),
    ("linear", 129, 1e-7, 1e-9, 5),
    ("robertson", 257, 1e-4, 1e-8, 0),
]


@pytest.mark.parametrize("meth,mo", METHODS)
@pytest.mark.parametrize("system,n,rtol,atol,ns", CASES)
def test_ros_record_and_adjoint_match_oracle(meth, mo, system, n, rtol, atol, ns):
    print(f"case {meth} {system} n={n} rtol={rtol} atol={atol} ns={ns}", flush=True)
    t1 = T1[system]
    y0, p = _gen(system)(n, seed=5)
    st = list(W.save_times(0.0, t1, ns)) if ns else None
    so = SYS_O[system]
    ref = O.record(so, mo, y0, p, 0.0, t1, rtol, atol, save_t=st)
    assert np.all(ref["status"] == O.ST_OK)
    gp_o, gy_o, ll_o = O.adjoint(so, mo, y0, p, ref)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))

    hd = B.ensemble_record(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                           save_times=st, steps_hint=int(ref["S"].max()) + 16)
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    own_mesh_parity(hd, so, mo, y0, p, ref, TOL64, gp=gp, gy=gy)

    # the oracle's mesh replayed on the device, every lane
    S = ref["S"]
    cap = max(1, int(S.max()))
    h_dev = _dev(np.ascontiguousarray(ref["h"][:, :cap].T))
    S_dev = torch.tensor(S, dtype=torch.int32, device="cuda")
    hf = B.ensemble_replay_mesh(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, h_dev, S_dev,
                                save_times=st)
    gp2, gy2, _ = B.ensemble_adjoint(hf)
    torch.cuda.synchronize()
    e_state = _rel(hf.y_save.cpu().numpy(), ys_o)
    e_gp = _rel(gp2.cpu().numpy(), gp_o.T)
    e_gy = _rel(gy2.cpu().numpy(), gy_o.T)
    print(f"  oracle mesh: max rel err states {e_state.max():.2e} grad_p {e_gp.max():.2e} "
          f"grad_y0 {e_gy.max():.2e}")
    assert e_state.max() <= TOL64 and e_gp.max() <= TOL64 and e_gy.max() <= TOL64


@pytest.mark.parametrize("meth,mo", METHODS)
@pytest.mark.parametrize("system,K", [("robertson", 16), ("hires", 64)])
def test_ros_checkpointed_tape_gives_the_same_bits(meth, mo, system, K):
    print(f"case {meth} {system} checkpoint every {K}", flush=True)
    n, t1 = 700, T1[system]
    y0, p = _gen(system)(n, seed=6)
    st = list(W.save_times(0.0, t1, 20))
    full = B.ensemble_record(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-10,
                             save_times=st, steps_hint=HINT[meth])
    ck = B.ensemble_record(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-10,
                           save_times=st, steps_hint=HINT[meth], ckpt_every=K)
    g1 = B.ensemble_adjoint(full)
    g2 = B.ensemble_adjoint(ck)
    torch.cuda.synchronize()
    assert torch.equal(full.y_save, ck.y_save)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    assert ck.pool.numel() < full.pool.numel()


@pytest.mark.parametrize("meth,mo", METHODS)
def test_ros_shared_parameters_sum(meth, mo):
    n = 600
    y0, _ = W.hires(n, seed=7)
    p = np.array(W.HIRES_THETA)
    st = list(W.save_times(0.0, T1["hires"], 10))
    print(f"case {meth} hires shared params", flush=True)
    hd = B.ensemble_record("hires", meth, _dev(y0.T), _dev(p), 0.0, T1["hires"], 1e-6, 1e-10,
                           save_times=st, params_shared=True, steps_hint=HINT[meth])
    gp, _, _ = B.ensemble_adjoint(hd)
    gp_b, _, _ = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert torch.equal(gp, gp_b)  # fixed-order reduction
    ref = O.record(O.HIRES, mo, y0, p, 0.0, T1["hires"], 1e-6, 1e-10, save_t=st,
                   params_shared=True)
    own_mesh_parity(hd, O.HIRES, mo, y0, p, ref, TOL64, params_shared=True)
    gp_o, _, _ = O.adjoint(O.HIRES, mo, y0, p, oracle_mesh(hd), params_shared=True)
    ref_sum = gp_o.sum(axis=0)
    err = np.abs(gp.cpu().numpy() - ref_sum) / np.abs(ref_sum).max()
    print(f"  max err / max |grad| {err.max():.2e}")
    assert err.max() <= 1e-12


@pytest.mark.parametrize("meth,mo", METHODS)
def test_ros_save_at_t0_and_t1_and_invariants(meth, mo):
    """A save at t0 is a zero-length side step (the identity); saves at t1
    come after the last step.  Robertson conserves y0 + y1 + y2 and so the
    gradient of the total at any save is zero in k and one in y0."""
    n, t1 = 300, 1e4
    y0, p = W.robertson(n, seed=8)
    st = [0.0, 1.0, 100.0, t1]
    print(f"case {meth} robertson saves at t0/t1", flush=True)
    hd = B.ensemble_record("robertson", meth, _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-10,
                           save_times=st, steps_hint=HINT[meth])
    ys = hd.y_save.cpu().numpy()
    assert np.array_equal(ys[0], y0.T)
    tot = ys.sum(axis=1)
    assert np.abs(tot - 1.0).max() <= 1e-13
    # cotangent of the sum of species at every save: d/dk = 0, d/dy0 = n_save
    cot = torch.ones((len(st), 3, n), dtype=torch.float64, device="cuda")
    gp, gy, _ = B.ensemble_adjoint(hd, loss="cotangent", data=cot, want_loss=False)
    gref, _, _ = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    gp_n, gy_n = gp.cpu().numpy(), gy.cpu().numpy()
    assert np.abs(gy_n - len(st)).max() < 1e-11
    # against each lane's gradient scale for the sum-of-squares loss
    assert np.abs(gp_n / np.abs(gref.cpu().numpy()).max(axis=0, keepdims=True)).max() < 1e-11
    ref = O.record(O.ROBERTSON, mo, y0, p, 0.0, t1, 1e-6, 1e-10, save_t=st)
    own_mesh_parity(hd, O.ROBERTSON, mo, y0, p, ref, TOL64)


@pytest.mark.parametrize("meth,mo", METHODS)
@pytest.mark.parametrize("system", ["robertson", "hires"])
def test_ros_full_size_sampled(meth, mo, system):
    """2^18 lanes, the largest stiff ensemble, in the launch that is timed:
    64 sampled lanes against the oracle run on those lanes alone."""
    cfg, y0, p, st = W.make(f"{system}_2p18" + ("_t1e5" if system == "robertson" else ""))
    n = cfg["n"]
    print(f"case {meth} {system} n={n} sampled", flush=True)
    hd = B.ensemble_record(system, meth, _dev(y0.T), _dev(p.T), cfg["t0"], cfg["t1"],
                           cfg["rtol"], cfg["atol"], save_times=list(st), steps_hint=HINT[meth])
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    status = hd.status.cpu().numpy()
    assert np.all(status == 0)
    idx = np.sort(np.random.default_rng(9).choice(n, 64, replace=False))
    ref = O.record(SYS_O[system], mo, y0[idx], p[idx], cfg["t0"], cfg["t1"], cfg["rtol"],
                   cfg["atol"], save_t=list(st))
    own_mesh_parity(hd, SYS_O[system], mo, y0, p, ref, TOL64, lanes=idx, gp=gp, gy=gy,
                    label="sampled ")


@pytest.mark.parametrize("meth,mo", METHODS)
@pytest.mark.parametrize("system,n", [("robertson", 500), ("hires", 300)])
def test_ros_solve_matches_oracle(meth, mo, system, n):
    """The forward-only solve (no record) against the oracle's adaptive
    solve: per-trajectory normwise state error at 20 save times (the two
    meshes may differ at the controller's noise floor, which these
    contractive stiff flows do not amplify), and the same bits as the
    record's save states."""
    print(f"case {meth} solve {system} n={n}", flush=True)
    y0, p = _gen(system)(n, 5)
    t1 = T1[system]
    st = list(W.save_times(0.0, t1, 20))
    ref = O.record(SYS_O[system], mo, y0, p, 0.0, t1, 1e-6, 1e-10, save_t=st)
    assert np.all(ref["status"] == O.ST_OK)
    ys, status = B.ensemble_solve(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-10,
                                  save_times=st)
    hd = B.ensemble_record(system, meth, _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-10,
                           save_times=st, steps_hint=HINT[meth])
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    assert torch.equal(ys, hd.y_save) and torch.equal(status, hd.status)
    e = _rel(ys.cpu().numpy(), np.transpose(ref["y_save"], (1, 2, 0)))
    print(f"  per-trajectory state error median {np.median(e):.2e} p99 "
          f"{np.quantile(e, 0.99):.2e} max {e.max():.2e}", flush=True)
    assert e.max() <= 1e-9
