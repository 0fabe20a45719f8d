"""Dense output on the GPU (save states from the continuous extension of the
accepted step, no extra step), through the C ABI, against the oracle's dense
replay and adjoint on the same mesh (FP64 bar 1e-11; FP32 1e-4), with the
adaptive mesh compared by its statistics."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import check_mesh, oracle_mesh, rel
from paper_2609_02876_amd import _abi as A
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"lorenz": O.LORENZ, "vdp": O.VDP, "robertson": O.ROBERTSON, "hires": O.HIRES,
         "linear": O.LINEAR}
MET_O = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}
T1 = {"lorenz": 10.0, "vdp": 6.3, "robertson": 1e5, "hires": 321.8122, "linear": 8.0}
TOLS = {"lorenz": (1e-6, 1e-8), "vdp": (1e-6, 1e-8), "robertson": (1e-6, 1e-10),
        "hires": (1e-6, 1e-10), "linear": (1e-7, 1e-9)}
HINT = {"ros23": 2560}


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _record(system, method, y0, p, st, dtype=torch.float64, **kw):
    rtol, atol = TOLS[system]
    return B.ensemble_record(system, method, _dev(y0.T, dtype), _dev(p.T, dtype), 0.0,
                             T1[system], rtol, atol, save_times=st, dense=True,
                             steps_hint=HINT.get(method, 512), **kw)


@pytest.mark.parametrize("system,method,n", [
    ("lorenz", "tsit5", 1000), ("lorenz", "vern7", 400), ("vdp", "tsit5", 513),
    ("linear", "tsit5", 129), ("robertson", "rodas4", 500), ("robertson", "ros23", 257),
    ("hires", "rodas4", 300), ("linear", "rodas4", 65)])
def test_dense_record_and_adjoint_match_oracle(system, method, n):
    print(f"case dense {system} {method} n={n}", flush=True)
    y0, p = W.GENERATORS[system](n, seed=51)
    st = list(W.save_times(0.0, T1[system], 20))
    hd = _record(system, method, y0, p, st)
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    so, mo = SYS_O[system], MET_O[method]
    rtol, atol = TOLS[system]
    gm = oracle_mesh(hd)
    check_mesh(gm, O.record(so, mo, y0, p, 0.0, T1[system], rtol, atol, save_t=st))
    ys_o = O.replay(so, mo, y0, p, gm, dense=True)
    gp_o, gy_o, ll_o = O.adjoint(so, mo, y0, p, gm, dense=True)
    e = (rel(hd.y_save.cpu().numpy(), np.transpose(ys_o, (1, 2, 0))).max(),
         rel(gp.cpu().numpy(), gp_o.T).max(), rel(gy.cpu().numpy(), gy_o.T).max())
    print(f"  dense vs oracle on the GPU's mesh: states {e[0]:.2e} grad_p {e[1]:.2e} "
          f"grad_y0 {e[2]:.2e}", flush=True)
    assert max(e) <= 1e-11
    assert np.allclose(ll.cpu().numpy(), ll_o, rtol=1e-12, atol=0)
    # the oracle's mesh replayed on the GPU with dense saves
    ref = O.record(so, mo, y0, p, 0.0, T1[system], rtol, atol, save_t=st)
    cap = int(ref["S"].max())
    hr = B.ensemble_replay_mesh(system, method, _dev(y0.T), _dev(p.T), 0.0, T1[system],
                                _dev(ref["h"][:, :cap].T),
                                torch.tensor(ref["S"], dtype=torch.int32, device="cuda"),
                                save_times=st, dense=True)
    gp2, gy2, _ = B.ensemble_adjoint(hr)
    torch.cuda.synchronize()
    ys2 = O.replay(so, mo, y0, p, ref, dense=True)
    gp2_o, gy2_o, _ = O.adjoint(so, mo, y0, p, ref, dense=True)
    e2 = (rel(hr.y_save.cpu().numpy(), np.transpose(ys2, (1, 2, 0))).max(),
          rel(gp2.cpu().numpy(), gp2_o.T).max(), rel(gy2.cpu().numpy(), gy2_o.T).max())
    print(f"  oracle's mesh replayed: {max(e2):.2e}", flush=True)
    assert max(e2) <= 1e-11


@pytest.mark.parametrize("system,method,K", [("lorenz", "tsit5", 64), ("robertson", "rodas4", 16)])
def test_dense_checkpointed_tape_solve_and_saves_at_the_ends(system, method, K):
    print(f"case dense {system} {method} checkpoint {K}", flush=True)
    n = 600
    y0, p = W.GENERATORS[system](n, seed=52)
    st = [0.0] + list(W.save_times(0.0, T1[system], 10))   # a save at t0 and at t1
    full = _record(system, method, y0, p, st)
    ck = _record(system, method, y0, p, st, ckpt_every=K)
    g1, g2 = B.ensemble_adjoint(full), B.ensemble_adjoint(ck)
    rtol, atol = TOLS[system]
    ys, status = B.ensemble_solve(system, method, _dev(y0.T), _dev(p.T), 0.0, T1[system], rtol,
                                  atol, save_times=st, dense=True)
    torch.cuda.synchronize()
    assert torch.equal(full.y_save, ck.y_save)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    assert torch.equal(ys, full.y_save) and torch.equal(status, full.status)
    assert torch.equal(full.y_save[0], _dev(y0.T))       # theta = 0 at t0: y0 itself


def test_dense_shared_parameters_and_fp32():
    print("case dense shared hires and fp32 vdp", flush=True)
    n = 400
    y0, _ = W.hires(n, seed=53)
    p = np.array(W.HIRES_THETA)
    st = list(W.save_times(0.0, T1["hires"], 10))
    hd = B.ensemble_record("hires", "rodas4", _dev(y0.T), _dev(p), 0.0, T1["hires"], 1e-6,
                           1e-10, save_times=st, params_shared=True, dense=True)
    gp, _, _ = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    gp_o, _, _ = O.adjoint(O.HIRES, O.RODAS, y0, p, oracle_mesh(hd), params_shared=True,
                           dense=True)
    ref = gp_o.sum(axis=0)
    assert np.abs(gp.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    # FP32 dense against the FP64 oracle on the GPU's mesh
    y1, p1 = W.vdp(512, seed=54)
    y1 = y1.astype(np.float32).astype(np.float64)
    p1 = p1.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, 6.3, 20))
    h32 = _record("vdp", "tsit5", y1, p1, st, dtype=torch.float32)
    gp32, _, _ = B.ensemble_adjoint(h32)
    torch.cuda.synchronize()
    gm = oracle_mesh(h32)
    ys_o = O.replay(O.VDP, O.TSIT5, y1, p1, gm, dense=True)
    gp_o, _, _ = O.adjoint(O.VDP, O.TSIT5, y1, p1, gm, dense=True)
    assert rel(h32.y_save.double().cpu().numpy(), np.transpose(ys_o, (1, 2, 0))).max() <= 1e-4
    assert np.median(rel(gp32.double().cpu().numpy(), gp_o.T)) <= 1e-4


def test_dense_refusals():
    y0, p = W.lorenz(64, seed=55)
    h = _record("lorenz", "tsit5", y0, p, [0.5, 1.0])
    with pytest.raises(A.EnsembleError, match="dense"):
        B.ensemble_jvp(h)
    hs, S = B.ensemble_mesh_export(h)
    with pytest.raises(A.EnsembleError, match="dense"):
        B.ensemble_refresh("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, 1e-6, 1e-8, hs, S,
                           save_times=[0.5, 1.0], dense=True)
    yu, th = W.ude(64, seed=0)
    with pytest.raises(A.EnsembleError, match="dense"):
        B.ensemble_record("ude", "tsit5", _dev(yu.T, torch.float32), _dev(th, torch.float32), 0.0,
                          10.0, 1e-6, 1e-6, save_times=[5.0], params_shared=True, dense=True)
    torch.cuda.synchronize()


def test_dense_full_size_sampled():
    """The headline shape with dense saves: 2^20 Lorenz trajectories on
    [0, 10], 20 saves, in one launch; 64 sampled trajectories."""
    cfg, y0, p, st = W.make("lorenz_2p20_t10")
    n = cfg["n"]
    print(f"case dense lorenz n={n} sampled", flush=True)
    hd = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, 1e-6, 1e-8,
                           save_times=list(st), steps_hint=352, dense=True)
    gp, gy, _ = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    idx = np.sort(np.random.default_rng(56).choice(n, 64, replace=False))
    gm = oracle_mesh(hd, idx)
    ys_o = O.replay(O.LORENZ, O.TSIT5, y0[idx], p[idx], gm, dense=True)
    gp_o, gy_o, _ = O.adjoint(O.LORENZ, O.TSIT5, y0[idx], p[idx], gm, dense=True)
    e = max(rel(hd.y_save.cpu().numpy()[..., idx], np.transpose(ys_o, (1, 2, 0))).max(),
            rel(gp.cpu().numpy()[:, idx], gp_o.T).max(), rel(gy.cpu().numpy()[:, idx], gy_o.T).max())
    print(f"  sampled max rel err {e:.2e}", flush=True)
    assert e <= 1e-11
