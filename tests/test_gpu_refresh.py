"""GPU parity of the mesh refresh (the mesh-drift policy) against the
oracle's refresh, through the C ABI: the old mesh is the GPU's own record,
refreshed at perturbed parameters by both.  The steps kept are compared
trajectory by trajectory; the refreshed meshes (adaptive after the drift
point) by their statistics; save states and the reverse sweep's gradients
against the oracle on the GPU's refreshed mesh, to the FP64 bar."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import check_mesh, oracle_mesh, own_mesh_parity
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"lorenz": O.LORENZ, "vdp": O.VDP, "robertson": O.ROBERTSON, "hires": O.HIRES,
         "linear": O.LINEAR}
MET_O = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}
TOL64 = 1e-11

CASES = [
    # system, method, t1, rtol, atol, n, relative parameter change
    ("lorenz", "tsit5", 10.0, 1e-6, 1e-8, 700, 1e-3),
    ("lorenz", "vern7", 3.0, 1e-8, 1e-10, 300, 1e-2),
    ("vdp", "tsit5", 6.3, 1e-6, 1e-8, 257, 5e-2),
    ("robertson", "rodas4", 1e5, 1e-6, 1e-10, 300, 5e-2),
    ("robertson", "ros23", 1e4, 1e-5, 1e-9, 129, 5e-2),
    ("hires", "rodas4", 321.8122, 1e-6, 1e-10, 200, 2e-2),
]


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


@pytest.mark.parametrize("system,method,t1,rtol,atol,n,dp", CASES)
def test_refresh_matches_oracle(system, method, t1, rtol, atol, n, dp):
    print(f"case refresh {system} {method} n={n} dp={dp}", flush=True)
    y0, p = W.GENERATORS[system](n, seed=11)
    st = list(W.save_times(0.0, t1, 20))
    p2 = p * (1.0 + dp * np.random.default_rng(12).standard_normal(p.shape))
    hint = 2048 if method == "ros23" else 1024
    old = B.ensemble_record(system, method, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                            save_times=st, steps_hint=hint)
    h_old, S_old = B.ensemble_mesh_export(old)
    new, drift = B.refresh_record(old, _dev(y0.T), _dev(p2.T), steps_hint=hint)
    gp, gy, ll = B.ensemble_adjoint(new)
    torch.cuda.synchronize()
    assert np.all(old.status.cpu().numpy() == 0) and np.all(new.status.cpu().numpy() == 0)

    mesh = dict(h=h_old.cpu().numpy().T.copy(), S=S_old.cpu().numpy())
    ref = O.refresh(SYS_O[system], MET_O[method], y0, p2, 0.0, t1, rtol, atol, mesh,
                    save_t=st, cap=8192)
    dr = drift.cpu().numpy()
    print(f"  lanes that left the old mesh: {np.mean(dr < mesh['S']):.3f}; steps kept equal "
          f"on {np.mean(dr == ref['drift_at']):.4f}")
    assert np.mean(dr == ref["drift_at"]) >= 0.999
    S_new = new.steps().cpu().numpy()
    eq = S_new == ref["S"]
    assert np.mean(new.n_trial().cpu().numpy()[eq] == ref["n_trial"][eq]) >= 0.999
    own_mesh_parity(new, SYS_O[system], MET_O[method], y0, p2, ref, TOL64, gp=gp, gy=gy)
    # the kept prefix is the old mesh, bit for bit
    hn, _ = B.ensemble_mesh_export(new, cap=int(S_new.max()))
    hn, ho = hn.cpu().numpy(), h_old.cpu().numpy()
    for l in range(n):
        assert np.array_equal(hn[:dr[l], l], ho[:dr[l], l])


def test_refresh_at_the_recorded_inputs_is_the_record_and_checkpoints_agree():
    n, t1 = 500, 10.0
    y0, p = W.lorenz(n, seed=13)
    st = list(W.save_times(0.0, t1, 20))
    print("case refresh lorenz unchanged inputs", flush=True)
    old = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, t1, 1e-6, 1e-8,
                            save_times=st, steps_hint=512)
    same, drift = B.refresh_record(old, _dev(y0.T), _dev(p.T), steps_hint=512)
    g_old = B.ensemble_adjoint(old)
    g_same = B.ensemble_adjoint(same)
    torch.cuda.synchronize()
    assert torch.equal(drift, old.steps()) and torch.equal(same.steps(), old.steps())
    assert torch.equal(same.n_trial(), old.steps())
    assert torch.equal(same.y_save, old.y_save)
    for a, b in zip(g_old, g_same):
        assert torch.equal(a, b)
    # a perturbed refresh into a checkpointed tape equals the full tape's
    p2 = p * (1.0 + 1e-3 * np.random.default_rng(14).standard_normal(p.shape))
    h, S = B.ensemble_mesh_export(old)
    full, d1 = B.ensemble_refresh("lorenz", "tsit5", _dev(y0.T), _dev(p2.T), 0.0, t1, 1e-6, 1e-8,
                                  h, S, save_times=st, steps_hint=512)
    ck, d2 = B.ensemble_refresh("lorenz", "tsit5", _dev(y0.T), _dev(p2.T), 0.0, t1, 1e-6, 1e-8,
                                h, S, save_times=st, steps_hint=512, ckpt_every=64)
    ga, gb = B.ensemble_adjoint(full), B.ensemble_adjoint(ck)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2) and torch.equal(full.y_save, ck.y_save)
    for a, b in zip(ga, gb):
        assert torch.equal(a, b)


def test_refresh_full_size_sampled():
    """The 2^20 Lorenz record refreshed after a 1e-3 relative parameter step,
    in the launch the bench times: 64 sampled trajectories against the
    oracle's refresh of the same old meshes."""
    cfg, y0, p, st = W.make("lorenz_2p20_t10")
    n = cfg["n"]
    print(f"case refresh lorenz n={n} sampled", flush=True)
    p2 = p * (1.0 + 1e-3 * np.random.default_rng(15).standard_normal(p.shape))
    old = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), cfg["t0"], cfg["t1"],
                            cfg["rtol"], cfg["atol"], save_times=list(st), steps_hint=352)
    new, drift = B.refresh_record(old, _dev(y0.T), _dev(p2.T), steps_hint=352)
    gp, gy, _ = B.ensemble_adjoint(new)
    torch.cuda.synchronize()
    assert np.all(new.status.cpu().numpy() == 0)
    idx = np.sort(np.random.default_rng(16).choice(n, 64, replace=False))
    h_old, S_old = B.ensemble_mesh_export(old)
    mesh = dict(h=h_old.cpu().numpy()[:, idx].T.copy(), S=S_old.cpu().numpy()[idx])
    ref = O.refresh(O.LORENZ, O.TSIT5, y0[idx], p2[idx], cfg["t0"], cfg["t1"], cfg["rtol"],
                    cfg["atol"], mesh, save_t=list(st))
    assert np.array_equal(drift.cpu().numpy()[idx], ref["drift_at"])
    frac = float((drift < S_old).float().mean())
    print(f"  lanes that left the old mesh {frac:.3f}")
    own_mesh_parity(new, O.LORENZ, O.TSIT5, y0, p2, ref, TOL64, lanes=idx, gp=gp, gy=gy,
                    label="sampled ")


def test_refresh_in_fp32_keeps_its_prefix_and_is_idempotent():
    """FP32 (states and stages; h, the error norm and the controller in FP64):
    at the recorded inputs the refresh is the record; after a parameter step
    the kept prefix is the old mesh, and a second refresh keeps everything."""
    n, t1 = 700, 6.3
    y0, p = W.vdp(n, seed=17)
    st = list(W.save_times(0.0, t1, 20))
    f32 = torch.float32
    print("case refresh vdp tsit5 fp32", flush=True)
    old = B.ensemble_record("vdp", "tsit5", _dev(y0.T, f32), _dev(p.T, f32), 0.0, t1, 1e-5,
                            1e-7, save_times=st, steps_hint=512)
    same, d0 = B.refresh_record(old, _dev(y0.T, f32), _dev(p.T, f32), steps_hint=512)
    p2 = p * (1.0 + 0.05 * np.random.default_rng(18).standard_normal(p.shape))
    r1, d1 = B.refresh_record(old, _dev(y0.T, f32), _dev(p2.T, f32), steps_hint=512)
    r2, d2 = B.refresh_record(r1, _dev(y0.T, f32), _dev(p2.T, f32), steps_hint=512)
    torch.cuda.synchronize()
    assert torch.equal(d0, old.steps()) and torch.equal(same.y_save, old.y_save)
    assert np.all(r1.status.cpu().numpy() == 0)
    k = d1.cpu().numpy()
    assert np.any(k < old.steps().cpu().numpy())
    h_old, _ = B.ensemble_mesh_export(old)
    h1, _ = B.ensemble_mesh_export(r1)
    h_old, h1 = h_old.cpu().numpy(), h1.cpu().numpy()
    for l in range(n):
        assert np.array_equal(h1[:k[l], l], h_old[:k[l], l])
    assert torch.equal(d2, r1.steps()) and torch.equal(r2.y_save, r1.y_save)
