"""Full-size launches, as the benchmark runs them, checked on sampled
trajectories that the oracle computes one by one.

* 2^20 Lorenz trajectories on [0, 10] (Tsit5, FP64, 20 save times): the
  headline workload, with the benchmark's pool plan (a pilot record sets the
  per-trajectory reservation);
* 2^20 Lorenz with Vern7 and 2^20 Van der Pol (FP64), and 2^20 Van der Pol
  (Vern7) in FP32 against the FP64 oracle on the GPU's own mesh;
* 2^18 UDE trajectories (FP32): sampled states against the oracle's
  adaptive solve, and sampled y0-gradients against the oracle's adjoint on
  the mesh the GPU recorded for those trajectories.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"lorenz": O.LORENZ, "vdp": O.VDP, "ude": O.LV_UDE}
MET_O = {"tsit5": O.TSIT5, "vern7": O.VERN7}


def _rel(a, b):
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def _planned_record(system, method, y0_d, p_d, t1, rtol, atol, st, shared=False):
    """The benchmark's plan: a pilot record of 8192 trajectories sets the
    reservation per trajectory (mean steps x 1.12 + 16), then the full run."""
    m = min(y0_d.shape[1], 8192)
    pilot = B.ensemble_record(system, method, y0_d[:, :m].contiguous(),
                              p_d if shared else p_d[:, :m].contiguous(), 0.0, t1, rtol, atol,
                              save_times=st, steps_hint=4096, params_shared=shared)
    hint = B.steps_hint_for(float(pilot.steps().double().mean().item()), margin=1.12)
    del pilot
    n = y0_d.shape[1]
    nbytes = B.ensemble_record_bytes(system, method, n, 0.0, t1, hint, len(st) if st else 0,
                                     y0_d.dtype, 0, shared)
    pool = torch.empty(nbytes, dtype=torch.uint8, device=y0_d.device)
    return B.ensemble_record(system, method, y0_d, p_d, 0.0, t1, rtol, atol, save_times=st,
                             pool=pool, steps_per_traj=hint, params_shared=shared)


@pytest.mark.parametrize("system,method,t1,dtype", [
    ("lorenz", "tsit5", 10.0, torch.float64),    # the headline workload
    ("lorenz", "vern7", 10.0, torch.float64),
    ("vdp", "tsit5", 6.3, torch.float64),
    ("vdp", "vern7", 6.3, torch.float32),   # FP32 (chaotic Lorenz on [0, 10] amplifies
                                            # FP32 rounding far beyond 1e-4; its FP32
                                            # parity runs on [0, 2] in test_gpu_parity)
])
def test_full_size_sampled(system, method, t1, dtype):
    n = 1 << 20
    print(f"case full size {system} {method} {dtype} n={n}", flush=True)
    gen = {"lorenz": W.lorenz, "vdp": W.vdp}[system]
    y0, p = gen(n, seed=0)
    if dtype == torch.float32:
        y0 = y0.astype(np.float32).astype(np.float64)
        p = p.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, t1, 20))
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=dtype, device="cuda")
    p_d = torch.tensor(np.ascontiguousarray(p.T), dtype=dtype, device="cuda")
    rec = _planned_record(system, method, y0_d, p_d, t1, 1e-6, 1e-8, st)
    gp, gy, ll = B.ensemble_adjoint(rec)
    torch.cuda.synchronize()
    status = rec.status.cpu().numpy()
    assert np.all(status == 0)
    idx = np.sort(np.random.default_rng(1).choice(n, 64, replace=False))
    idx[0], idx[-1] = 0, n - 1          # the first and last trajectories too
    so, mo = SYS_O[system], MET_O[method]
    if dtype == torch.float64:
        ref = O.record(so, mo, y0[idx], p[idx], 0.0, t1, 1e-6, 1e-8, save_t=st)
        tol = 1e-11
    else:
        # FP32: the oracle's FP64 solution on the GPU's own (FP32) mesh
        cap = int(rec.steps().max().item())
        h, s = B.ensemble_mesh_export(rec, cap)
        h = h.cpu().numpy()[:, idx].T.copy()
        s = s.cpu().numpy()[idx]
        ref = O.record(so, mo, y0[idx], p[idx], 0.0, t1, 1e-6, 1e-8, save_t=st)
        ref["h"], ref["S"] = h, s
        ref["save_idx"] = rec_save_idx(rec, idx)
        ref["save_dt"] = rec_save_dt(rec, idx)
        tol = 1e-4
    gp_o, gy_o, _ = O.adjoint(so, mo, y0[idx], p[idx], ref)
    ys_o = O.replay(so, mo, y0[idx], p[idx], ref)
    ys = rec.y_save.cpu().numpy()[..., idx].astype(np.float64)
    e_s = _rel(ys, np.transpose(ys_o, (1, 2, 0))).max()
    gp_n = gp.cpu().numpy()[:, idx].astype(np.float64)
    gy_n = gy.cpu().numpy()[:, idx].astype(np.float64)
    if dtype == torch.float64:
        e_p, e_y = _rel(gp_n, gp_o.T).max(), _rel(gy_n, gy_o.T).max()
    else:  # per-lane scale as in the FP32 parity test (R13)
        sc = np.sqrt(np.mean(np.sum(gp_o ** 2, axis=1)))
        e_p = (np.linalg.norm(gp_n - gp_o.T, axis=0) / np.maximum(np.linalg.norm(gp_o, axis=1), sc)).max()
        scy = np.sqrt(np.mean(np.sum(gy_o ** 2, axis=1)))
        e_y = (np.linalg.norm(gy_n - gy_o.T, axis=0) / np.maximum(np.linalg.norm(gy_o, axis=1), scy)).max()
    print(f"  sampled: states {e_s:.2e} grad_p {e_p:.2e} grad_y0 {e_y:.2e}")
    assert e_s <= tol and e_p <= tol and e_y <= tol


def rec_save_idx(rec, idx):
    """Save bookkeeping of a record for the sampled trajectories ([k][n_save])."""
    ns = rec.rec.n_save
    n = rec.n
    off = rec.rec.save_idx - rec.pool.data_ptr()
    a = rec.pool[off: off + 4 * ns * n].view(torch.int32).view(ns, n).cpu().numpy()
    return np.ascontiguousarray(a[:, idx].T)


def rec_save_dt(rec, idx):
    ns = rec.rec.n_save
    n = rec.n
    off = rec.rec.save_dt - rec.pool.data_ptr()
    a = rec.pool[off: off + 8 * ns * n].view(torch.float64).view(ns, n).cpu().numpy()
    return np.ascontiguousarray(a[:, idx].T)


def test_ude_max_size_sampled():
    n = 1 << 18
    print(f"case full size ude n={n}", flush=True)
    y0, th = W.ude(n, seed=0)
    y0 = y0.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    st = [0.5 * s for s in range(1, 21)]
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=torch.float32, device="cuda")
    th_d = torch.tensor(th, dtype=torch.float32, device="cuda")
    rec = _planned_record("ude", "tsit5", y0_d, th_d, 10.0, 1e-6, 1e-6, st, shared=True)
    gp, gy, ll = B.ensemble_adjoint(rec)
    torch.cuda.synchronize()
    assert np.all(rec.status.cpu().numpy() == 0)
    assert np.all(np.isfinite(gp.cpu().numpy()))
    idx = np.sort(np.random.default_rng(2).choice(n, 32, replace=False))
    idx[-1] = n - 1
    # states against the oracle's own adaptive solve (both at tolerance 1e-6)
    ref = O.record(O.LV_UDE, O.TSIT5, y0[idx], th, 0.0, 10.0, 1e-6, 1e-6, save_t=st,
                   params_shared=True)
    ys = rec.y_save.cpu().numpy()[..., idx].astype(np.float64)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))
    e_s = np.abs(ys - ys_o).max() / np.abs(ys_o).max()
    # y0-gradients against the oracle's adjoint on the GPU's mesh of these lanes
    cap = int(rec.steps().max().item())
    h, s = B.ensemble_mesh_export(rec, cap)
    mesh = dict(ref)
    mesh["h"] = h.cpu().numpy()[:, idx].T.copy()
    mesh["S"] = s.cpu().numpy()[idx]
    mesh["save_idx"] = rec_save_idx(rec, idx)
    mesh["save_dt"] = rec_save_dt(rec, idx)
    _, gy_o, _ = O.adjoint(O.LV_UDE, O.TSIT5, y0[idx], th, mesh, params_shared=True)
    gy_n = gy.cpu().numpy()[:, idx].astype(np.float64)
    e_y = np.abs(gy_n - gy_o.T).max() / np.abs(gy_o).max()
    print(f"  sampled: states {e_s:.2e} grad_y0 {e_y:.2e}")
    assert e_s <= 1e-4 and e_y <= 1e-4
