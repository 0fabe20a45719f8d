"""Full-size launches, as the benchmark runs them, checked on sampled
trajectories that the oracle computes one by one.

* 2^20 Lorenz trajectories on [0, 10] (Tsit5, FP64, 20 save times): the
  headline workload, with the benchmark's pool plan (a pilot record sets the
  per-trajectory reservation);
* 2^20 Lorenz with Vern7 and 2^20 Van der Pol (FP64), and 2^20 Van der Pol
  (Vern7) in FP32 against the FP64 oracle on the GPU's own mesh;
* 2^20 Lorenz on [0, 10] in FP32: the per-trajectory error against FP64 on
  the shared mesh, reported and bounded;
* 2^18 UDE trajectories (FP32): sampled states and y0-gradients, per
  trajectory, against the oracle on the mesh the GPU recorded for them.
FP64 adaptive meshes are compared with the oracle's by their statistics,
and states and gradients against the oracle on the GPU's own mesh.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import oracle_mesh, own_mesh_parity
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


def _per_lane_scaled(g32, g64):
    """FP32 gradient error per lane against max(|g_lane|, RMS over lanes)
    (a lane whose gradient nearly vanishes has no meaningful relative error)."""
    gn = np.linalg.norm(g64, axis=0)
    return np.linalg.norm(g32 - g64, axis=0) / np.maximum(gn, np.sqrt(np.mean(gn ** 2)))


@pytest.mark.parametrize("system,method,t1,dtype", [
    ("lorenz", "tsit5", 10.0, torch.float64),    # the headline workload
    ("lorenz", "vern7", 10.0, torch.float64),
    ("vdp", "tsit5", 6.3, torch.float64),
    ("vdp", "vern7", 6.3, torch.float32),
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
        own_mesh_parity(rec, so, mo, y0, p, ref, 1e-11, lanes=idx, gp=gp, gy=gy,
                        label="sampled ")
        return
    # FP32: the oracle's FP64 solution on the GPU's own (FP32) mesh
    gm = oracle_mesh(rec, idx)
    gp_o, gy_o, _ = O.adjoint(so, mo, y0[idx], p[idx], gm)
    ys_o = O.replay(so, mo, y0[idx], p[idx], gm)
    ys = rec.y_save.cpu().numpy()[..., idx].astype(np.float64)
    e_s = _rel(ys, np.transpose(ys_o, (1, 2, 0))).max()
    e_p = _per_lane_scaled(gp.cpu().numpy()[:, idx].astype(np.float64), gp_o.T).max()
    e_y = _per_lane_scaled(gy.cpu().numpy()[:, idx].astype(np.float64), gy_o.T).max()
    print(f"  sampled: states {e_s:.2e} grad_p {e_p:.2e} grad_y0 {e_y:.2e}")
    assert e_s <= 1e-4 and e_p <= 1e-4 and e_y <= 1e-4


def test_fp32_lorenz_headline_span_error():
    """FP32 on the headline span: 2^20 Lorenz trajectories on [0, 10] in
    single precision against the FP64 oracle on the same (the GPU's) mesh,
    256 sampled trajectories.  The chaotic flow amplifies FP32 rounding by
    about e^(0.9 t) ~ 8e3 over the span, so the 1e-4 bar of the shorter
    FP32 cases does not hold for every trajectory here; the per-trajectory
    errors are reported (median, p99, max) and bounded as stated: median
    below 1e-4, p99 below 5e-4, every one below 1e-3 (measured: the largest
    1.2e-4, in the parameter gradient)."""
    n = 1 << 20
    t1 = 10.0
    print(f"case fp32 lorenz headline span n={n}", flush=True)
    y0, p = W.lorenz(n, seed=0)
    y0 = y0.astype(np.float32).astype(np.float64)
    p = p.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, t1, 20))
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=torch.float32, device="cuda")
    p_d = torch.tensor(np.ascontiguousarray(p.T), dtype=torch.float32, device="cuda")
    rec = _planned_record("lorenz", "tsit5", y0_d, p_d, t1, 1e-6, 1e-8, st)
    gp, gy, _ = B.ensemble_adjoint(rec)
    torch.cuda.synchronize()
    assert np.all(rec.status.cpu().numpy() == 0)
    idx = np.sort(np.random.default_rng(3).choice(n, 256, replace=False))
    gm = oracle_mesh(rec, idx)
    gp_o, gy_o, _ = O.adjoint(O.LORENZ, O.TSIT5, y0[idx], p[idx], gm)
    ys_o = np.transpose(O.replay(O.LORENZ, O.TSIT5, y0[idx], p[idx], gm), (1, 2, 0))
    ys = rec.y_save.cpu().numpy()[..., idx].astype(np.float64)
    e = {"states": _rel(ys, ys_o),
         "grad_p": _rel(gp.cpu().numpy()[:, idx].astype(np.float64), gp_o.T),
         "grad_y0": _rel(gy.cpu().numpy()[:, idx].astype(np.float64), gy_o.T)}
    for k, v in e.items():
        print(f"  {k}: per-trajectory relative error median {np.median(v):.2e} "
              f"p99 {np.quantile(v, 0.99):.2e} max {v.max():.2e}", flush=True)
        assert np.median(v) <= 1e-4 and np.quantile(v, 0.99) <= 5e-4 and v.max() <= 1e-3


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
    # per trajectory, normwise: the FP32 states and y0-gradients against the
    # FP64 oracle on the mesh the GPU recorded for these trajectories
    gm = oracle_mesh(rec, idx)
    ys_o = np.transpose(O.replay(O.LV_UDE, O.TSIT5, y0[idx], th, gm, params_shared=True),
                        (1, 2, 0))
    _, gy_o, _ = O.adjoint(O.LV_UDE, O.TSIT5, y0[idx], th, gm, params_shared=True)
    ys = rec.y_save.cpu().numpy()[..., idx].astype(np.float64)
    e_s = _rel(ys, ys_o)
    e_y = _rel(gy.cpu().numpy()[:, idx].astype(np.float64), gy_o.T)
    print(f"  sampled per trajectory: states median {np.median(e_s):.2e} max {e_s.max():.2e}; "
          f"grad_y0 median {np.median(e_y):.2e} max {e_y.max():.2e}")
    assert e_s.max() <= 1e-4 and e_y.max() <= 1e-4
