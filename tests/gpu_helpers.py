"""Helpers of the GPU tests (no method arithmetic here): a GPU record's mesh
in the oracle's row layout, and the statistics that compare an adaptive mesh
with the oracle's.

Adaptive meshes are compared by statistics (several meshes are correct:
the mesh is whatever the controller's arithmetic makes of it): the step
counts must agree on at least 99.9 % of trajectories, and where they agree
the step sizes must agree to the controller's noise floor.  That floor is
set by the error estimate, a small difference of large stage terms: at
rtol 1e-6 it carries relative rounding noise near 1e-10 (more at tighter
rtol, or where atol governs small components), so any change of rounding
(an ulp of one factor) moves later step sizes by 1e-11..1e-8 relative
(tests/test_controller_noise_floor.py shows it on the CPU; measured on the
GPU against the oracle: medians 1e-10..2e-8, largest 4e-5 at rtol 1e-8).
The bound asserted: the median over trajectories of the largest relative
step-size difference <= 1e-6, and every difference <= 1e-3.  States and
gradients are then compared on one shared mesh: the oracle runs on the
GPU's own mesh.
"""
import numpy as np
import torch

from paper_2609_02876_amd import binding as B


def oracle_mesh(handle, lanes=None):
    """The GPU record's mesh (h, S, save_idx, save_dt), one row per
    trajectory, as the oracle's replay and adjoint take it; `lanes` selects
    trajectories (on the device, before the copy)."""
    h, S = B.ensemble_mesh_export(handle)
    si, sd = handle.save_index(), handle.save_offset()
    if lanes is not None:
        idx = torch.as_tensor(np.asarray(lanes), dtype=torch.long, device=h.device)
        h, S, si, sd = h[:, idx], S[idx], si[:, idx], sd[:, idx]
    torch.cuda.synchronize()
    return dict(h=np.ascontiguousarray(h.cpu().numpy().T),
                S=np.ascontiguousarray(S.cpu().numpy().astype(np.int32)),
                save_idx=np.ascontiguousarray(si.cpu().numpy().T.astype(np.int32)),
                save_dt=np.ascontiguousarray(sd.cpu().numpy().T))


def mesh_stats(gm, ref):
    """(fraction of trajectories with equal step counts, fraction with
    bit-identical meshes, largest relative step-size difference where the
    counts agree, its median over those trajectories)."""
    eq = gm["S"] == ref["S"]
    worst = []
    ident = 0
    for l in np.nonzero(eq)[0]:
        s = int(ref["S"][l])
        a, b = gm["h"][l, :s], ref["h"][l, :s]
        ident += int(np.array_equal(a, b))
        worst.append(float(np.max(np.abs(a - b) / np.abs(b))) if s else 0.0)
    worst = np.array(worst) if worst else np.zeros(1)
    return float(eq.mean()), ident / len(eq), float(worst.max()), float(np.median(worst))


H_MEDIAN = 1e-6   # median over trajectories of the largest relative step-size difference
H_MAX = 1e-3      # any relative step-size difference


def check_mesh(gm, ref, label=""):
    """Assert the adaptive-mesh statistics: equal counts on >= 99.9 % of
    trajectories; where counts agree, relative step-size differences with
    median (over trajectories, of each one's largest) <= H_MEDIAN and
    maximum <= H_MAX."""
    f_eq, f_id, hmax, hmed = mesh_stats(gm, ref)
    print(f"  {label}mesh: S equal on {f_eq:.4f}, bit-identical on {f_id:.4f}, "
          f"h rel diff max {hmax:.2e} median {hmed:.2e}", flush=True)
    assert f_eq >= 0.999, f_eq
    assert hmed <= H_MEDIAN and hmax <= H_MAX, (hmed, hmax)
    return f_eq, f_id, hmax


def rel(a, b):
    """Per-lane normwise relative error (lanes along the last axis)."""
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def own_mesh_parity(hd, so, mo, y0, p, ref, tol, lanes=None, params_shared=False,
                    gp=None, gy=None, label=""):
    """The GPU record hd (and its sweep's gp [P][n], gy [d][n], if given)
    against the oracle run on the GPU's own mesh, after the mesh statistics
    against the oracle's adaptive record ref (of the same lanes).  Returns
    the largest per-lane normwise errors (states, grad_p, grad_y0)."""
    import oracle as O
    gm = oracle_mesh(hd, lanes)
    check_mesh(gm, ref, label)
    sel = slice(None) if lanes is None else np.asarray(lanes)
    y0s = y0[sel]
    ps = p if params_shared else p[sel]
    ys = hd.y_save.double().cpu().numpy()[..., sel]
    ys_g = np.transpose(O.replay(so, mo, y0s, ps, gm, params_shared=params_shared), (1, 2, 0))
    e = [float(rel(ys, ys_g).max()), 0.0, 0.0]
    if gp is not None:
        gp_g, gy_g, _ = O.adjoint(so, mo, y0s, ps, gm, params_shared=params_shared)
        if not params_shared:
            e[1] = float(rel(gp.double().cpu().numpy()[:, sel], gp_g.T).max())
        if gy is not None:
            e[2] = float(rel(gy.double().cpu().numpy()[:, sel], gy_g.T).max())
    print(f"  {label}own mesh vs oracle on it: max rel err states {e[0]:.2e} grad_p {e[1]:.2e} "
          f"grad_y0 {e[2]:.2e}", flush=True)
    assert max(e) <= tol, e
    return e
