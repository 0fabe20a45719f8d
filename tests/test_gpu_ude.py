"""GPU parity of the universal differential equation (Lotka-Volterra plus a
2-32-32-2 tanh MLP with shared weights; Tsit5, FP32 on matrix cores) against
the FP64 oracle.

The device computes in FP32 and the oracle in FP64, so the bar is the FP32
one: 1e-4, measured against the scale of the compared quantity (the largest
|state| for save states, the largest |gradient| for the shared-weight
gradient, which is a sum over the ensemble, and the cancelling terms
scale * sum |y|^2 for the MSE loss).  Gradients are compared on the
oracle's mesh replayed on the GPU (the same discrete map); the GPU's own
adaptive record is compared on its states.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2609_02876_amd import autograd as AG
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-4
T1 = 10.0
ST = [0.5 * s for s in range(1, 21)]


def _dev(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _case(n, seed=0):
    y0, th = W.ude(n, seed)
    # FP32 inputs: the oracle sees the same (rounded) values
    y0 = y0.astype(np.float32).astype(np.float64)
    th = th.astype(np.float32).astype(np.float64)
    return y0, th


def _targets(y0):
    """Synthetic targets: the teacher network's solution (FP64 oracle, rtol 1e-10)."""
    tt = W.ude_teacher()
    rec = O.record(O.LV_UDE, O.TSIT5, y0, tt, 0.0, T1, 1e-10, 1e-10, save_t=ST,
                   params_shared=True)
    assert np.all(rec["status"] == O.ST_OK)
    return rec["y_save"]          # [n][n_save][2]


@pytest.mark.parametrize("n", [100, 1000])
def test_ude_replay_and_adjoint_match_oracle(n):
    print(f"case ude n={n} oracle mesh", flush=True)
    y0, th = _case(n, seed=1)
    tgt = _targets(y0)
    scale = 1.0 / (n * len(ST) * 2)
    ref = O.record(O.LV_UDE, O.TSIT5, y0, th, 0.0, T1, 1e-6, 1e-6, save_t=ST, params_shared=True)
    assert np.all(ref["status"] == O.ST_OK)
    gp_o, gy_o, ll_o = O.adjoint(O.LV_UDE, O.TSIT5, y0, th, ref, O.LOSS_MSE_TARGET, tgt, scale,
                                 params_shared=True)
    g_o = gp_o.sum(axis=0)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))      # [ns, 2, n]

    S = ref["S"]
    cap = int(S.max())
    h_dev = _dev(np.ascontiguousarray(ref["h"][:, :cap].T), torch.float64)
    S_dev = torch.tensor(S, dtype=torch.int32, device="cuda")
    hd = B.ensemble_replay_mesh("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, h_dev, S_dev,
                                save_times=ST, params_shared=True)
    data = _dev(np.transpose(tgt, (1, 2, 0)))
    gp, gy, ll = B.ensemble_adjoint(hd, "mse", data, scale)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    ys = hd.y_save.cpu().numpy().astype(np.float64)
    e_state = np.abs(ys - ys_o).max() / np.abs(ys_o).max()
    g = gp.cpu().numpy().astype(np.float64)
    e_g = np.abs(g - g_o).max() / np.abs(g_o).max()
    gy_n = gy.cpu().numpy().astype(np.float64)
    e_gy = np.abs(gy_n - gy_o.T).max() / np.abs(gy_o).max()
    # the MSE is a sum of squared differences of nearly equal states (the
    # student and teacher networks differ little): its FP32 error is measured
    # against the size of the cancelling terms, scale * sum |y|^2
    mag = scale * (ys_o ** 2).sum(axis=(0, 1))
    e_ll = np.abs(ll.cpu().numpy() - ll_o).max() / mag.max()
    print(f"  vs FP64 oracle: states {e_state:.2e}  weight grad {e_g:.2e}  "
          f"y0 grad {e_gy:.2e}  loss {e_ll:.2e}")
    assert e_state <= TOL32 and e_g <= TOL32 and e_gy <= TOL32 and e_ll <= TOL32
    # per trajectory, normwise (floor 1e-30), beside the scale-relative figures
    pl_s = np.linalg.norm((ys - ys_o).reshape(-1, n), axis=0) / np.maximum(
        np.linalg.norm(ys_o.reshape(-1, n), axis=0), 1e-30)
    pl_y = np.linalg.norm(gy_n - gy_o.T, axis=0) / np.maximum(np.linalg.norm(gy_o, axis=1), 1e-30)
    print(f"  per trajectory: states median {np.median(pl_s):.2e} max {pl_s.max():.2e}; "
          f"y0 grad median {np.median(pl_y):.2e} p99 {np.quantile(pl_y, 0.99):.2e} "
          f"max {pl_y.max():.2e}")
    assert pl_s.max() <= TOL32 and np.median(pl_y) <= TOL32


def test_ude_adaptive_record_states():
    n = 500
    print(f"case ude n={n} own mesh", flush=True)
    y0, th = _case(n, seed=2)
    ref = O.record(O.LV_UDE, O.TSIT5, y0, th, 0.0, T1, 1e-6, 1e-6, save_t=ST, params_shared=True)
    hd = B.ensemble_record("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                           save_times=ST, params_shared=True, steps_hint=256)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    S_g = hd.steps().cpu().numpy()
    ys = hd.y_save.cpu().numpy().astype(np.float64)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))
    e = np.abs(ys - ys_o).max() / np.abs(ys_o).max()
    print(f"  steps GPU mean {S_g.mean():.1f} oracle {ref['S'].mean():.1f}; states {e:.2e}")
    # two solutions at tolerance 1e-6 on meshes that differ by FP32 rounding
    assert e <= TOL32
    assert abs(S_g.mean() - ref["S"].mean()) <= 0.05 * ref["S"].mean()


def test_ude_solve_against_oracle():
    """The forward-only solve of the UDE (no record) against the FP64
    oracle's adaptive solve: per-trajectory normwise state error at the 20
    save times within the FP32 bar, and the same bits as the record's save
    states."""
    n = 700
    print(f"case ude solve n={n}", flush=True)
    y0, th = _case(n, seed=4)
    ref = O.record(O.LV_UDE, O.TSIT5, y0, th, 0.0, T1, 1e-6, 1e-6, save_t=ST, params_shared=True)
    ys, status = B.ensemble_solve("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                                  save_times=ST, params_shared=True)
    hd = B.ensemble_record("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                           save_times=ST, params_shared=True, steps_hint=256)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    assert torch.equal(ys, hd.y_save)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))
    d = ys.double().cpu().numpy() - ys_o
    e = np.linalg.norm(d.reshape(-1, n), axis=0) / np.maximum(
        np.linalg.norm(ys_o.reshape(-1, n), axis=0), 1e-30)
    print(f"  per-trajectory state error median {np.median(e):.2e} p99 "
          f"{np.quantile(e, 0.99):.2e} max {e.max():.2e}", flush=True)
    assert e.max() <= TOL32


def test_ude_trajectory_independent_of_its_wavefront():
    """A trajectory's record and per-trajectory gradient do not depend on the
    trajectories sharing its wavefront (they share matrix-core operations)."""
    y0, th = _case(256, seed=3)
    print("case ude alone vs in the ensemble", flush=True)
    full = B.ensemble_record("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                             save_times=ST, params_shared=True, steps_hint=256)
    _, gy_full, _ = B.ensemble_adjoint(full)
    for idx in ([0], [37, 5], list(range(64, 200))):
        sub = B.ensemble_record("ude", "tsit5", _dev(y0[idx].T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                                save_times=ST, params_shared=True, steps_hint=256)
        _, gy_sub, _ = B.ensemble_adjoint(sub)
        torch.cuda.synchronize()
        assert torch.equal(full.y_save[..., idx], sub.y_save)
        assert torch.equal(full.steps()[idx], sub.steps())
        assert torch.equal(gy_full[:, idx], gy_sub)


def test_ude_checkpointed_tape_and_determinism():
    n = 700
    print(f"case ude n={n} checkpoint 64", flush=True)
    y0, th = _case(n, seed=4)
    full = B.ensemble_record("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                             save_times=ST, params_shared=True, steps_hint=256)
    ck = B.ensemble_record("ude", "tsit5", _dev(y0.T), _dev(th), 0.0, T1, 1e-6, 1e-6,
                           save_times=ST, params_shared=True, steps_hint=256, ckpt_every=64)
    g1 = B.ensemble_adjoint(full)
    g2 = B.ensemble_adjoint(ck)
    g3 = B.ensemble_adjoint(full)
    torch.cuda.synchronize()
    assert torch.equal(full.y_save, ck.y_save)
    # same tape, same bits
    for a, c in zip(g1, g3):
        assert torch.equal(a, c)
    # per-trajectory results are the same to the bit with a checkpointed tape;
    # the weight gradient is summed across each wavefront in iteration order,
    # and the segment replays shift that order, so it agrees to FP32 rounding
    assert torch.equal(g1[1], g2[1]) and torch.equal(g1[2], g2[2])
    e = ((g1[0] - g2[0]).abs().max() / g1[0].abs().max()).item()
    print(f"  weight gradient, checkpointed vs full tape: {e:.2e}")
    assert e <= 1e-5
    assert ck.pool.numel() < full.pool.numel()


def test_ude_autograd_matches_direct_adjoint():
    n = 300
    print(f"case ude n={n} autograd", flush=True)
    y0, th = _case(n, seed=5)
    tgt = _dev(np.transpose(_targets(y0), (1, 2, 0)))
    Y0 = _dev(y0.T).requires_grad_(True)
    TH = _dev(th).requires_grad_(True)
    ys = AG.odeint("ude", "tsit5", Y0, TH, 0.0, T1, 1e-6, 1e-6, save_times=ST,
                   params_shared=True, steps_hint=256, ckpt_every="auto",
                   tape_budget_bytes=1 << 20)
    loss = ((ys - tgt) ** 2).mean()
    loss.backward()
    hd = B.ensemble_record("ude", "tsit5", Y0.detach(), TH.detach(), 0.0, T1, 1e-6, 1e-6,
                           save_times=ST, params_shared=True, steps_hint=256)
    gp, gy, ll = B.ensemble_adjoint(hd, "mse", tgt, 1.0 / (n * len(ST) * 2))
    torch.cuda.synchronize()
    assert torch.allclose(TH.grad, gp, rtol=1e-5, atol=1e-6 * gp.abs().max().item())
    assert torch.allclose(Y0.grad, gy, rtol=1e-5, atol=1e-6 * gy.abs().max().item())
