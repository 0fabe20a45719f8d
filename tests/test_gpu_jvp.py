"""GPU parity of the forward mode (ensemble_jvp) against the oracle's
dual-number replay on the same mesh.

The oracle's dual replay is pinned on the CPU against the reverse sweep and
the complex step (test_oracle_adjoint, test_oracle_rosenbrock).  Here: the
tangents of the save states (FP64: per-lane relative error <= 1e-11, in
practice 0), the loss tangent against its definition on the oracle's states
and tangents, forward against reverse on the GPU, checkpointed against full
tapes, failed lanes, FP32 (1e-4 against the FP64 oracle) and the full-size
headline launch on sampled trajectories.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import check_mesh, oracle_mesh
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"lorenz": O.LORENZ, "vdp": O.VDP, "linear": O.LINEAR, "robertson": O.ROBERTSON}
MET_O = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}
GEN = {"lorenz": W.lorenz, "vdp": W.vdp, "linear": W.damped_rotation, "robertson": W.robertson}
TOL = {"lorenz": (1e-6, 1e-8), "vdp": (1e-6, 1e-8), "linear": (1e-6, 1e-8),
       "robertson": (1e-6, 1e-10)}


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    """Per-lane normwise relative error (lanes last)."""
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def _tangents(y0, p, seed=7):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(y0.shape), rng.standard_normal(p.shape) * p


def _oracle(system, method, y0, p, dy, dp, h):
    """The oracle's dual-number replay on the mesh of the GPU record h."""
    rec = oracle_mesh(h)
    ys, dys = O.replay_dual(SYS_O[system], MET_O[method], y0, p, dy, dp, rec)
    return rec, ys, dys


@pytest.mark.parametrize("system,method,t1,n", [
    ("lorenz", "tsit5", 10.0, 1000), ("lorenz", "vern7", 10.0, 300),
    ("vdp", "tsit5", 6.3, 600), ("vdp", "vern7", 6.3, 257),
    ("linear", "tsit5", 5.0, 65), ("robertson", "rodas4", 1e5, 257),
    ("linear", "rodas4", 5.0, 63), ("robertson", "ros23", 1e5, 129),
    ("linear", "ros23", 5.0, 63),
])
def test_jvp_matches_oracle_dual_replay(system, method, t1, n):
    print(f"case jvp {system} {method} n={n}", flush=True)
    y0, p = GEN[system](n, seed=3)
    dy, dp = _tangents(y0, p)
    st = list(W.save_times(0.0, t1, 20))
    rtol, atol = TOL[system]
    # the GPU's own adaptive record; the oracle's dual replay on its mesh
    h = B.ensemble_record(system, method, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                          save_times=st, steps_hint=2048 if method == "ros23" else 512)
    ysd, ld = B.ensemble_jvp(h, _dev(dy.T), _dev(dp.T))
    torch.cuda.synchronize()
    assert np.all(h.status.cpu().numpy() == 0)
    rec, ys_o, dys_o = _oracle(system, method, y0, p, dy, dp, h)
    check_mesh(rec, O.record(SYS_O[system], MET_O[method], y0, p, 0.0, t1, rtol, atol,
                             save_t=st))
    # that mesh replayed on the GPU gives the same tangents
    cap = int(rec["S"].max())
    hr = B.ensemble_replay_mesh(system, method, _dev(y0.T), _dev(p.T), 0.0, t1,
                                _dev(rec["h"][:, :cap].T),
                                torch.tensor(rec["S"], dtype=torch.int32, device="cuda"),
                                save_times=st)
    ysd_r, ld_r = B.ensemble_jvp(hr, _dev(dy.T), _dev(dp.T))
    torch.cuda.synchronize()
    assert torch.equal(h.steps(), hr.steps())
    ref = np.transpose(dys_o, (1, 2, 0))                     # [ns, d, n]
    got = ysd.cpu().numpy()
    e = _rel(got, ref).max()
    print(f"  state tangents vs oracle: {e:.2e}")
    assert e <= 1e-11
    assert torch.equal(ysd, ysd_r) and torch.equal(ld, ld_r)
    # loss tangent: 2 sum y . ydot on the oracle's states and tangents
    l_ref = 2.0 * np.sum(ys_o * dys_o, axis=(1, 2))
    mag = 2.0 * np.sum(np.abs(ys_o * dys_o), axis=(1, 2))
    el = (np.abs(ld.cpu().numpy() - l_ref) / np.maximum(mag, 1e-300)).max()
    print(f"  loss tangent vs definition: {el:.2e}")
    assert el <= 1e-13


def test_jvp_loss_kinds():
    n = 300
    y0, p = W.lorenz(n, seed=4)
    dy, dp = _tangents(y0, p, seed=8)
    st = list(W.save_times(0.0, 3.0, 20))
    h = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 3.0, 1e-6, 1e-8,
                          save_times=st, steps_hint=256)
    torch.cuda.synchronize()
    rec, ys_o, dys_o = _oracle("lorenz", "tsit5", y0, p, dy, dp, h)
    rng = np.random.default_rng(9)
    tgt = ys_o + 0.1 * rng.standard_normal(ys_o.shape)
    cot = rng.standard_normal(ys_o.shape)
    scale = 1.0 / (n * 20 * 3)
    _, l_mse = B.ensemble_jvp(h, _dev(dy.T), _dev(dp.T), loss="mse",
                              data=_dev(np.transpose(tgt, (1, 2, 0))), scale=scale,
                              want_states=False)
    _, l_cot = B.ensemble_jvp(h, _dev(dy.T), _dev(dp.T), loss="cotangent",
                              data=_dev(np.transpose(cot, (1, 2, 0))), want_states=False)
    torch.cuda.synchronize()
    r_mse = 2.0 * scale * np.sum((ys_o - tgt) * dys_o, axis=(1, 2))
    m_mse = 2.0 * scale * np.sum(np.abs((ys_o - tgt) * dys_o), axis=(1, 2))
    r_cot = np.sum(cot * dys_o, axis=(1, 2))
    m_cot = np.sum(np.abs(cot * dys_o), axis=(1, 2))
    assert (np.abs(l_mse.cpu().numpy() - r_mse) / m_mse).max() <= 1e-13
    assert (np.abs(l_cot.cpu().numpy() - r_cot) / m_cot).max() <= 1e-13


@pytest.mark.parametrize("system,method,t1", [("lorenz", "tsit5", 10.0),
                                              ("robertson", "rodas4", 1e5),
                                              ("robertson", "ros23", 1e5)])
def test_forward_passes_equal_reverse_gradient(system, method, t1):
    """One pass per input with the same unit tangent in every trajectory gives
    every trajectory's gradient: P + d passes against one reverse sweep."""
    n = 512
    print(f"case jvp forward vs reverse {system}", flush=True)
    y0, p = GEN[system](n, seed=5)
    rtol, atol = TOL[system]
    st = list(W.save_times(0.0, t1, 20))
    h = B.ensemble_record(system, method, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                          save_times=st, steps_hint=2048 if method == "ros23" else 512)
    gp, gy, ll = B.ensemble_adjoint(h)
    d, npar = y0.shape[1], p.shape[1]
    for k in range(npar + d):
        dp = torch.zeros((npar, n), dtype=torch.float64, device="cuda")
        dy = torch.zeros((d, n), dtype=torch.float64, device="cuda")
        if k < npar:
            dp[k] = 1.0
        else:
            dy[k - npar] = 1.0
        _, ld = B.ensemble_jvp(h, dy, dp, want_states=False)
        ref = gp[k] if k < npar else gy[k - npar]
        torch.cuda.synchronize()
        err = ((ld - ref).abs().max() / ref.abs().max()).item()
        print(f"  input {k}: forward vs reverse {err:.2e}")
        assert err <= 1e-9


@pytest.mark.parametrize("system,method,t1,st,cluster", [
    # a save at t0, a repeated save time, four saves inside one step, one at t1
    ("lorenz", "tsit5", 3.0, [0.0, 0.5, 0.5, 1.0, 1.0 + 1e-4, 1.0 + 2e-4, 1.0 + 3e-4, 3.0], 3),
    ("robertson", "rodas4", 1e5, [0.0, 1e-3, 1e-3, 10.0, 4e4, 4e4 + 1.0, 4e4 + 2.0, 1e5], 4),
])
def test_jvp_save_order_edges(system, method, t1, st, cluster):
    """Save steps and mesh steps share the pass's loop, one step a trip:
    saves whose base is the same mesh point (a save at t0, repeated and
    clustered save times) are taken in save order before the next mesh
    step, and saves at t1 after the last one."""
    n = 200 if system == "lorenz" else 129
    print(f"case jvp save edges {system} {method} n={n}", flush=True)
    y0, p = GEN[system](n, seed=12)
    dy, dp = _tangents(y0, p, seed=13)
    rtol, atol = TOL[system]
    h = B.ensemble_record(system, method, _dev(y0.T), _dev(p.T), 0.0, t1, rtol, atol,
                          save_times=st, steps_hint=512)
    ysd, ld = B.ensemble_jvp(h, _dev(dy.T), _dev(dp.T))
    torch.cuda.synchronize()
    assert np.all(h.status.cpu().numpy() == 0)
    rec, ys_o, dys_o = _oracle(system, method, y0, p, dy, dp, h)
    si = rec["save_idx"]
    # the cases this test is for occur: a save at t0 (base index 0, offset 0),
    # saves sharing a base point, and saves at t1 (base index S)
    assert np.all(si[:, 0] == 0) and np.all(rec["save_dt"][:, 0] == 0.0)
    assert np.all(si[:, 1] == si[:, 2])
    assert np.mean(si[:, cluster] == si[:, cluster + 2]) > 0.5
    assert np.all(si[:, -1] == rec["S"])
    e = _rel(ysd.cpu().numpy(), np.transpose(dys_o, (1, 2, 0))).max()
    print(f"  state tangents vs oracle: {e:.2e}")
    assert e <= 1e-11
    l_ref = 2.0 * np.sum(ys_o * dys_o, axis=(1, 2))
    mag = 2.0 * np.sum(np.abs(ys_o * dys_o), axis=(1, 2))
    assert (np.abs(ld.cpu().numpy() - l_ref) / np.maximum(mag, 1e-300)).max() <= 1e-13


def test_jvp_checkpointed_tape_and_failed_lanes():
    n = 700
    y0, p = W.lorenz(n, seed=6)
    dy, dp = _tangents(y0, p)
    st = list(W.save_times(0.0, 10.0, 20))
    args = ("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, 1e-6, 1e-8)
    full = B.ensemble_record(*args, save_times=st, steps_hint=512)
    ck = B.ensemble_record(*args, save_times=st, steps_hint=512, ckpt_every=16)
    a = B.ensemble_jvp(full, _dev(dy.T), _dev(dp.T))
    b = B.ensemble_jvp(ck, _dev(dy.T), _dev(dp.T))
    # a trial budget far too small: every lane fails, every tangent is NaN
    bad = B.ensemble_record(*args, save_times=st, steps_hint=512, max_steps=40)
    c = B.ensemble_jvp(bad, _dev(dy.T), _dev(dp.T))
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert np.all(bad.status.cpu().numpy() != 0)
    assert torch.isnan(c[0]).all() and torch.isnan(c[1]).all()


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_jvp_ragged_sizes(n):
    y0, p = W.vdp(n, seed=10)
    dy, dp = _tangents(y0, p)
    st = list(W.save_times(0.0, 6.3, 20))
    h = B.ensemble_record("vdp", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 6.3, 1e-6, 1e-8,
                          save_times=st, steps_hint=256)
    ysd, _ = B.ensemble_jvp(h, _dev(dy.T), _dev(dp.T))
    torch.cuda.synchronize()
    rec, ys_o, dys_o = _oracle("vdp", "tsit5", y0, p, dy, dp, h)
    assert _rel(ysd.cpu().numpy(), np.transpose(dys_o, (1, 2, 0))).max() <= 1e-11


def test_jvp_fp32_against_fp64_oracle():
    """FP32 tangents against the FP64 oracle's dual replay on the GPU's mesh
    (Lorenz on [0, 2]: on [0, 10] chaos amplifies FP32 rounding past 1e-4)."""
    n = 400
    y0, p = W.lorenz(n, seed=11)
    y0 = y0.astype(np.float32).astype(np.float64)
    p = p.astype(np.float32).astype(np.float64)
    dy, dp = _tangents(y0, p)
    dy = dy.astype(np.float32).astype(np.float64)
    dp = dp.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, 2.0, 20))
    f32 = torch.float32
    h = B.ensemble_record("lorenz", "tsit5", _dev(y0.T, f32), _dev(p.T, f32), 0.0, 2.0, 1e-6,
                          1e-8, save_times=st, steps_hint=256)
    ysd, _ = B.ensemble_jvp(h, _dev(dy.T, f32), _dev(dp.T, f32))
    torch.cuda.synchronize()
    _, dys_o = O.replay_dual(O.LORENZ, O.TSIT5, y0, p, dy, dp, oracle_mesh(h))
    ref = np.transpose(dys_o, (1, 2, 0))
    got = ysd.cpu().numpy().astype(np.float64)
    sc = np.sqrt(np.mean(np.sum(ref.reshape(-1, n) ** 2, axis=0)))
    num = np.linalg.norm((got - ref).reshape(-1, n), axis=0)
    den = np.maximum(np.linalg.norm(ref.reshape(-1, n), axis=0), sc)
    e = (num / den).max()
    print(f"  FP32 tangents vs FP64 oracle: {e:.2e}")
    assert e <= 1e-4


def test_jvp_rejects_unsupported():
    y0, p = W.hires(8, seed=0)
    h = B.ensemble_record("hires", "rodas4", _dev(y0.T), _dev(p.T), 0.0, 321.8122, 1e-6, 1e-10,
                          steps_hint=512)
    with pytest.raises(RuntimeError, match="forward mode"):
        B.ensemble_jvp(h)
    y0, p = W.lorenz(8, seed=0)
    hs = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p[0]), 0.0, 1.0, 1e-6, 1e-8,
                           params_shared=True, steps_hint=128)
    with pytest.raises(RuntimeError, match="per-trajectory"):
        B.ensemble_jvp(hs)
    torch.cuda.synchronize()


def test_jvp_full_size_sampled():
    """The launch the bench times: 2^20 Lorenz trajectories on [0, 10], one
    tangent pass, 64 sampled trajectories against the oracle's dual replay."""
    n = 1 << 20
    print(f"case jvp full size n={n}", flush=True)
    y0, p = W.lorenz(n, seed=0)
    st = list(W.save_times(0.0, 10.0, 20))
    from test_gpu_fullsize import _planned_record
    rec = _planned_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 10.0, 1e-6, 1e-8, st)
    rng = np.random.default_rng(12)
    dp = rng.standard_normal(p.shape) * p
    ysd, ld = B.ensemble_jvp(rec, None, _dev(dp.T))
    torch.cuda.synchronize()
    assert np.all(rec.status.cpu().numpy() == 0)
    idx = np.sort(np.random.default_rng(1).choice(n, 64, replace=False))
    idx[0], idx[-1] = 0, n - 1
    ref_rec = oracle_mesh(rec, idx)
    check_mesh(ref_rec, O.record(O.LORENZ, O.TSIT5, y0[idx], p[idx], 0.0, 10.0, 1e-6, 1e-8,
                                 save_t=st))
    ys_o, dys_o = O.replay_dual(O.LORENZ, O.TSIT5, y0[idx], p[idx], np.zeros_like(y0[idx]),
                                dp[idx], ref_rec)
    got = ysd.cpu().numpy()[..., idx]
    e = _rel(got, np.transpose(dys_o, (1, 2, 0))).max()
    l_ref = 2.0 * np.sum(ys_o * dys_o, axis=(1, 2))
    el = (np.abs(ld.cpu().numpy()[idx] - l_ref) /
          (2.0 * np.sum(np.abs(ys_o * dys_o), axis=(1, 2)))).max()
    print(f"  sampled: state tangents {e:.2e} loss tangent {el:.2e}")
    assert e <= 1e-11 and el <= 1e-13
