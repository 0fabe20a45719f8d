"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Gradients are compared on the same mesh (paper, Appendix B.6 shared-mesh
check): the oracle run on the GPU's own adaptive mesh, and the oracle's mesh
replayed on the GPU.  The two adaptive meshes themselves are compared by
statistics (equal step counts on >= 99.9 % of trajectories, step sizes to a
stated relative bound where they agree).  Bar (FP64): per-lane normwise
relative error <= 1e-11 for states and gradients; FP32: 1e-4 against the
FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import check_mesh, oracle_mesh
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SYS_O = {"lorenz": O.LORENZ, "vdp": O.VDP, "linear": O.LINEAR}
MET_O = {"tsit5": O.TSIT5, "vern7": O.VERN7}
TOL64 = 1e-11
TOL32 = 1e-4


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _case(system, n, seed=0):
    gen = {"lorenz": W.lorenz, "vdp": W.vdp, "linear": W.damped_rotation}[system]
    return gen(n, seed)


def _rel(a, b):
    """Per-lane normwise relative error along axis 0 (lanes last)."""
    num = np.linalg.norm((a - b).reshape(-1, a.shape[-1]), axis=0)
    den = np.linalg.norm(b.reshape(-1, b.shape[-1]), axis=0)
    return num / np.maximum(den, 1e-300)


def _gpu_record(system, method, y0, p, t1, rtol, atol, st, dtype=torch.float64, **kw):
    h = B.ensemble_record(system, method, _dev(y0.T, dtype), _dev(p.T, dtype), 0.0, t1, rtol,
                          atol, save_times=st, **kw)
    return h


def _oracle_mesh_to_gpu(rec, n):
    S = rec["S"]
    cap = max(1, int(S.max()))
    h = np.ascontiguousarray(rec["h"][:, :cap].T)
    return _dev(h), torch.tensor(S, dtype=torch.int32, device="cuda")


CASES = [
    # system, method, n, t1, rtol, atol, n_save
    ("lorenz", "tsit5", 1024, 1.0, 1e-6, 1e-8, 0),     # the small parity workload
    ("lorenz", "tsit5", 1000, 10.0, 1e-6, 1e-8, 20),   # headline shape, ragged n
    ("lorenz", "vern7", 777, 10.0, 1e-8, 1e-8, 20),
    ("vdp", "tsit5", 513, 6.3, 1e-6, 1e-8, 20),
    ("vdp", "vern7", 300, 6.3, 1e-8, 1e-8, 20),
    ("linear", "tsit5", 129, 8.0, 1e-7, 1e-9, 5),
]


@pytest.mark.parametrize("system,method,n,t1,rtol,atol,ns", CASES)
def test_record_and_adjoint_match_oracle(system, method, n, t1, rtol, atol, ns):
    print(f"case {system} {method} n={n} t1={t1} rtol={rtol}", flush=True)
    y0, p = _case(system, n)
    st = list(W.save_times(0.0, t1, ns)) if ns else None
    so, mo = SYS_O[system], MET_O[method]
    ref = O.record(so, mo, y0, p, 0.0, t1, rtol, atol, save_t=st)
    assert np.all(ref["status"] == O.ST_OK)
    gp_o, gy_o, ll_o = O.adjoint(so, mo, y0, p, ref)

    # 1) the GPU's adaptive record: its mesh against the oracle's by the
    # statistics, then states and gradients against the oracle on the GPU's mesh
    hd = _gpu_record(system, method, y0, p, t1, rtol, atol, st, steps_hint=int(ref["S"].max()) + 16)
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    gm = oracle_mesh(hd)
    check_mesh(gm, ref)
    ys_g = O.replay(so, mo, y0, p, gm)
    gp_g, gy_g, ll_g = O.adjoint(so, mo, y0, p, gm)
    ys = hd.y_save.cpu().numpy()                      # [ns, d, n]
    gp_n, gy_n = gp.cpu().numpy(), gy.cpu().numpy()
    e_state = _rel(ys, np.transpose(ys_g, (1, 2, 0)))
    e_gp = _rel(gp_n, gp_g.T)
    e_gy = _rel(gy_n, gy_g.T)
    print(f"  own mesh: max rel err states {e_state.max():.2e} grad_p {e_gp.max():.2e} grad_y0 {e_gy.max():.2e}")
    assert e_state.max() <= TOL64 and e_gp.max() <= TOL64 and e_gy.max() <= TOL64
    assert np.allclose(ll.cpu().numpy(), ll_g, rtol=1e-13, atol=0)
    ys_o = np.transpose(ref["y_save"], (1, 2, 0))

    # 2) the oracle's mesh replayed on the GPU, every lane
    h_dev, S_dev = _oracle_mesh_to_gpu(ref, n)
    hf = B.ensemble_replay_mesh(system, method, _dev(y0.T), _dev(p.T), 0.0, t1, h_dev, S_dev,
                                save_times=st)
    gp2, gy2, ll2 = B.ensemble_adjoint(hf)
    torch.cuda.synchronize()
    e_state = _rel(hf.y_save.cpu().numpy(), ys_o)
    e_gp = _rel(gp2.cpu().numpy(), gp_o.T)
    e_gy = _rel(gy2.cpu().numpy(), gy_o.T)
    print(f"  oracle mesh: max rel err states {e_state.max():.2e} grad_p {e_gp.max():.2e} grad_y0 {e_gy.max():.2e}")
    assert e_state.max() <= TOL64 and e_gp.max() <= TOL64 and e_gy.max() <= TOL64


@pytest.mark.parametrize("system,method", [("lorenz", "tsit5"), ("vdp", "vern7")])
def test_fp32_against_fp64_oracle(system, method):
    n, t1 = 512, (2.0 if system == "lorenz" else 6.3)
    y0, p = _case(system, n, seed=3)
    y0 = y0.astype(np.float32).astype(np.float64)
    p = p.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, t1, 10))
    so, mo = SYS_O[system], MET_O[method]
    ref = O.record(so, mo, y0, p, 0.0, t1, 1e-6, 1e-8, save_t=st)
    gp_o, gy_o, _ = O.adjoint(so, mo, y0, p, ref)
    # FP32 replay of the FP64 oracle's mesh: same mesh, single precision
    h_dev, S_dev = _oracle_mesh_to_gpu(ref, n)
    hf = B.ensemble_replay_mesh(system, method, _dev(y0.T, torch.float32), _dev(p.T, torch.float32),
                                0.0, t1, h_dev, S_dev, save_times=st)
    gp, gy, _ = B.ensemble_adjoint(hf)
    torch.cuda.synchronize()
    e_s = _rel(hf.y_save.double().cpu().numpy(), np.transpose(ref["y_save"], (1, 2, 0)))
    g32, g64 = gp.double().cpu().numpy(), gp_o.T
    e_g = _rel(g32, g64)
    # a lane whose gradient nearly vanishes has no meaningful relative error:
    # scale each lane's error by max(|g_lane|, RMS of |g| over the ensemble)
    gn = np.linalg.norm(g64, axis=0)
    e_gs = np.linalg.norm(g32 - g64, axis=0) / np.maximum(gn, np.sqrt(np.mean(gn ** 2)))
    print(f"fp32 {system} {method}: states max {e_s.max():.2e}; grad per-lane median "
          f"{np.median(e_g):.2e} p99 {np.quantile(e_g, 0.99):.2e} max {e_g.max():.2e}; "
          f"ensemble-scaled max {e_gs.max():.2e}")
    assert e_s.max() <= TOL32 and e_gs.max() <= TOL32 and np.median(e_g) <= TOL32


def test_solve_matches_record_states():
    y0, p = _case("lorenz", 4096, seed=1)
    st = list(W.save_times(0.0, 10.0, 20))
    ys, status = B.ensemble_solve("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, 1e-6, 1e-8,
                                  save_times=st)
    hd = _gpu_record("lorenz", "tsit5", y0, p, 10.0, 1e-6, 1e-8, st, steps_hint=400)
    torch.cuda.synchronize()
    assert torch.equal(status, hd.status)
    assert torch.equal(ys, hd.y_save)


SOLVE_CASES = [
    # system, method, dtype, n, t1, rtol, atol, bound on the per-trajectory
    # state error against the oracle's adaptive solve (FP64: the meshes may
    # differ by ulps of h, which the states carry with their own
    # sensitivity; FP32: the single-precision bar)
    ("lorenz", "tsit5", "f64", 1024, 1.0, 1e-6, 1e-8, 1e-11),
    ("lorenz", "tsit5", "f64", 1000, 10.0, 1e-6, 1e-8, 1e-9),
    ("lorenz", "vern7", "f64", 500, 10.0, 1e-8, 1e-8, 1e-9),
    ("vdp", "tsit5", "f64", 700, 6.3, 1e-6, 1e-8, 1e-11),
    ("vdp", "vern7", "f64", 700, 6.3, 1e-8, 1e-8, 1e-11),
    ("lorenz", "tsit5", "f32", 512, 1.0, 1e-6, 1e-8, 1e-4),
    ("lorenz", "vern7", "f32", 512, 1.0, 1e-6, 1e-8, 1e-4),
    ("vdp", "tsit5", "f32", 512, 6.3, 1e-6, 1e-8, 1e-4),
    ("vdp", "vern7", "f32", 512, 6.3, 1e-6, 1e-8, 1e-4),
]


@pytest.mark.parametrize("system,method,dt,n,t1,rtol,atol,tol", SOLVE_CASES)
def test_solve_matches_oracle(system, method, dt, n, t1, rtol, atol, tol):
    """The forward-only solve (no record) against the oracle's adaptive
    solve on the same inputs (FP32 inputs rounded first): states at 20 save
    times, per trajectory, normwise.  Also the same bits as the record's
    save states."""
    print(f"case solve {system} {method} {dt} n={n} t1={t1}", flush=True)
    y0, p = _case(system, n, seed=31)
    tdt = torch.float64 if dt == "f64" else torch.float32
    if dt == "f32":
        y0 = y0.astype(np.float32).astype(np.float64)
        p = p.astype(np.float32).astype(np.float64)
    st = list(W.save_times(0.0, t1, 20))
    ref = O.record(SYS_O[system], MET_O[method], y0, p, 0.0, t1, rtol, atol, save_t=st)
    ys, status = B.ensemble_solve(system, method, _dev(y0.T, tdt), _dev(p.T, tdt), 0.0, t1, rtol,
                                  atol, save_times=st)
    hd = _gpu_record(system, method, y0, p, t1, rtol, atol, st, dtype=tdt,
                     steps_hint=int(ref["S"].max()) + 16)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    assert torch.equal(ys, hd.y_save) and torch.equal(status, hd.status)
    e = _rel(ys.double().cpu().numpy(), np.transpose(ref["y_save"], (1, 2, 0)))
    print(f"  per-trajectory state error median {np.median(e):.2e} p99 "
          f"{np.quantile(e, 0.99):.2e} max {e.max():.2e}", flush=True)
    assert e.max() <= tol


def test_mesh_roundtrip_and_determinism():
    n = 2000
    y0, p = _case("lorenz", n, seed=2)
    st = list(W.save_times(0.0, 10.0, 20))
    a = _gpu_record("lorenz", "tsit5", y0, p, 10.0, 1e-6, 1e-8, st, steps_hint=400)
    b = _gpu_record("lorenz", "tsit5", y0, p, 10.0, 1e-6, 1e-8, st, steps_hint=400)
    ga = B.ensemble_adjoint(a)
    gb = B.ensemble_adjoint(b)
    torch.cuda.synchronize()
    assert torch.equal(a.y_save, b.y_save) and torch.equal(a.steps(), b.steps())
    for x, y in zip(ga, gb):
        assert torch.equal(x, y)
    # export the mesh into a wider rectangle (entries past S are ignored) and
    # replay it: identical results
    h, S = B.ensemble_mesh_export(a)
    cap = h.shape[0] + 5
    hp = torch.zeros((cap, n), dtype=torch.float64, device="cuda")
    hp[: h.shape[0]] = h
    r = B.ensemble_replay_mesh("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, hp, S,
                               save_times=st)
    gr = B.ensemble_adjoint(r)
    torch.cuda.synchronize()
    assert torch.equal(r.y_save, a.y_save)
    for x, y in zip(ga, gr):
        assert torch.equal(x, y)


@pytest.mark.parametrize("system,method,dtype,n", [
    ("lorenz", "tsit5", "f64", 1), ("lorenz", "tsit5", "f64", 7), ("lorenz", "tsit5", "f64", 65),
    ("lorenz", "tsit5", "f32", 71), ("vdp", "vern7", "f64", 136), ("linear", "tsit5", "f32", 9)])
def test_cooperative_tape_small_wavefronts(system, method, dtype, n):
    """The explicit pairs' record writes its tape a wavefront at a time, eight
    lanes to a group of four records; a wavefront with fewer live lanes than a
    group has chunks (n mod 64 < 8 in the last one) writes each lane's groups
    itself.  At such sizes the tape must hold exactly the record's mesh and
    base states: replaying the exported mesh (whose tape each lane writes on
    its own) gives the same save states and gradients to the bit, and in FP64
    the oracle on the GPU's mesh agrees within 1e-11."""
    print(f"case cooperative tape {system} {method} {dtype} n={n}", flush=True)
    y0, p = _case(system, n, seed=n)
    t1 = {"lorenz": 10.0, "vdp": 6.3, "linear": 8.0}[system]
    st = list(W.save_times(0.0, t1, 20))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    hd = _gpu_record(system, method, y0, p, t1, 1e-6, 1e-8, st, dtype=tdt)
    gp, gy, ll = B.ensemble_adjoint(hd, want_loss=True)
    h, S = B.ensemble_mesh_export(hd)
    hr = B.ensemble_replay_mesh(system, method, _dev(y0.T, tdt), _dev(p.T, tdt), 0.0, t1, h, S,
                                save_times=st)
    gp2, gy2, ll2 = B.ensemble_adjoint(hr, want_loss=True)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0) and np.all(hr.status.cpu().numpy() == 0)
    assert torch.equal(hd.y_save, hr.y_save)
    assert torch.equal(gp, gp2) and torch.equal(gy, gy2) and torch.equal(ll, ll2)
    if dtype == "f64":
        so, mo = SYS_O[system], MET_O[method]
        gm = oracle_mesh(hd)
        ys_g = O.replay(so, mo, y0, p, gm)
        gp_g, gy_g, _ = O.adjoint(so, mo, y0, p, gm)
        e = (_rel(hd.y_save.cpu().numpy(), np.transpose(ys_g, (1, 2, 0))).max(),
             _rel(gp.cpu().numpy(), gp_g.T).max(), _rel(gy.cpu().numpy(), gy_g.T).max())
        print(f"  own mesh vs oracle: states {e[0]:.2e} grad_p {e[1]:.2e} grad_y0 {e[2]:.2e}")
        assert max(e) <= TOL64


def test_loss_kinds_match_oracle():
    n, t1 = 300, 3.0
    y0, p = _case("lorenz", n, seed=4)
    st = list(W.save_times(0.0, t1, 6))
    ref = O.record(O.LORENZ, O.TSIT5, y0, p, 0.0, t1, 1e-6, 1e-8, save_t=st)
    h_dev, S_dev = _oracle_mesh_to_gpu(ref, n)
    hf = B.ensemble_replay_mesh("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, t1, h_dev, S_dev,
                                save_times=st)
    rng = np.random.default_rng(9)
    tgt = ref["y_save"] + rng.normal(size=ref["y_save"].shape)
    for kind, okind, data, scale in (("mse", O.LOSS_MSE_TARGET, tgt, 0.37),
                                     ("cotangent", O.LOSS_COTANGENT, tgt, 1.0)):
        gp_o, gy_o, ll_o = O.adjoint(O.LORENZ, O.TSIT5, y0, p, ref, okind, data, scale)
        gp, gy, ll = B.ensemble_adjoint(hf, kind, _dev(np.transpose(data, (1, 2, 0))), scale)
        torch.cuda.synchronize()
        assert _rel(gp.cpu().numpy(), gp_o.T).max() <= TOL64
        assert _rel(gy.cpu().numpy(), gy_o.T).max() <= TOL64
        if kind == "mse":
            assert np.allclose(ll.cpu().numpy(), ll_o, rtol=1e-13)


def test_lane_failures_are_isolated():
    n = 256
    y0, p = _case("lorenz", n, seed=5)
    p[7, 1] = np.nan
    # tiny trial budget for the whole ensemble
    hd = _gpu_record("lorenz", "tsit5", y0, p, 1.0, 1e-6, 1e-8, None, max_steps=5, steps_hint=32)
    torch.cuda.synchronize()
    s = hd.status.cpu().numpy()
    assert s[7] == B.A.LANE_NONFINITE
    assert np.all(np.delete(s, 7) == B.A.LANE_MAX_STEPS)
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    assert torch.isnan(gp).all()
    # a pool with too few pages: some lanes run out, the others finish and
    # agree bit for bit with a run that had room for everyone
    y0, p = _case("lorenz", n, seed=6)
    full = _gpu_record("lorenz", "tsit5", y0, p, 1.0, 1e-6, 1e-8, None, steps_hint=128)
    g_full = B.ensemble_adjoint(full)[0]
    # 3 reserved pages (48 steps) each and an overflow area for 3/8 of the
    # lanes; every lane needs a 4th page (about 55 steps)
    nbytes = B.ensemble_record_bytes("lorenz", "tsit5", n, 0.0, 1.0, 48)
    pool = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    hd = _gpu_record("lorenz", "tsit5", y0, p, 1.0, 1e-6, 1e-8, None, pool=pool, steps_per_traj=48)
    gp, gy, ll = B.ensemble_adjoint(hd)
    torch.cuda.synchronize()
    s = hd.status.cpu().numpy()
    assert np.all(full.status.cpu().numpy() == 0)
    assert 0 < np.sum(s == B.A.LANE_NOSPACE) < n
    ok = torch.tensor(s == 0, device="cuda")
    assert torch.equal(gp[:, ok], g_full[:, ok])
    assert torch.isnan(gp[:, ~ok]).all()
    assert torch.isnan(hd.y_save[:, :, ~ok]).all()


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_small_and_ragged_sizes(n):
    y0, p = _case("vdp", n, seed=n)
    st = [0.0, 1.0, 1.0, 3.15, 6.3]   # a save at t0 and a repeated save time
    ref = O.record(O.VDP, O.TSIT5, y0, p, 0.0, 6.3, 1e-6, 1e-8, save_t=st)
    gp_o, gy_o, _ = O.adjoint(O.VDP, O.TSIT5, y0, p, ref)
    h_dev, S_dev = _oracle_mesh_to_gpu(ref, n)
    hf = B.ensemble_replay_mesh("vdp", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 6.3, h_dev, S_dev,
                                save_times=st)
    gp, gy, _ = B.ensemble_adjoint(hf)
    torch.cuda.synchronize()
    assert _rel(hf.y_save.cpu().numpy(), np.transpose(ref["y_save"], (1, 2, 0))).max() <= TOL64
    assert _rel(gp.cpu().numpy(), gp_o.T).max() <= TOL64
    assert _rel(gy.cpu().numpy(), gy_o.T).max() <= TOL64


@pytest.mark.parametrize("method", ["tsit5", "vern7"])
def test_save_states_from_overflow_pages(method):
    """Most taped steps in overflow pages (two reserved pages per trajectory):
    the save states the separate save kernel forms from bases reached through
    the page links, and the sweep's gradients, against the oracle."""
    n, t1 = 300, 10.0
    y0, p = W.lorenz(n, seed=21)
    st = list(W.save_times(0.0, t1, 20))
    print(f"case overflow pages lorenz {method} n={n}", flush=True)
    ref = O.record(O.LORENZ, MET_O[method], y0, p, 0.0, t1, 1e-6, 1e-8, save_t=st)
    nbytes = B.ensemble_record_bytes("lorenz", method, n, 0.0, t1, 3 * int(ref["S"].max()), 20)
    pool = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    hd = _gpu_record("lorenz", method, y0, p, t1, 1e-6, 1e-8, st, pool=pool, steps_per_traj=32)
    gp, gy, _ = B.ensemble_adjoint(hd)
    stats = B.ensemble_record_stats(hd)
    torch.cuda.synchronize()
    assert np.all(hd.status.cpu().numpy() == 0)
    assert stats["overflow_pages_used"] > 4 * n   # most pages are overflow pages
    # the oracle on the GPU's mesh (read back through the page links)
    gm = oracle_mesh(hd)
    check_mesh(gm, ref)
    gp_o, gy_o, _ = O.adjoint(O.LORENZ, MET_O[method], y0, p, gm)
    ys = hd.y_save.cpu().numpy()
    ys_o = np.transpose(O.replay(O.LORENZ, MET_O[method], y0, p, gm), (1, 2, 0))
    e = (_rel(ys, ys_o).max(), _rel(gp.cpu().numpy(), gp_o.T).max(),
         _rel(gy.cpu().numpy(), gy_o.T).max())
    print(f"  overflow pages {stats['overflow_pages_used']}; max rel err {e}")
    assert max(e) <= TOL64
