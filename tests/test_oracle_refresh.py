"""Pins for the oracle's mesh refresh (the mesh-drift policy: the paper's
stated future work for long fits, Section 5, of re-recording only what
drifted).  A refresh replays each trajectory's old mesh at new inputs,
keeps every old step whose error estimate stays within `slack`, and at the
first one that fails goes on with the adaptive controller (that trial
counting as rejected).

* at the inputs the mesh was recorded with, every step is kept and the
  result is the record itself, bit for bit, for every method;
* an empty old mesh gives exactly a fresh record;
* an unbounded slack gives exactly the frozen-mesh replay;
* refreshing a refreshed mesh at the same inputs keeps every step;
* a stricter slack leaves the old mesh no later, and the kept prefix is the
  old mesh itself;
* on the damped rotation, whose exact solution is known, a refresh after a
  large parameter change restores the tolerance that the stale mesh loses.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from paper_2609_02876_amd import workloads as W
from oracle_helpers import rot_matrix

CASES = [
    ("lorenz", O.LORENZ, O.TSIT5, 10.0, 1e-6, 1e-8),
    ("lorenz", O.LORENZ, O.VERN7, 3.0, 1e-8, 1e-10),
    ("vdp", O.VDP, O.TSIT5, 6.3, 1e-6, 1e-8),
    ("robertson", O.ROBERTSON, O.RODAS, 1e5, 1e-6, 1e-10),
    ("robertson", O.ROBERTSON, O.ROS23, 1e4, 1e-5, 1e-9),
]
KEYS = ("h", "S", "status", "save_idx", "save_dt", "y_save")


def _inputs(name, n, seed):
    return W.GENERATORS[name](n, seed=seed)


def _same(a, b, keys=KEYS):
    for k in keys:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        if k == "h":
            c = min(x.shape[1], y.shape[1])
            x, y = x[:, :c], y[:, :c]
        assert np.array_equal(x, y, equal_nan=True), k


@pytest.mark.parametrize("name,sys_,meth,t1,rtol,atol", CASES)
def test_refresh_at_the_recorded_inputs_is_the_record(name, sys_, meth, t1, rtol, atol):
    y0, p = _inputs(name, 48, 1)
    st = list(W.save_times(0.0, t1, 20))
    rec = O.record(sys_, meth, y0, p, 0.0, t1, rtol, atol, save_t=st, cap=8192)
    ref = O.refresh(sys_, meth, y0, p, 0.0, t1, rtol, atol, rec, save_t=st, cap=8192)
    assert np.all(rec["status"] == O.ST_OK)
    assert np.array_equal(ref["drift_at"], rec["S"])
    assert np.array_equal(ref["n_trial"], rec["S"])     # no rejected trial
    _same(ref, rec)


@pytest.mark.parametrize("name,sys_,meth,t1,rtol,atol", CASES)
def test_refresh_of_an_empty_mesh_is_a_fresh_record(name, sys_, meth, t1, rtol, atol):
    y0, p = _inputs(name, 24, 2)
    st = list(W.save_times(0.0, t1, 5))
    empty = dict(h=np.zeros((24, 1)), S=np.zeros(24, np.int32))
    ref = O.refresh(sys_, meth, y0, p, 0.0, t1, rtol, atol, empty, save_t=st, cap=8192)
    rec = O.record(sys_, meth, y0, p, 0.0, t1, rtol, atol, save_t=st, cap=8192)
    _same(ref, rec)
    assert np.array_equal(ref["n_trial"], rec["n_trial"]) and np.all(ref["drift_at"] == 0)


@pytest.mark.parametrize("name,sys_,meth,t1,rtol,atol", CASES)
def test_unbounded_slack_is_the_frozen_replay(name, sys_, meth, t1, rtol, atol):
    y0, p = _inputs(name, 24, 3)
    st = list(W.save_times(0.0, t1, 20))
    rec = O.record(sys_, meth, y0, p, 0.0, t1, rtol, atol, save_t=st, cap=8192)
    p2 = p * (1.0 + 0.05 * np.random.default_rng(3).standard_normal(p.shape))
    ref = O.refresh(sys_, meth, y0, p2, 0.0, t1, rtol, atol, rec, save_t=st, slack=np.inf,
                    cap=8192)
    assert np.array_equal(ref["S"], rec["S"]) and np.array_equal(ref["drift_at"], rec["S"])
    assert np.array_equal(ref["h"][:, :rec["h"].shape[1]], rec["h"])
    assert np.array_equal(ref["y_save"], O.replay(sys_, meth, y0, p2, rec))


@pytest.mark.parametrize("name,sys_,meth,t1,rtol,atol", CASES)
def test_refresh_is_idempotent_and_keeps_the_old_prefix(name, sys_, meth, t1, rtol, atol):
    n = 48
    y0, p = _inputs(name, n, 4)
    st = list(W.save_times(0.0, t1, 20))
    rec = O.record(sys_, meth, y0, p, 0.0, t1, rtol, atol, save_t=st, cap=8192)
    p2 = p * (1.0 + 0.1 * np.random.default_rng(4).standard_normal(p.shape))
    r1 = O.refresh(sys_, meth, y0, p2, 0.0, t1, rtol, atol, rec, save_t=st, cap=8192)
    r_strict = O.refresh(sys_, meth, y0, p2, 0.0, t1, rtol, atol, rec, save_t=st, slack=0.5,
                         cap=8192)
    assert np.all(r1["status"] == O.ST_OK)
    k = r1["drift_at"]
    assert np.any(k < rec["S"]), "the perturbation should move some meshes"
    for l in range(n):
        assert np.array_equal(r1["h"][l, :k[l]], rec["h"][l, :k[l]])
    assert np.all(r_strict["drift_at"] <= k)
    r2 = O.refresh(sys_, meth, y0, p2, 0.0, t1, rtol, atol, r1, save_t=st, cap=8192)
    assert np.array_equal(r2["drift_at"], r1["S"])
    _same(r2, r1)


def test_refresh_restores_the_tolerance_on_the_damped_rotation():
    n, t1, rtol = 16, 8.0, 1e-7
    rng = np.random.default_rng(5)
    y0 = rng.normal(size=(n, 2))
    a = 0.05 + 0.1 * rng.random(n)
    old = O.record(O.LINEAR, O.TSIT5, y0, np.stack([a, np.full(n, 1.0)], 1), 0.0, t1, rtol,
                   rtol * 1e-2)
    p2 = np.stack([a, np.full(n, 4.0)], 1)          # four times the rotation rate
    fresh = O.record(O.LINEAR, O.TSIT5, y0, p2, 0.0, t1, rtol, rtol * 1e-2)
    ref = O.refresh(O.LINEAR, O.TSIT5, y0, p2, 0.0, t1, rtol, rtol * 1e-2, old)
    stale = O.replay(O.LINEAR, O.TSIT5, y0, p2, old)
    assert np.all(ref["drift_at"] < old["S"])
    err = lambda ys: np.array([np.linalg.norm(ys[l, 0] - expm(rot_matrix(*p2[l]) * t1) @ y0[l])
                               / np.linalg.norm(y0[l]) for l in range(n)])
    e_ref, e_fresh, e_stale = err(ref["y_save"]), err(fresh["y_save"]), err(stale)
    assert e_ref.max() < 3 * e_fresh.max() + 1e-12, (e_ref.max(), e_fresh.max())
    assert e_stale.min() > 30 * e_ref.max(), (e_stale.min(), e_ref.max())
