"""Checkpointed tape: one state per segment plus the step sizes; the reverse
sweep replays each segment before sweeping it.  Results must equal the full
tape's bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import oracle_mesh
from paper_2609_02876_amd import autograd as AG
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64, grad=False):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda", requires_grad=grad)


@pytest.mark.parametrize("system,method,n,t1,ckpt", [
    ("lorenz", "tsit5", 3000, 10.0, 64),
    ("lorenz", "tsit5", 777, 10.0, 16),
    ("lorenz", "vern7", 513, 10.0, 256),
    ("vdp", "tsit5", 65, 6.3, 32),
])
def test_checkpoint_equals_full_tape(system, method, n, t1, ckpt):
    gen = {"lorenz": W.lorenz, "vdp": W.vdp}[system]
    y0, p = gen(n, seed=21)
    st = list(W.save_times(0.0, t1, 20))
    Y0, P = _dev(y0.T), _dev(p.T)
    full = B.ensemble_record(system, method, Y0, P, 0.0, t1, 1e-6, 1e-8, save_times=st,
                             steps_hint=400)
    ck = B.ensemble_record(system, method, Y0, P, 0.0, t1, 1e-6, 1e-8, save_times=st,
                           steps_hint=400, ckpt_every=ckpt)
    g_full = B.ensemble_adjoint(full)
    g_ck = B.ensemble_adjoint(ck)
    torch.cuda.synchronize()
    assert torch.equal(full.status, ck.status) and bool((ck.status == 0).all())
    assert torch.equal(full.y_save, ck.y_save)
    h1, s1 = B.ensemble_mesh_export(full)
    h2, s2 = B.ensemble_mesh_export(ck)
    assert torch.equal(h1, h2) and torch.equal(s1, s2)
    for a, b in zip(g_full, g_ck):
        assert torch.equal(a, b)
    # and the oracle agrees with both, on their (shared) mesh
    so = {"lorenz": O.LORENZ, "vdp": O.VDP}[system]
    mo = {"tsit5": O.TSIT5, "vern7": O.VERN7}[method]
    gp_o, gy_o, _ = O.adjoint(so, mo, y0, p, oracle_mesh(ck))
    assert np.array_equal(g_ck[0].cpu().numpy(), gp_o.T)
    assert np.array_equal(g_ck[1].cpu().numpy(), gy_o.T)


def test_checkpoint_shared_params_and_frozen_mesh():
    n = 600
    rng = np.random.default_rng(22)
    y0 = np.stack([1 + rng.random(n), rng.random(n), rng.random(n)], 1)
    p = np.array([10.0, 28.0, 8.0 / 3.0])
    st = [1.0, 2.5, 4.0]
    Y0 = _dev(y0.T)
    grads = []
    for ck in (0, 64):
        P = _dev(p, grad=True)
        ys = AG.odeint("lorenz", "tsit5", Y0, P, 0.0, 4.0, save_times=st, params_shared=True,
                       ckpt_every=ck, steps_hint=200)
        (ys ** 2).sum().backward()
        grads.append(P.grad.clone())
    assert torch.equal(grads[0], grads[1])
    # frozen mesh replayed into a checkpointed tape
    P = _dev(p, grad=True)
    mesh = AG.frozen_mesh("lorenz", "tsit5", Y0, P, 0.0, 4.0, save_times=st, params_shared=True,
                          steps_hint=200)
    ys = AG.odeint("lorenz", "tsit5", Y0, P, 0.0, 4.0, save_times=st, params_shared=True,
                   mesh=mesh, ckpt_every=64)
    (ys ** 2).sum().backward()
    assert torch.equal(P.grad, grads[0])


def test_checkpoint_pool_overflow_pages():
    """Reserve fewer segments than needed: overflow pages are linked and the
    sweep still matches the full tape."""
    n = 512
    y0, p = W.lorenz(n, seed=23)
    st = list(W.save_times(0.0, 10.0, 20))
    Y0, P = _dev(y0.T), _dev(p.T)
    full = B.ensemble_record("lorenz", "tsit5", Y0, P, 0.0, 10.0, 1e-6, 1e-8, save_times=st,
                             steps_hint=400)
    nbytes = B.ensemble_record_bytes("lorenz", "tsit5", n, 0.0, 10.0, 400, 20, ckpt_every=64)
    pool = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ck = B.ensemble_record("lorenz", "tsit5", Y0, P, 0.0, 10.0, 1e-6, 1e-8, save_times=st,
                           pool=pool, steps_per_traj=128, ckpt_every=64)
    g_full, g_ck = B.ensemble_adjoint(full), B.ensemble_adjoint(ck)
    torch.cuda.synchronize()
    assert bool((ck.status == 0).all())
    assert B.ensemble_record_stats(ck)["overflow_pages_used"] > 0
    for a, b in zip(g_full, g_ck):
        assert torch.equal(a, b)


def _align_mode(steps, k):
    """Which of the sweep's lane alignments a wavefront takes (restated from
    the sweep's source): 'r_max', 'k' (first segments padded to K) or None."""
    r = [(s - 1) % k + 1 for s in steps]
    f = [(s - q) // k for s, q in zip(steps, r)]
    if max(r) + k * max(f) <= max(steps):
        return "r_max"
    if 4 * k * (max(f) + 1) <= 5 * max(steps):
        return "k"
    return None


@pytest.mark.parametrize("k", [16, 32, 64, 128, 256])
def test_checkpoint_alignment_on_given_meshes(k):
    """Step counts chosen so that the checkpointed sweep's lane alignment
    takes each of its forms (at K = 64 one wavefront is left unaligned, one
    aligned to its longest first segment and two padded to K): the sweep
    equals the full tape's bit for bit and the oracle's on the same mesh."""
    n = 256
    lane = np.arange(64)
    steps = np.concatenate([250 + lane % 13, 300 + lane % 11, 60 + lane % 11,
                            np.random.default_rng(5).integers(5, 400, 64)]).astype(np.int32)
    # the sweep takes a block's lanes in step-count order, so wavefront w
    # holds the counts of rank 64 w .. 64 w + 63 of the block (one block here)
    srt = sorted(int(s) for s in steps)
    modes = [_align_mode(srt[w * 64:(w + 1) * 64], k) for w in range(4)]
    print(f"case ckpt alignment k={k} modes={modes}", flush=True)
    if k == 64:
        assert set(modes) == {"r_max", "k", None}
    t1 = 2.0
    cap = int(steps.max())
    h = np.zeros((cap, n))
    for l in range(n):
        h[:steps[l], l] = t1 / steps[l]
    y0, p = W.damped_rotation(n, seed=8)
    st = list(W.save_times(0.0, t1, 20))
    args = ("linear", "tsit5", _dev(y0.T), _dev(p.T), 0.0, t1, _dev(h),
            torch.tensor(steps, device="cuda"))
    full = B.ensemble_replay_mesh(*args, save_times=st)
    ck = B.ensemble_replay_mesh(*args, save_times=st, ckpt_every=k)
    g_full = B.ensemble_adjoint(full)
    g_ck = B.ensemble_adjoint(ck)
    torch.cuda.synchronize()
    assert bool((ck.status == 0).all()) and torch.equal(full.steps(), ck.steps())
    assert torch.equal(full.y_save, ck.y_save)
    for a, b in zip(g_full, g_ck):
        assert torch.equal(a, b)
    gp_o, gy_o, _ = O.adjoint(O.LINEAR, O.TSIT5, y0, p, oracle_mesh(ck))
    for got, ref in ((g_ck[0].cpu().numpy(), gp_o.T), (g_ck[1].cpu().numpy(), gy_o.T)):
        # per-lane normwise relative error (lanes last)
        err = (np.linalg.norm(got - ref, axis=0) /
               np.maximum(np.linalg.norm(ref, axis=0), 1e-300)).max()
        assert err <= 1e-11, err
