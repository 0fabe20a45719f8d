"""ensemble_adjoint_static, the adjoint for callers that cannot allocate:
its results equal ensemble_adjoint's (caller workspace) bit for bit, on two
calls in a row with the second smaller (the shared device array keeps the
first call's contents), for every part of the workspace (per-save
cotangents; shared-parameter partials; a checkpointed tape's segment
scratch); a record needing more than the array holds is refused."""
import numpy as np
import pytest
import torch

from paper_2609_02876_amd import _abi as A
from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _same(h, **kw):
    a = B.ensemble_adjoint(h, **kw)
    b = B.ensemble_adjoint_static(h, **kw)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        if x is None:
            assert y is None
        else:
            assert torch.equal(x, y)
    return a


def test_static_adjoint_equals_caller_workspace_twice_second_smaller():
    print("case static adjoint: lorenz 4096 then 1000 trajectories", flush=True)
    y0, p = W.lorenz(4096, seed=41)
    st = list(W.save_times(0.0, 10.0, 20))
    big = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 10.0, 1e-6, 1e-8,
                            save_times=st, steps_hint=400)
    g_big = _same(big)
    assert B.ensemble_adjoint_workspace_bytes(big) > 1 << 20
    y1, p1 = W.lorenz(1000, seed=42)
    small = B.ensemble_record("lorenz", "tsit5", _dev(y1.T), _dev(p1.T), 0.0, 5.0, 1e-6, 1e-8,
                              save_times=list(W.save_times(0.0, 5.0, 7)), steps_hint=256)
    _same(small)
    # the first record again, after the smaller call: still the same bits
    again = B.ensemble_adjoint_static(big)
    torch.cuda.synchronize()
    for x, y in zip(g_big, again):
        assert torch.equal(x, y)


@pytest.mark.parametrize("ckpt", [0, 64])
def test_static_adjoint_shared_params_and_checkpoints(ckpt):
    print(f"case static adjoint: shared params, checkpoint {ckpt}", flush=True)
    n = 3000
    rng = np.random.default_rng(43)
    y0 = np.stack([1 + rng.random(n), rng.random(n), rng.random(n)], 1)
    p = np.array([10.0, 28.0, 8.0 / 3.0])
    st = list(W.save_times(0.0, 4.0, 10))
    h = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p), 0.0, 4.0, 1e-6, 1e-8,
                          save_times=st, params_shared=True, steps_hint=200, ckpt_every=ckpt)
    _same(h)
    y1 = y0[:700]
    h2 = B.ensemble_record("lorenz", "tsit5", _dev(y1.T), _dev(p), 0.0, 4.0, 1e-6, 1e-8,
                           save_times=st[:3], params_shared=True, steps_hint=200,
                           ckpt_every=ckpt)
    _same(h2, loss="cotangent", data=torch.ones((3, 3, 700), dtype=torch.float64, device="cuda"))


def test_static_adjoint_refuses_records_beyond_its_size():
    n = 1 << 18
    y0, p = W.lorenz(n, seed=44)
    st = list(W.save_times(0.0, 0.01, 20))
    h = B.ensemble_record("lorenz", "tsit5", _dev(y0.T), _dev(p.T), 0.0, 0.01, 1e-6, 1e-8,
                          save_times=st, steps_hint=32)
    torch.cuda.synchronize()
    assert B.ensemble_adjoint_workspace_bytes(h) > A.STATIC_WORKSPACE_BYTES
    with pytest.raises(A.EnsembleError, match="static workspace holds"):
        B.ensemble_adjoint_static(h)
