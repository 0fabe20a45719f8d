"""Serving: jobs of different systems, sizes and tolerances submitted while
others run give, each of them, the results of ensemble_record +
ensemble_adjoint run alone on that job -- to the bit, since a trajectory's
arithmetic does not depend on what it is packed with.  Also: admission waits
for memory, and a job whose record runs out of pages is run again."""
import numpy as np
import pytest
import torch

from paper_2609_02876_amd import binding as B
from paper_2609_02876_amd import serving as SV
from paper_2609_02876_amd import workloads as W

pytestmark = pytest.mark.gpu

SPAN = {"lorenz": 10.0, "vdp": 6.3, "robertson": 1e5, "hires": 321.8122}
METHOD = {"lorenz": "tsit5", "vdp": "vern7", "robertson": "rodas4", "hires": "rodas4"}
HINT = {"lorenz": 1536, "vdp": 512, "robertson": 1024, "hires": 1024}


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _job(k, system, n, rtol):
    y0, p = W.GENERATORS[system](n, seed=100 + k)
    atol = rtol * (1e-2 if system in ("lorenz", "vdp") else 1e-4)
    st = list(W.save_times(0.0, SPAN[system], 4))
    return dict(system=system, method=METHOD[system], y0=_dev(y0.T), p=_dev(p.T), t1=SPAN[system],
                rtol=rtol, atol=atol, st=st, hint=HINT[system])


def _solo(j, hint):
    h = B.ensemble_record(j["system"], j["method"], j["y0"], j["p"], 0.0, j["t1"], j["rtol"],
                          j["atol"], save_times=j["st"], steps_hint=hint)
    gp, gy, ll = B.ensemble_adjoint(h)
    torch.cuda.synchronize()
    return h.y_save, h.status, gp, gy, ll


def _same(sj, ref):
    ys, st, gp, gy, ll = ref
    return (torch.equal(sj.y_save, ys) and torch.equal(sj.status, st) and
            torch.equal(sj.grad_params, gp) and torch.equal(sj.grad_y0, gy) and
            torch.equal(sj.loss, ll))


def test_served_mix_equals_solo_runs():
    rng = np.random.default_rng(0)
    specs = []
    for k in range(16):
        system = ["lorenz", "vdp", "robertson", "hires"][k % 4]
        n = int(rng.integers(1, 3000))
        rtol = [1e-4, 1e-6, 1e-8][int(rng.integers(0, 3))]
        if system == "hires" and rtol == 1e-8:
            rtol = 1e-6
        specs.append(_job(k, system, n, rtol))
    print("case serving: 16 mixed jobs, 3 slots", flush=True)
    srv = SV.Server(2 << 30, n_slots=3)
    served = []
    for j in specs:
        served.append(srv.submit(j["system"], j["method"], j["y0"], j["p"], 0.0, j["t1"],
                                 j["rtol"], j["atol"], save_times=j["st"], steps_hint=j["hint"]))
        srv.progress()
    srv.drain()
    st = srv.stats()
    print(f"  completed {st['completed']} failed {st['failed']} retried {st['retried']} "
          f"p50 {st['p50_latency_s'] * 1e3:.1f} ms p99 {st['p99_latency_s'] * 1e3:.1f} ms "
          f"peak pool {st['pool_peak'] / 2**20:.0f} MiB")
    assert st["completed"] == len(specs) and st["failed"] == 0
    for j, sj in zip(specs, served):
        assert sj.done()
        assert _same(sj, _solo(j, j["hint"])), (j["system"], j["rtol"])
    srv.close()


def test_admission_waits_for_memory_and_retries_short_plans():
    """A pool that holds about two records at a time; one job planned far
    too short (its lanes run out of pages) is run again with a larger plan."""
    specs = [_job(50 + k, "lorenz", 2048, 1e-6) for k in range(5)]
    print("case serving: admission by memory, short plan", flush=True)
    one = B.ensemble_record_bytes("lorenz", "tsit5", 2048, 0.0, 10.0, 512, 4)
    srv = SV.Server(int(2.5 * one) + (16 << 20), n_slots=4)
    served = [srv.submit(j["system"], j["method"], j["y0"], j["p"], 0.0, j["t1"], j["rtol"],
                         j["atol"], save_times=j["st"], steps_hint=512) for j in specs[:4]]
    waiting = srv.stats()["waiting"]
    short = specs[4]
    served.append(srv.submit(short["system"], short["method"], short["y0"], short["p"], 0.0,
                             short["t1"], short["rtol"], short["atol"], save_times=short["st"],
                             steps_hint=64))
    srv.drain()
    st = srv.stats()
    print(f"  waiting after 4 submits {waiting}; retried {st['retried']}; "
          f"peak {st['pool_peak'] / one:.2f} records")
    assert waiting >= 1
    assert st["retried"] >= 1 and st["failed"] == 0 and st["completed"] == 5
    assert st["pool_peak"] <= st["pool_arena"]
    for j, sj in zip(specs, served):
        assert _same(sj, _solo(j, 512))
    srv.close()
