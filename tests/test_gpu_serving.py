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


SYS_O = {"lorenz": 1, "vdp": 2, "robertson": 3, "hires": 4}    # oracle system ids
MET_O = {"tsit5": 1, "vern7": 2, "rodas4": 3}                    # oracle method ids


def test_poisson_stream_of_mixed_sizes_matches_solo_and_oracle():
    """The serving pattern's shape at test scale: 96 jobs over the four
    systems, sizes log-uniform in 2^8..2^14 lanes, rtol in {1e-4, 1e-6,
    1e-8} (HIRES: 1e-4, 1e-6), arriving as a Poisson stream while earlier
    jobs run.  Every served job equals its solo run to the bit; on a sample
    of jobs (two per system) a few trajectories are also checked against the
    oracle run on the solo record's own mesh (states and gradients within
    1e-11 per trajectory).  The adaptive meshes themselves are compared with
    the oracle's by the parity tests of each system and method."""
    import time

    import oracle as O
    from gpu_helpers import oracle_mesh, rel

    rng = np.random.default_rng(7)
    specs = []
    for k in range(96):
        system = ["lorenz", "vdp", "robertson", "hires"][k % 4]
        n = int(round(2 ** (8 + 6 * rng.random())))
        rtols = [1e-4, 1e-6] if system == "hires" else [1e-4, 1e-6, 1e-8]
        specs.append(_job(200 + k, system, n, rtols[int(rng.integers(0, len(rtols)))]))
    gaps = rng.exponential(0.002, len(specs))
    print(f"case serving: Poisson stream of {len(specs)} jobs, "
          f"{sum(j['y0'].shape[1] for j in specs)} trajectories, 4 slots", flush=True)
    srv = SV.Server(6 << 30, n_slots=4)
    served = []
    for j, gap in zip(specs, gaps):
        t_next = time.perf_counter() + gap
        while time.perf_counter() < t_next:
            srv.progress()
        served.append(srv.submit(j["system"], j["method"], j["y0"], j["p"], 0.0, j["t1"],
                                 j["rtol"], j["atol"], save_times=j["st"], steps_hint=j["hint"]))
    srv.drain()
    st = srv.stats()
    print(f"  completed {st['completed']} failed {st['failed']} retried {st['retried']} "
          f"p50 {st['p50_latency_s'] * 1e3:.1f} ms p99 {st['p99_latency_s'] * 1e3:.1f} ms",
          flush=True)
    assert st["completed"] == len(specs) and st["failed"] == 0

    sample = {}
    for k, j in enumerate(specs):
        sample.setdefault(j["system"], [])
        if len(sample[j["system"]]) < 2:
            sample[j["system"]].append(k)
    picked = {k for ks in sample.values() for k in ks}
    worst = 0.0
    for k, (j, sj) in enumerate(zip(specs, served)):
        # a generous plan: a served job that ran out of pages was run again
        # with a larger one, and the plan does not change the arithmetic
        h = B.ensemble_record(j["system"], j["method"], j["y0"], j["p"], 0.0, j["t1"], j["rtol"],
                              j["atol"], save_times=j["st"], steps_hint=4 * j["hint"])
        gp, gy, ll = B.ensemble_adjoint(h)
        torch.cuda.synchronize()
        assert _same(sj, (h.y_save, h.status, gp, gy, ll)), (k, j["system"], j["rtol"])
        if k not in picked:
            continue
        n = j["y0"].shape[1]
        lanes = sorted({0, n // 3, n // 2, n - 1})
        gm = oracle_mesh(h, lanes)
        y0 = j["y0"].cpu().numpy().T[lanes]
        p = j["p"].cpu().numpy().T[lanes]
        so, mo = SYS_O[j["system"]], MET_O[j["method"]]
        ys_o = np.transpose(O.replay(so, mo, y0, p, gm), (1, 2, 0))
        gp_o, gy_o, _ = O.adjoint(so, mo, y0, p, gm)
        e = max(float(rel(sj.y_save.cpu().numpy()[..., lanes], ys_o).max()),
                float(rel(sj.grad_params.cpu().numpy()[:, lanes], gp_o.T).max()),
                float(rel(sj.grad_y0.cpu().numpy()[:, lanes], gy_o.T).max()))
        print(f"  job {k} {j['system']} rtol {j['rtol']:.0e} n {n}: served vs oracle on its mesh "
              f"max rel err {e:.2e}", flush=True)
        worst = max(worst, e)
    assert worst <= 1e-11, worst
    srv.close()
