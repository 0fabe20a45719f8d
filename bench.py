"""Benchmark: trajectory-gradients per second (record + reverse sweep).

Default workload: 2^20 Lorenz trajectories (sigma ~ U[9,11], rho ~ U[27,29],
beta ~ U[2.5,3], y0 = (1,0,0)) on t in [0, 10], Tsit5, FP64, rtol 1e-6,
atol 1e-8, loss = sum of squared states at 20 evenly spaced save times,
gradient with respect to the three parameters of every trajectory.

One step = ensemble_record + ensemble_adjoint over the whole ensemble, inputs
already resident in device memory.  Prints one JSON line.
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 FLOP/clk
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
METRIC = "trajectory-gradients/s (fwd+adjoint) at 2^20 Lorenz, rtol 1e-6"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    # six warm-ups: the GPU's clock needs sustained load to settle (after the
    # set-up's idle spell, three warm-ups leave the first two timed steps of
    # the headline 20 % and 8 % slow; a cold GPU needs longer still)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", default="lorenz_2p20_t10")
    ap.add_argument("--registered", action="store_true",
                    help="run the workload's system as a copy registered at run time from source "
                         "(ensemble_system_register; Lorenz and Robertson)")
    ap.add_argument("--mode", choices=("reverse", "forward", "refresh", "solve"),
                    default="reverse",
                    help="gradient by the reverse sweep (default) or by forward-mode passes, "
                         "one per parameter, on the recorded mesh; refresh: the mesh-drift "
                         "policy (an old record refreshed at moved parameters, then the sweep); "
                         "solve: the forward-only solve (states at the save times, no record)")
    ap.add_argument("--refresh-step", type=float, default=1e-3,
                    help="relative parameter change for --mode refresh (seeded normal)")
    ap.add_argument("--n", type=int, default=None, help="override the trajectory count")
    ap.add_argument("--dense", action="store_true",
                    help="save states from the continuous extension (dense output) instead "
                         "of an extra step")
    ap.add_argument("--grid", choices=("explicit", "stiff", "ude"), default=None,
                    help="run a size / tolerance sweep of the benchmark configurations, one "
                         "line per configuration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--traffic", default=None,
                    help="JSON with measured HBM bytes per launch of the kernels (default: "
                         "profiles/<workload>_traffic.json when its source hash matches)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy MIB MiB on the device before the timed steps (a kernel of known "
                         "traffic for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--write-traffic", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU run: turn the counter output of two rocprofv3 --pmc runs of this "
                         "script (FETCH_SIZE, then WRITE_SIZE, both with --copy-calibration) into "
                         "profiles/<workload>_traffic.json")
    ap.add_argument("--serve-jobs", type=int, default=2000,
                    help="jobs in the serving workload (--workload serve_mix)")
    ap.add_argument("--serve-max-log2", type=int, default=18,
                    help="job sizes are log-uniform in 2^8..2^this lanes")
    ap.add_argument("--serve-repeat", type=int, default=3,
                    help="the Poisson streams submit the job list this many times (each time "
                         "in a new random order), so that a window lasts several seconds")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="offered loads (fractions of the one-shot capacity)")
    return ap.parse_args()


def kernel_source_hash(forward=False):
    """Hash of the HIP sources: measured traffic is used only for the build it
    was measured on.  The forward-mode kernel's own source counts only for
    forward-mode traffic, the one measurement that runs it."""
    import hashlib
    d = os.path.join(ROOT, "paper_2609_02876_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f == "jvp.h" and not forward:
            continue
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(path, workload):
    """Measured HBM bytes per launch {record, adjoint}, or None when absent
    or taken on other kernel sources."""
    if path is None:
        path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("source_hash") != kernel_source_hash(workload.endswith("_forward")):
        return None
    return tr


def write_traffic(fetch_dir, write_dir, workload, n, mib, path=None, solve=False):
    """HBM bytes per launch of the record and the sweep kernel, from rocprofv3
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch).  Each counter is scaled by
    known / counted for the calibration copy of `mib` MiB (the device copy
    kernel with the largest count); the full-size dispatches of each kernel
    (the largest grid: the pool-sizing pilot is smaller; the instantiation
    dispatched most often) are averaged.  `solve`: the forward-only solve
    kernel alone, as "record" (the record of the same inputs that counts the
    work runs once, outside the timed steps)."""
    import csv
    import glob

    def read(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        if not rows:
            raise SystemExit(f"no {counter} rows under {d}")
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not copies:
            raise SystemExit(f"no calibration copy in {d} (run with --copy-calibration)")
        factor = (mib << 10) / max(copies)
        if not 0.25 <= factor <= 4.0:
            raise SystemExit(f"the largest copy in {d} counts {max(copies):.0f} KiB, not near "
                             f"{mib << 10} KiB: no calibration copy of {mib} MiB in this run")
        out = {}
        # a part's kernels: the explicit pairs' full-tape record is two
        # launches (the loop, then the save states; the dense record's loop,
        # then the states from the continuous extension), each counted once
        parts = ((("record", ("_forward_kernel<",)),) if solve else
                 (("record", ("_forward_kernel<", "erk_record_deferred_kernel<",
                              "erk_saves_kernel<", "dense_saves_kernel<")),
                  ("adjoint", ("_adjoint_kernel<",)), ("jvp", ("jvp_kernel<",))))
        for part, keys in parts:
            ks = [r for r in rows if any(k in r["Kernel_Name"] for k in keys)]
            if not ks:
                if part == "record":
                    raise SystemExit(f"no record kernel rows under {d}")
                continue
            g = max(int(r["Grid_Size"]) for r in ks)
            kib, disp, names_used = 0.0, None, []
            for key in keys:
                kk = [r for r in ks if key in r["Kernel_Name"] and int(r["Grid_Size"]) == g]
                if not kk:
                    continue
                # the instantiation dispatched most often: the timed launches (a
                # forward-only solve of the same size, e.g. for targets, runs once)
                names = [r["Kernel_Name"] for r in kk]
                top = max(set(names), key=names.count)
                vals = [float(r["Counter_Value"]) for r in kk if r["Kernel_Name"] == top]
                kib += sum(vals) / len(vals)
                disp = len(vals) if disp is None else min(disp, len(vals))
                names_used.append(top.split("(")[0])
            out[part] = {"kib": kib, "dispatches": disp, "grid": g, "kernels": names_used}
        return out, factor

    fe, ff = read(fetch_dir, "FETCH_SIZE")
    wr, wf = read(write_dir, "WRITE_SIZE")
    tr = {"workload": workload, "n": n,
          "source_hash": kernel_source_hash(workload.endswith("_forward")),
          "calibration": {"copy_mib": mib, "fetch_factor": ff, "write_factor": wf}}
    for part in [q for q in ("record", "adjoint", "jvp") if q in fe and q in wr]:
        fb, wb = fe[part]["kib"] * 1024 * ff, wr[part]["kib"] * 1024 * wf
        tr[part] = fb + wb
        tr[part + "_detail"] = {"fetch_bytes": fb, "write_bytes": wb,
                                "fetch_kib_counted": fe[part]["kib"],
                                "write_kib_counted": wr[part]["kib"],
                                "dispatches": fe[part]["dispatches"],
                                "grid_threads": fe[part]["grid"],
                                "kernels": fe[part]["kernels"]}
    if path is None:
        path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(tr, f, indent=1)
        f.write("\n")
    print(json.dumps(tr))
    return tr


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


_ORACLE_BUILD = None


def load_oracle():
    """The oracle, built with -O3 -march=native for this host when g++ can
    (the build takes seconds), else the in-tree portable build."""
    global _ORACLE_BUILD
    import oracle as O
    from oracle import build as OB
    if _ORACLE_BUILD is None:
        out = os.path.join(tempfile.mkdtemp(prefix="ens_oracle_"), "liboracle_native.so")
        try:
            OB.build_native(out)
            O.use_library(out)
            _ORACLE_BUILD = OB.flags(native=True)
        except (OSError, subprocess.CalledProcessError, RuntimeError):
            _ORACLE_BUILD = OB.flags(native=False)
    return O


def cpu_info():
    return {"cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "cpu": cpu_model(), "build": _ORACLE_BUILD}


def cpu_baseline(cfg, y0, p, st, target_s, cap, loss_data=None, scale=1.0, dense=False):
    """The FP64 CPU oracle (record + adjoint) on a bounded sample of the workload."""
    import numpy as np
    O = load_oracle()
    so = {"lorenz": O.LORENZ, "vdp": O.VDP, "robertson": O.ROBERTSON, "hires": O.HIRES,
          "linear": O.LINEAR, "ude": O.LV_UDE}[cfg["system"]]
    mo = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}[cfg["method"]]
    save = list(st)
    shared = cfg.get("shared", False)

    def run(m):
        pm = p if shared else p[:m]
        t = time.perf_counter()
        rec = O.record(so, mo, y0[:m], pm, cfg["t0"], cfg["t1"], cfg["rtol"], cfg["atol"],
                       save_t=save, cap=cap, params_shared=shared)
        if loss_data is None:
            O.adjoint(so, mo, y0[:m], pm, rec, params_shared=shared, dense=dense)
        else:
            O.adjoint(so, mo, y0[:m], pm, rec, O.LOSS_MSE_TARGET, loss_data[:m], scale,
                      params_shared=shared, dense=dense)
        return time.perf_counter() - t

    # grow the sample until it takes about target_s (small samples run below
    # the threads' full rate, so one extrapolation falls short)
    m2 = 256 if cfg["system"] == "ude" else 2048
    dt2 = run(m2)
    for _ in range(3):
        if dt2 >= 0.7 * target_s or m2 >= len(y0):
            break
        m2 = int(min(len(y0), m2 * target_s / max(dt2, 1e-3)))
        m2 = max(64, (m2 // 64) * 64)
        dt2 = run(m2)
    return {"value": m2 / dt2, "unit": "trajectory-gradients/s", **cpu_info(), "kind": "oracle",
            "sample": f"first {m2} trajectories of the workload, record + adjoint, {dt2:.1f} s"}


def main():
    args = parse()
    if args.write_traffic:
        from paper_2609_02876_amd import workloads as W
        n = args.n or W.WORKLOADS[args.workload]["n"]
        key = args.workload + {"forward": "_forward", "solve": "_solve"}.get(args.mode, "")
        key += ("_dense" if args.dense else "") + ("_registered" if args.registered else "")
        return write_traffic(*args.write_traffic, key, n, args.copy_calibration or 1024,
                             solve=args.mode == "solve")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the ensemble "
              "shards by trajectory with no exchange, so more GPUs are not exercised here.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2609_02876_amd import workloads as W

    if args.grid:
        return grid_bench(args)
    if args.workload == "serve_mix":
        return serve_bench(args)
    if args.mode == "forward":
        return forward_bench(args)
    if args.mode == "refresh":
        return refresh_bench(args)
    if args.mode == "solve":
        return solve_bench(args)
    cfg, y0, p, st = W.make(args.workload, n=args.n)
    torch.cuda.set_device(torch.device("cuda:0"))
    out = reverse_bench(cfg, y0, p, st, args.steps, args.warmup, workload=args.workload,
                        dense=args.dense, registered=args.registered,
                        cpu_seconds=None if args.no_cpu_baseline else args.cpu_seconds,
                        traffic_path=args.traffic, copy_mib=args.copy_calibration)
    print(json.dumps(out), flush=True)


def reverse_bench(cfg, y0, p, st, steps, warmup, workload, dense=False, registered=False,
                  cpu_seconds=None, traffic_path=None, copy_mib=0):
    """Time `steps` steps of record + reverse sweep of one ensemble (inputs
    resident on the GPU) and return the benchmark line as a dict."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import flops
    from paper_2609_02876_amd import workloads as W

    n = cfg["n"]
    save = list(st) if cfg["n_save"] else None
    dev = torch.device("cuda:0")
    f32 = cfg.get("dtype", "f64") == "f32"
    tdt = torch.float32 if f32 else torch.float64
    shared = cfg.get("shared", False)
    ckpt = cfg.get("ckpt_every", 0)
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=tdt, device=dev)
    p_d = torch.tensor(np.ascontiguousarray(p if shared else p.T), dtype=tdt, device=dev)
    gsys = registered_system(cfg["system"]) if registered else cfg["system"]
    args_common = (gsys, cfg["method"], y0_d, p_d, cfg["t0"], cfg["t1"], cfg["rtol"],
                   cfg["atol"])

    # loss: sum of squares, or MSE to targets from the teacher network (UDE)
    loss_kind, loss_data, scale, tgt_host = "sumsq", None, 1.0, None
    if cfg.get("loss") == "mse":
        th_t = torch.tensor(W.ude_teacher(), dtype=tdt, device=dev)
        loss_data, _ = B.ensemble_solve(cfg["system"], cfg["method"], y0_d, th_t, cfg["t0"],
                                        cfg["t1"], cfg["rtol"], cfg["atol"], save_times=save,
                                        params_shared=True)
        loss_kind, scale = "mse", 1.0 / (n * cfg["n_save"] * y0.shape[1])
        tgt_host = np.transpose(loss_data.double().cpu().numpy(), (2, 0, 1))

    # pool plan from a pilot record of a sample of the ensemble
    m = min(n, 8192)
    pilot = B.ensemble_record(gsys, cfg["method"], y0_d[:, :m].contiguous(),
                              p_d if shared else p_d[:, :m].contiguous(), cfg["t0"], cfg["t1"],
                              cfg["rtol"], cfg["atol"], save_times=save, steps_hint=4096,
                              params_shared=shared)
    s_pilot = pilot.steps().double()
    cap_cpu = int(s_pilot.max().item() * 1.5) + 64
    hint = B.steps_hint_for(float(s_pilot.mean().item()), margin=1.12)
    del pilot
    nbytes = B.ensemble_record_bytes(gsys, cfg["method"], n, cfg["t0"], cfg["t1"], hint,
                                     cfg["n_save"], tdt, ckpt, dense=dense)
    pool = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    ws = None

    stream = torch.cuda.current_stream()

    def step(events=None):
        if events:
            events[0].record(stream)
        rec = B.ensemble_record(*args_common, save_times=save, pool=pool, steps_per_traj=hint,
                                params_shared=shared, ckpt_every=ckpt, dense=dense)
        if events:
            events[1].record(stream)
        gp, gy, ll = B.ensemble_adjoint(rec, loss_kind, loss_data, scale, want_y0=True,
                                        want_loss=True, workspace=ws)
        if events:
            events[2].record(stream)
        return rec, gp, gy, ll

    if copy_mib:
        calibration_copy(copy_mib, dev)
    # events made and the warm-up's status counted on the device before the
    # timed steps, so that the GPU does not idle between the warm-up and the
    # timed steps (after an idle spell its first steps run at a lower clock)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    bad_warm = None
    for _ in range(warmup):
        rec, gp, gy, ll = step()
        if ws is None:
            wsb = B.ensemble_adjoint_workspace_bytes(rec)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    if warmup:
        bad_warm = (rec.status != 0).sum()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        rec, gp, gy, ll = step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / steps
    step_ev = sorted(e[0].elapsed_time(e[2]) for e in evs)

    if bad_warm is not None and int(bad_warm.item()):
        raise RuntimeError(f"{int(bad_warm.item())} trajectories did not finish in the warm-up")
    bad = int((rec.status != 0).sum().item())
    if bad:
        raise RuntimeError(f"{bad} trajectories did not finish (status != OK)")
    stats = B.ensemble_record_stats(rec)
    n_saves = n * (cfg["n_save"] or 1)
    zero_sides = n_saves - stats["side_steps"]
    f_rec = flops.record_flops(cfg["method"], cfg["system"], stats["trials"],
                               stats["steps_accepted"], stats["side_steps"], dense)
    f_adj = flops.adjoint_flops(cfg["method"], cfg["system"], stats["steps_accepted"],
                                stats["side_steps"], zero_sides, dense)
    ms_per_step = wall * 1e3 / steps
    value = n * steps / wall

    dominant = "adjoint" if adj_ms >= rec_ms else "record"
    f_dom, ms_dom = (f_adj, adj_ms) if dominant == "adjoint" else (f_rec, rec_ms)
    achieved = f_dom / (ms_dom * 1e-3) / 1e12
    traffic = None
    # measured bytes belong to the kernels they were taken on: the dense and
    # the registered records have files of their own
    tr = load_traffic(traffic_path, workload + ("_dense" if dense else "") +
                      ("_registered" if registered else ""))
    if tr is not None and tr.get("n") == n:
        traffic = tr.get(dominant)
    if cfg["system"] == "ude":
        bound, peak = "mfma", PEAK_FP32_TFLOPS
        kname = f"ude_{'adjoint' if dominant == 'adjoint' else 'forward'}_kernel (f32)"
    else:
        bound, peak = "alu", (PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS)
        deferred = cfg["method"] in ("tsit5", "vern7") and not ckpt and not dense
        kname = ("erk_adjoint_kernel" if dominant == "adjoint" else
                 # explicit pairs' full-tape record: the loop, then the save states
                 "erk_record_deferred_kernel + erk_saves_kernel" if deferred else
                 "erk_forward_kernel")
        kname += f" ({cfg['system']}, {cfg['method']}, {'f32' if f32 else 'f64'}"
        kname += ", dense output)" if dense else ")"
    out = {
        "metric": METRIC if workload == "lorenz_2p20_t10" and not dense
        else "trajectory-gradients/s (fwd+adjoint)",
        "value": value,
        "unit": "trajectory-gradients/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if f32 else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "system": cfg["system"], "method": cfg["method"],
                   "registered_at_run_time": bool(registered),
                   "n": n, "t_span": [cfg["t0"], cfg["t1"]], "rtol": cfg["rtol"],
                   "atol": cfg["atol"], "n_save": cfg["n_save"], "ckpt_every": ckpt,
                   "save_states": ("dense output (continuous extension)" if dense
                                   else "extra step from the last mesh point"),
                   "loss": ("MSE to teacher-network trajectories" if loss_kind == "mse"
                            else "sum of squared save states"),
                   "gradient": "shared weights" if shared else "per-trajectory params"},
        "roofline": {"bound": bound, "kernel": kname,
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic},
        "kernels_ms": {"record": rec_ms, "adjoint": adj_ms},
        # per-step event times (record start to sweep end) and the sweep
        # alone against an existing record (the paper's per-gradient view)
        "step_event_ms": {"median": step_ev[len(step_ev) // 2], "best": step_ev[0],
                          "mean": sum(step_ev) / len(step_ev), "worst": step_ev[-1]},
        "adjoint_only_per_s": n / (adj_ms * 1e-3),
        "algorithmic_flop": {"record": f_rec, "adjoint": f_adj,
                             "total_tflops": (f_rec + f_adj) / (ms_per_step * 1e-3) / 1e12},
        "record_stats": {"accepted_per_traj": stats["steps_accepted"] / n,
                         "trials_per_traj": stats["trials"] / n,
                         "side_steps": stats["side_steps"], "overflow_pages_used": stats["overflow_pages_used"],
                         "pool_gb": nbytes / 1e9},
    }
    if cpu_seconds:
        out["cpu_baseline"] = cpu_baseline(cfg, y0, p, st, cpu_seconds, cap_cpu, tgt_host,
                                           scale, dense)
    return out


# The size / tolerance sweeps of the benchmark configurations: explicit pairs
# on Lorenz and Van der Pol (both methods, both precisions, two tolerances,
# 2^12..2^20 trajectories, 20 save times), the stiff systems with both
# Rosenbrock methods at 2^10..2^18, the UDE at 2^14..2^18 with the full and
# the checkpointed tape.
def grid_configs(which):
    from paper_2609_02876_amd import workloads as W
    out = []
    if which == "explicit":
        for system, t1 in (("lorenz", 10.0), ("vdp", 6.3)):
            for method in ("tsit5", "vern7"):
                for dtype in ("f64", "f32"):
                    for rtol in (1e-6, 1e-8):
                        for k in (12, 14, 16, 18, 20):
                            out.append(dict(system=system, method=method, n=1 << k, t0=0.0,
                                            t1=t1, rtol=rtol, atol=1e-8, n_save=20,
                                            dtype=dtype))
    elif which == "stiff":
        for system, t1 in (("robertson", 1e5), ("hires", 321.8122)):
            for method in ("rodas4", "ros23"):
                for k in (10, 12, 14, 16, 18):
                    out.append(dict(system=system, method=method, n=1 << k, t0=0.0, t1=t1,
                                    rtol=1e-6, atol=1e-10, n_save=20))
    elif which == "ude":
        for k in (14, 15, 16, 17, 18):
            for ck in (0, 64):
                cfg = dict(W.WORKLOADS["ude_2p16"])
                cfg.update(n=1 << k, ckpt_every=ck)
                out.append(cfg)
    else:
        raise SystemExit(f"unknown grid {which!r}: explicit, stiff or ude")
    return out


def grid_bench(args):
    """One JSON line per configuration of the chosen sweep (a few timed steps
    each; the oracle on a small sample for the configurations at 2^12, 2^10
    and 2^14 trajectories only)."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import workloads as W
    torch.cuda.set_device(torch.device("cuda:0"))
    for cfg in grid_configs(args.grid):
        gen = W.GENERATORS[cfg["system"]]
        y0, p = gen(cfg["n"], 0)
        if cfg.get("dtype") == "f32":
            y0 = y0.astype(np.float32).astype(np.float64)
            p = p.astype(np.float32).astype(np.float64)
        st = W.save_times(cfg["t0"], cfg["t1"], cfg["n_save"])
        small = cfg["n"] == {"explicit": 1 << 12, "stiff": 1 << 10, "ude": 1 << 14}[args.grid]
        name = (f"{cfg['system']}_{cfg['method']}_{cfg.get('dtype', 'f64')}_rtol{cfg['rtol']:g}"
                f"_n{cfg['n']}" + (f"_ckpt{cfg['ckpt_every']}" if cfg.get("ckpt_every") else ""))
        out = reverse_bench(cfg, y0, p, st, args.steps, args.warmup, workload=name,
                            dense=args.dense,
                            cpu_seconds=(3.0 if small and not args.no_cpu_baseline else None))
        print(json.dumps(out), flush=True)


def registered_system(system):
    """Register the example source of a built-in system (same operations) and
    return the name it runs under."""
    from paper_2609_02876_amd import _abi as A
    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import user_systems as U
    src = {"lorenz": (U.LORENZ, False), "robertson": (U.ROBERTSON, True)}
    if system not in src:
        raise SystemExit("--registered runs Lorenz or Robertson workloads")
    name = system + "_registered"
    if name not in A.SYSTEMS:
        d, npar = A.SYSTEMS[system][1:]
        B.register_system(name, src[system][0], d, npar, jacobian=src[system][1])
    return name


def calibration_copy(mib, dev):
    """A device copy of known size in the profiled run: the reference for
    scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def refresh_bench(args):
    """The mesh-drift policy on one step of a fit: a record at the workload's
    parameters (untimed), then at parameters moved by --refresh-step
    (relative, seeded normal) the timed step refreshes the old mesh
    (ensemble_refresh: old steps kept while they meet the tolerance, the rest
    re-recorded) and runs the reverse sweep on it.  For context, the same
    step with a fresh record and with the stale mesh replayed unchecked."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import flops
    from paper_2609_02876_amd import workloads as W

    cfg, y0, p, st = W.make(args.workload, n=args.n)
    if cfg.get("shared") or cfg["system"] == "ude":
        raise SystemExit("refresh is built for per-trajectory parameters (not the UDE)")
    n = cfg["n"]
    save = list(st) if cfg["n_save"] else None
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p2 = p * (1.0 + args.refresh_step * np.random.default_rng(17).standard_normal(p.shape))
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=torch.float64, device=dev)
    p_d = torch.tensor(np.ascontiguousarray(p.T), dtype=torch.float64, device=dev)
    p2_d = torch.tensor(np.ascontiguousarray(p2.T), dtype=torch.float64, device=dev)
    span = (cfg["t0"], cfg["t1"], cfg["rtol"], cfg["atol"])
    m = min(n, 8192)
    pilot = B.ensemble_record(cfg["system"], cfg["method"], y0_d[:, :m].contiguous(),
                              p_d[:, :m].contiguous(), *span, save_times=save, steps_hint=4096)
    hint = B.steps_hint_for(float(pilot.steps().double().mean().item()), margin=1.12)
    del pilot
    nbytes = B.ensemble_record_bytes(cfg["system"], cfg["method"], n, cfg["t0"], cfg["t1"],
                                     hint, cfg["n_save"], torch.float64)
    pools = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(2)]
    old = B.ensemble_record(cfg["system"], cfg["method"], y0_d, p_d, *span, save_times=save,
                            pool=pools[0], steps_per_traj=hint)
    h_old, S_old = B.ensemble_mesh_export(old)
    stream = torch.cuda.current_stream()

    def refresh_step(ev=None):
        if ev:
            ev[0].record(stream)
        rec, drift = B.ensemble_refresh(cfg["system"], cfg["method"], y0_d, p2_d, *span, h_old,
                                        S_old, save_times=save, pool=pools[1],
                                        steps_per_traj=hint)
        if ev:
            ev[1].record(stream)
        g = B.ensemble_adjoint(rec)
        if ev:
            ev[2].record(stream)
        return rec, drift, g

    def other_step(kind, ev):
        ev[0].record(stream)
        if kind == "record":
            rec = B.ensemble_record(cfg["system"], cfg["method"], y0_d, p2_d, *span,
                                    save_times=save, pool=pools[1], steps_per_traj=hint)
        else:
            rec = B.ensemble_replay_mesh(cfg["system"], cfg["method"], y0_d, p2_d, cfg["t0"],
                                         cfg["t1"], h_old, S_old, save_times=save,
                                         pool=pools[1], steps_per_traj=hint)
        ev[1].record(stream)
        B.ensemble_adjoint(rec)
        ev[2].record(stream)
        return rec

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for _ in range(args.warmup):
        refresh_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rec, drift, _ = refresh_step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int((rec.status != 0).sum().item()):
        raise RuntimeError("refreshed trajectories did not finish (status != OK)")
    ref_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    stats = B.ensemble_record_stats(rec)
    kept_all = float((drift == S_old).double().mean().item())
    kept_steps = float(drift.double().sum().item()) / max(1.0, float(S_old.double().sum().item()))
    ctx = {}
    for kind in ("record", "stale_replay"):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(3)]
        for e in ev:
            other_step(kind, e)
        torch.cuda.synchronize()
        ctx[kind] = {"forward_ms": sum(e[0].elapsed_time(e[1]) for e in ev) / 3,
                     "adjoint_ms": sum(e[1].elapsed_time(e[2]) for e in ev) / 3}
    n_saves = n * (cfg["n_save"] or 1)
    f_ref = flops.record_flops(cfg["method"], cfg["system"], stats["trials"],
                               stats["steps_accepted"], stats["side_steps"])
    f_adj = flops.adjoint_flops(cfg["method"], cfg["system"], stats["steps_accepted"],
                                stats["side_steps"], n_saves - stats["side_steps"])
    dominant = "adjoint" if adj_ms >= ref_ms else "refresh"
    f_dom, ms_dom = (f_adj, adj_ms) if dominant == "adjoint" else (f_ref, ref_ms)
    achieved = f_dom / (ms_dom * 1e-3) / 1e12
    out = {
        "metric": "trajectory-gradients/s (mesh refresh + adjoint)",
        "value": n * args.steps / wall,
        "unit": "trajectory-gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "system": cfg["system"], "method": cfg["method"],
                   "n": n, "t_span": [cfg["t0"], cfg["t1"]], "rtol": cfg["rtol"],
                   "atol": cfg["atol"], "n_save": cfg["n_save"],
                   "parameter_step": args.refresh_step, "slack": 1.0},
        "roofline": {"bound": "alu",
                     # the refresh phase: the record kernel, then the copy of the
                     # save base states from the tape
                     "kernel": ("erk_adjoint_kernel" if dominant == "adjoint" else
                                "erk_forward_kernel + save_bases_kernel")
                               + f" ({cfg['system']}, {cfg['method']}, f64"
                               f"{', refresh' if dominant == 'refresh' else ''})",
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None},
        "kernels_ms": {"refresh": ref_ms, "adjoint": adj_ms},
        "drift": {"trajectories_keeping_their_mesh": kept_all,
                  "old_steps_kept": kept_steps,
                  "trials_per_traj": stats["trials"] / n,
                  "accepted_per_traj": stats["steps_accepted"] / n},
        "context_same_step": {"fresh_record": ctx["record"],
                              "stale_mesh_replay_unchecked": ctx["stale_replay"]},
    }
    print(json.dumps(out), flush=True)


def solve_bench(args):
    """The forward-only solve (`ensemble_solve`: the adaptive loop and the
    states at the save times, no record, no gradient) on a workload: the
    forward-only throughput of the paper's fused kernels (Section 4.1).  The
    work counts come from one record of the same inputs outside the timed
    steps (the solve takes the same steps, to the bit)."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import flops
    from paper_2609_02876_amd import workloads as W

    cfg, y0, p, st = W.make(args.workload, n=args.n)
    n = cfg["n"]
    shared = bool(cfg.get("shared"))
    save = list(st) if cfg["n_save"] else None
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f32 = cfg.get("dtype", "f64") == "f32"
    tdt = torch.float32 if f32 else torch.float64
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=tdt, device=dev)
    p_d = (torch.tensor(np.ascontiguousarray(p), dtype=tdt, device=dev) if shared else
           torch.tensor(np.ascontiguousarray(p.T), dtype=tdt, device=dev))
    args_common = (cfg["system"], cfg["method"], y0_d, p_d, cfg["t0"], cfg["t1"], cfg["rtol"],
                   cfg["atol"])
    # the work of the solve, from a record of the same inputs
    m = min(n, 8192)
    pilot = B.ensemble_record(cfg["system"], cfg["method"], y0_d[:, :m].contiguous(),
                              p_d if shared else p_d[:, :m].contiguous(), cfg["t0"], cfg["t1"],
                              cfg["rtol"], cfg["atol"], save_times=save, params_shared=shared,
                              steps_hint=4096)
    s_pilot = pilot.steps().double()
    cap_cpu = int(s_pilot.max().item() * 1.5) + 64
    hint = B.steps_hint_for(float(s_pilot.mean().item()), margin=1.12)
    del pilot
    rec = B.ensemble_record(*args_common, save_times=save, params_shared=shared, steps_hint=hint)
    stats = B.ensemble_record_stats(rec)
    ref_states = rec.y_save.clone()
    del rec
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        calibration_copy(args.copy_calibration, dev)

    def step(events=None):
        if events:
            events[0].record(stream)
        out = B.ensemble_solve(*args_common, save_times=save, params_shared=shared)
        if events:
            events[1].record(stream)
        return out

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for _ in range(args.warmup):
        ys, status = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ys, status = step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = int((status != 0).sum().item())
    if bad:
        raise RuntimeError(f"{bad} trajectories did not finish (status != OK)")
    if not torch.equal(ys, ref_states):
        raise RuntimeError("the solve's states differ from the record's")
    solve_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    f_solve = flops.record_flops(cfg["method"], cfg["system"], stats["trials"],
                                 stats["steps_accepted"], stats["side_steps"])
    achieved = f_solve / (solve_ms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
    traffic = None
    tr = load_traffic(args.traffic, args.workload + "_solve")
    if tr is not None and tr.get("n") == n:
        traffic = tr.get("record")
    out = {
        "metric": "trajectories/s (forward-only solve, states at the save times)",
        "value": n * args.steps / wall, "unit": "trajectories/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "mode": "solve", "system": cfg["system"],
                   "method": cfg["method"], "n": n, "t_span": [cfg["t0"], cfg["t1"]],
                   "rtol": cfg["rtol"], "atol": cfg["atol"], "n_save": cfg["n_save"],
                   "params_shared": shared},
        "roofline": {"bound": "alu",
                     "kernel": f"erk_forward_kernel ({cfg['system']}, {cfg['method']}, solve)",
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic},
        "kernels_ms": {"solve": solve_ms},
        "algorithmic_flop": {"solve": f_solve},
        "record_stats": {"accepted_per_traj": stats["steps_accepted"] / n,
                         "trials_per_traj": stats["trials"] / n},
    }
    if not args.no_cpu_baseline:
        O = load_oracle()
        so = {"lorenz": O.LORENZ, "vdp": O.VDP, "robertson": O.ROBERTSON, "hires": O.HIRES,
              "linear": O.LINEAR, "ude": O.LV_UDE}[cfg["system"]]
        mo = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}[cfg["method"]]

        def run(mm):
            t = time.perf_counter()
            O.record(so, mo, y0[:mm], p if shared else p[:mm], cfg["t0"], cfg["t1"], cfg["rtol"],
                     cfg["atol"], save_t=save, cap=cap_cpu, params_shared=shared)
            return time.perf_counter() - t

        m2 = 2048
        dt2 = run(m2)
        for _ in range(3):
            if dt2 >= 0.7 * args.cpu_seconds or m2 >= n:
                break
            m2 = int(min(n, m2 * args.cpu_seconds / max(dt2, 1e-3)))
            m2 = max(64, (m2 // 64) * 64)
            dt2 = run(m2)
        out["cpu_baseline"] = {
            "value": m2 / dt2, "unit": "trajectories/s", **cpu_info(), "kind": "oracle",
            "sample": f"first {m2} trajectories, the oracle's adaptive solve, {dt2:.1f} s"}
    print(json.dumps(out), flush=True)


def forward_bench(args):
    """Record + one forward-mode pass per parameter (the same unit tangent in
    every trajectory), each pass returning every trajectory's derivative of
    the loss with respect to that parameter: the per-trajectory parameter
    gradient by forward mode on the recorded mesh."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import flops
    from paper_2609_02876_amd import workloads as W

    cfg, y0, p, st = W.make(args.workload, n=args.n)
    if cfg.get("shared") or cfg["system"] in ("ude", "hires"):
        raise SystemExit("forward mode is built for per-trajectory parameters of Lorenz, "
                         "Van der Pol, the damped rotation and Robertson")
    n = cfg["n"]
    save = list(st) if cfg["n_save"] else None
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f32 = cfg.get("dtype", "f64") == "f32"
    tdt = torch.float32 if f32 else torch.float64
    y0_d = torch.tensor(np.ascontiguousarray(y0.T), dtype=tdt, device=dev)
    p_d = torch.tensor(np.ascontiguousarray(p.T), dtype=tdt, device=dev)
    npar = p.shape[1]
    args_common = (cfg["system"], cfg["method"], y0_d, p_d, cfg["t0"], cfg["t1"], cfg["rtol"],
                   cfg["atol"])
    m = min(n, 8192)
    pilot = B.ensemble_record(cfg["system"], cfg["method"], y0_d[:, :m].contiguous(),
                              p_d[:, :m].contiguous(), cfg["t0"], cfg["t1"], cfg["rtol"],
                              cfg["atol"], save_times=save, steps_hint=4096)
    s_pilot = pilot.steps().double()
    cap_cpu = int(s_pilot.max().item() * 1.5) + 64
    hint = B.steps_hint_for(float(s_pilot.mean().item()), margin=1.12)
    del pilot
    nbytes = B.ensemble_record_bytes(cfg["system"], cfg["method"], n, cfg["t0"], cfg["t1"], hint,
                                     cfg["n_save"], tdt, 0)
    pool = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    tangents = []
    for k in range(npar):
        t = torch.zeros((npar, n), dtype=tdt, device=dev)
        t[k] = 1.0
        tangents.append(t)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        calibration_copy(args.copy_calibration, dev)

    def step(events=None):
        if events:
            events[0].record(stream)
        rec = B.ensemble_record(*args_common, save_times=save, pool=pool, steps_per_traj=hint)
        if events:
            events[1].record(stream)
        grads = [B.ensemble_jvp(rec, None, t, want_states=False)[1] for t in tangents]
        if events:
            events[2].record(stream)
        return rec, grads

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for _ in range(args.warmup):
        rec, grads = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        rec, grads = step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bad = int((rec.status != 0).sum().item())
    if bad:
        raise RuntimeError(f"{bad} trajectories did not finish (status != OK)")
    rec_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    fwd_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    pass_ms = fwd_ms / npar
    stats = B.ensemble_record_stats(rec)
    n_saves = n * (cfg["n_save"] or 1)
    f_rec = flops.record_flops(cfg["method"], cfg["system"], stats["trials"],
                               stats["steps_accepted"], stats["side_steps"])
    f_pass = flops.jvp_flops(cfg["method"], cfg["system"], stats["steps_accepted"],
                             stats["side_steps"], n_saves)
    dominant = "jvp" if fwd_ms >= rec_ms else "record"
    f_dom, ms_dom = (f_pass, pass_ms) if dominant == "jvp" else (f_rec, rec_ms)
    achieved = f_dom / (ms_dom * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
    traffic = None
    tr = load_traffic(args.traffic, args.workload + "_forward")
    if tr is not None and tr.get("n") == n:
        traffic = tr.get(dominant)
    ms_per_step = wall * 1e3 / args.steps
    out = {
        "metric": "trajectory-gradients/s (record + forward mode, one pass per parameter)",
        "value": n * args.steps / wall, "unit": "trajectory-gradients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if f32 else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "mode": "forward", "system": cfg["system"],
                   "method": cfg["method"], "n": n, "t_span": [cfg["t0"], cfg["t1"]],
                   "rtol": cfg["rtol"], "atol": cfg["atol"], "n_save": cfg["n_save"],
                   "passes": npar, "loss": "sum of squared save states",
                   "gradient": "per-trajectory params, one forward pass each"},
        "roofline": {"bound": "alu",
                     "kernel": (f"jvp_kernel ({cfg['system']}, {cfg['method']})"
                                if dominant == "jvp" else
                                f"erk_forward_kernel ({cfg['system']}, {cfg['method']})"),
                     "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic},
        "kernels_ms": {"record": rec_ms, "jvp_per_pass": pass_ms},
        "algorithmic_flop": {"record": f_rec, "jvp_per_pass": f_pass,
                             "total_tflops": (f_rec + npar * f_pass) / (ms_per_step * 1e-3) / 1e12},
    }
    if not args.no_cpu_baseline:
        O = load_oracle()
        so = {"lorenz": O.LORENZ, "vdp": O.VDP, "robertson": O.ROBERTSON,
              "linear": O.LINEAR}[cfg["system"]]
        mo = {"tsit5": O.TSIT5, "vern7": O.VERN7, "rodas4": O.RODAS, "ros23": O.ROS23}[cfg["method"]]

        def run(mm):
            t = time.perf_counter()
            r = O.record(so, mo, y0[:mm], p[:mm], cfg["t0"], cfg["t1"], cfg["rtol"], cfg["atol"],
                         save_t=save, cap=cap_cpu)
            for k in range(npar):
                dp = np.zeros_like(p[:mm])
                dp[:, k] = 1.0
                ys, dys = O.replay_dual(so, mo, y0[:mm], p[:mm], np.zeros_like(y0[:mm]), dp, r)
                np.sum(2.0 * ys * dys, axis=(1, 2))
            return time.perf_counter() - t

        m2 = 2048
        dt2 = run(m2)
        for _ in range(3):
            if dt2 >= 0.7 * args.cpu_seconds or m2 >= n:
                break
            m2 = int(min(n, m2 * args.cpu_seconds / max(dt2, 1e-3)))
            m2 = max(64, (m2 // 64) * 64)
            dt2 = run(m2)
        out["cpu_baseline"] = {
            "value": m2 / dt2, "unit": "trajectory-gradients/s", **cpu_info(),
            "kind": "oracle",
            "sample": f"first {m2} trajectories, record + {npar} dual-number replays, {dt2:.1f} s"}
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Mixed ensemble-gradient jobs through the server (continuous batching)
    against the same trajectories as one-shot launches (each (system, rtol)
    group's trajectories in launches of up to 2^20) and as plain per-job
    launches.  Jobs: systems uniform over Lorenz, Van der Pol (Tsit5),
    Robertson and HIRES (Rodas4); lanes log-uniform in 2^8..2^max;
    rtol in {1e-4, 1e-6, 1e-8} (HIRES: 1e-4, 1e-6); atol = 1e-2 rtol
    (explicit) or 1e-4 rtol (stiff); loss = |y(t1)|^2; parameters seeded by
    the job id; FP64.  Served passes: everything submitted at once (the
    served capacity), then Poisson streams whose offered trajectory rate is a
    fraction of the one-shot capacity; each stream submits the job list
    --serve-repeat times, so that its window lasts repeat x total / (load x
    capacity) seconds."""
    import numpy as np
    import torch

    from paper_2609_02876_amd import binding as B
    from paper_2609_02876_amd import serving as SV
    from paper_2609_02876_amd import workloads as W

    def note(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    span = {"lorenz": 10.0, "vdp": 6.3, "robertson": 1e5, "hires": 321.8122}
    method = {"lorenz": "tsit5", "vdp": "tsit5", "robertson": "rodas4", "hires": "rodas4"}
    rng = np.random.default_rng(2026)
    dev = torch.device("cuda:0")
    span_log2 = args.serve_max_log2 - 8
    jobs = []
    for k in range(args.serve_jobs):
        system = ["lorenz", "vdp", "robertson", "hires"][int(rng.integers(0, 4))]
        n = int(round(2 ** (8 + span_log2 * rng.random())))
        rtols = [1e-4, 1e-6] if system == "hires" else [1e-4, 1e-6, 1e-8]
        rtol = rtols[int(rng.integers(0, len(rtols)))]
        atol = rtol * (1e-2 if system in ("lorenz", "vdp") else 1e-4)
        y0, p = W.GENERATORS[system](n, seed=k)
        jobs.append(dict(system=system, method=method[system], n=n, rtol=rtol, atol=atol,
                         y0=torch.tensor(np.ascontiguousarray(y0.T), device=dev),
                         p=torch.tensor(np.ascontiguousarray(p.T), device=dev)))
    groups = {}
    for j in jobs:
        groups.setdefault((j["system"], j["rtol"]), []).append(j)
    total = sum(j["n"] for j in jobs)
    note(f"{len(jobs)} jobs, {total} trajectories, {len(groups)} (system, rtol) groups")

    # memory plan per group: the longest trajectory of a pilot record (up to
    # 16384 trajectories of the group's largest job), +20 %
    hints = {}
    for (system, rtol), js in groups.items():
        j = max(js, key=lambda x: x["n"])
        m = min(j["n"], 16384)
        h = B.ensemble_record(system, j["method"], j["y0"][:, :m].contiguous(),
                              j["p"][:, :m].contiguous(), 0.0, span[system], rtol, j["atol"],
                              steps_hint=4096)
        hints[(system, rtol)] = int(h.steps().max().item() * 1.2) + 32
        del h
    for j in jobs:
        j["hint"] = hints[(j["system"], j["rtol"])]
    note("pilot plans done")

    def run_plain(j, keep=False):
        h = B.ensemble_record(j["system"], j["method"], j["y0"], j["p"], 0.0, span[j["system"]],
                              j["rtol"], j["atol"], steps_hint=j["hint"])
        gp, gy, ll = B.ensemble_adjoint(h, want_y0=True, want_loss=True)
        return (h.y_save, h.status, gp, gy, ll) if keep else None

    # one-shot: each (system, rtol) group's trajectories as one ensemble, in
    # launches of at most 2^20 trajectories.  Each group is run once untimed
    # (which also leaves its record buffers in torch's cache) and then timed,
    # so the timed launches allocate nothing; the cache is emptied between
    # groups to bound the memory held.
    chunk = 1 << 20
    t_oneshot = 0.0
    for key, js in groups.items():
        y0 = torch.cat([j["y0"] for j in js], 1)
        pp = torch.cat([j["p"] for j in js], 1)
        parts = [dict(js[0], y0=y0[:, a:a + chunk].contiguous(), p=pp[:, a:a + chunk].contiguous())
                 for a in range(0, y0.shape[1], chunk)]
        del y0, pp
        torch.cuda.empty_cache()
        for c in parts:
            run_plain(c)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for c in parts:
            run_plain(c)
        torch.cuda.synchronize()
        t_oneshot += time.perf_counter() - t
        del parts
    torch.cuda.empty_cache()
    cap = total / t_oneshot
    note(f"one-shot: {t_oneshot:.2f} s, {cap:.4g} trajectory-gradients/s")

    # plain per-job launches; the outputs of a sample of jobs are kept to
    # check the served results against them
    sample = sorted(set(int(x) for x in rng.choice(len(jobs), 16, replace=False)))
    plain = {}
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k, j in enumerate(jobs):
        out = run_plain(j, keep=k in sample)
        if out is not None:
            plain[k] = out
    torch.cuda.synchronize()
    t_perjob = time.perf_counter() - t
    note(f"per-job launches: {t_perjob:.2f} s")

    # the pool: a third of what all the jobs' records would take at once,
    # at least 2.5 times the largest job, at most 96 GB
    need = [B.ensemble_record_bytes(j["system"], j["method"], j["n"], 0.0, span[j["system"]],
                                    j["hint"]) for j in jobs]
    pool = int(min(max(sum(need) // 3, int(2.5 * max(need)), 4 << 30), 96e9))
    torch.cuda.empty_cache()

    def serve(load, keep=(), repeat=1):
        srv = SV.Server(pool, n_slots=4)
        seq = [k for _ in range(repeat) for k in rng.permutation(len(jobs))] if repeat > 1 \
            else list(range(len(jobs)))
        arrive = np.cumsum(rng.exponential(total / len(jobs) / (load * cap), len(seq))) \
            if load else np.zeros(len(seq))
        served = {}
        t0 = time.perf_counter()
        for a, k in zip(arrive, seq):
            j = jobs[k]
            while time.perf_counter() - t0 < a:
                srv.progress()
            sj = srv.submit(j["system"], j["method"], j["y0"], j["p"], 0.0, span[j["system"]],
                            j["rtol"], j["atol"], steps_hint=j["hint"])
            if k in keep:
                served[k] = sj
        srv.drain()
        st = srv.stats()
        st["window_s"] = float(arrive[-1])
        srv.close()
        return st, served

    serve(0)  # warm-up
    sat, served = serve(0, keep=sample)   # everything submitted at once: the served capacity
    same = all(torch.equal(served[k].y_save, plain[k][0]) and
               torch.equal(served[k].status, plain[k][1]) and
               torch.equal(served[k].grad_params, plain[k][2]) and
               torch.equal(served[k].grad_y0, plain[k][3]) and
               torch.equal(served[k].loss, plain[k][4]) for k in sample)
    del served, plain
    note(f"saturated: {sat['throughput']:.4g} trajectory-gradients/s, "
         f"{sat['throughput'] / cap:.3f} of one-shot; sampled jobs equal per-job runs: {same}")
    loads = {}
    for x in [float(v) for v in args.serve_loads.split(",") if v]:
        st, _ = serve(x, repeat=args.serve_repeat)
        loads[str(x)] = {"offered": x * cap, "window_s": st["window_s"], "busy_s": st["busy_s"],
                         "throughput": st["throughput"],
                         "throughput_over_offered": st["throughput"] / (x * cap),
                         "p50_ms": st["p50_latency_s"] * 1e3, "p99_ms": st["p99_latency_s"] * 1e3,
                         "mean_ms": st["mean_latency_s"] * 1e3,
                         "jobs": int(st["completed"]), "retried": st["retried"],
                         "failed": st["failed"]}
        note(f"load {x}: {loads[str(x)]}")
    out = {
        "metric": "served trajectory-gradients/s (mixed jobs, continuous batching)",
        "value": sat["throughput"], "unit": "trajectory-gradients/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": sat["busy_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serve_mix", "jobs": len(jobs), "trajectories": total,
                   "systems": ["lorenz", "vdp", "robertson", "hires"],
                   "lanes": f"2^(8+{span_log2}u)", "rtol": [1e-4, 1e-6, 1e-8], "slots": 4,
                   "pool_gb": pool / 1e9, "oneshot_launch_max": chunk,
                   "poisson_repeat": args.serve_repeat},
        "oneshot_throughput": cap,
        "served_over_oneshot": sat["throughput"] / cap,
        "perjob_throughput": total / t_perjob,
        "saturated": {"p50_ms": sat["p50_latency_s"] * 1e3, "p99_ms": sat["p99_latency_s"] * 1e3,
                      "retried": sat["retried"], "failed": sat["failed"],
                      "pool_peak_gb": sat["pool_peak"] / 1e9},
        "sampled_jobs_equal_perjob": bool(same),
        "poisson_loads": loads,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
