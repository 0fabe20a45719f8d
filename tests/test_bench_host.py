"""Host logic of bench.py that needs no GPU: the conversion of rocprofv3
FETCH_SIZE / WRITE_SIZE counter output into per-launch HBM bytes, and the
source-hash gate on measured traffic."""
import csv
import json
import os

import bench

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
FWD = "void ens::erk_forward_kernel<ens::Lorenz, ens::Tsit5, double, 1, false>(ens::FwdArgs)"
SOLVE = "void ens::erk_forward_kernel<ens::Lorenz, ens::Tsit5, double, 0, false>(ens::FwdArgs)"
ADJ = "void ens::erk_adjoint_kernel<ens::Lorenz, ens::Tsit5, double, false, false>(ens::AdjArgs)"


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (grid, name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Grid_Size": grid, "Kernel_Name": name,
                        "Counter_Name": counter, "Counter_Value": value})


def test_write_traffic_calibrates_and_picks_the_timed_launches(tmp_path, capsys):
    mib = 1024
    # the copy of 1 GiB counts half its bytes fetched and all of them written
    fetch = [(131072, "__amd_rocclr_copyBuffer", 524288.0), (512, "__amd_rocclr_copyBuffer", 2.0),
             (8192, FWD, 999.0),                 # pool-sizing pilot (smaller grid)
             (1048576, SOLVE, 5000.0),           # a forward-only solve of the same size, once
             (1048576, FWD, 100.0), (1048576, FWD, 110.0), (1048576, FWD, 120.0),
             (1048576, ADJ, 4000.0), (1048576, ADJ, 4200.0)]
    write = [(131072, "__amd_rocclr_copyBuffer", 1048576.0),
             (1048576, SOLVE, 7.0),
             (1048576, FWD, 3000.0), (1048576, FWD, 3000.0), (1048576, FWD, 3300.0),
             (1048576, ADJ, 50.0), (1048576, ADJ, 70.0)]
    _write(tmp_path / "f", "FETCH_SIZE", fetch)
    _write(tmp_path / "w", "WRITE_SIZE", write)
    out = tmp_path / "t.json"
    tr = bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), "lorenz_2p20_t10", 1 << 20,
                             mib, path=str(out))
    capsys.readouterr()
    assert tr["calibration"]["fetch_factor"] == 2.0 and tr["calibration"]["write_factor"] == 1.0
    assert tr["record_detail"]["dispatches"] == 3 and tr["adjoint_detail"]["dispatches"] == 2
    assert tr["record"] == (110.0 * 2.0 + 3100.0) * 1024
    assert tr["adjoint"] == (4100.0 * 2.0 + 60.0) * 1024
    assert json.load(open(out))["source_hash"] == bench.kernel_source_hash()


DEF = "void ens::erk_record_deferred_kernel<ens::Lorenz, ens::Tsit5, double>(ens::FwdArgs)"
SAV = "void ens::erk_saves_kernel<ens::Lorenz, ens::Tsit5, double>(ens::FwdArgs)"


def test_write_traffic_adds_the_two_launches_of_a_deferred_record(tmp_path, capsys):
    # the record loop and the save-state kernel are one record; the pilot of
    # the pool plan (a smaller grid of the one-launch record) is left out
    fetch = [(131072, "__amd_rocclr_copyBuffer", 1048576.0),
             (8192, FWD, 999.0),
             (1048576, DEF, 100.0), (1048576, SAV, 40.0), (1048576, DEF, 120.0),
             (1048576, SAV, 60.0), (1048576, ADJ, 4000.0)]
    write = [(131072, "__amd_rocclr_copyBuffer", 1048576.0),
             (8192, FWD, 5.0),
             (1048576, DEF, 3000.0), (1048576, SAV, 10.0), (1048576, DEF, 3200.0),
             (1048576, SAV, 30.0), (1048576, ADJ, 50.0)]
    _write(tmp_path / "f", "FETCH_SIZE", fetch)
    _write(tmp_path / "w", "WRITE_SIZE", write)
    tr = bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), "lorenz_2p20_t10", 1 << 20,
                             1024, path=str(tmp_path / "t.json"))
    capsys.readouterr()
    assert tr["record"] == (110.0 + 50.0 + 3100.0 + 20.0) * 1024
    assert tr["record_detail"]["dispatches"] == 2
    assert [k.split("<")[0] for k in tr["record_detail"]["kernels"]] == [
        "void ens::erk_record_deferred_kernel", "void ens::erk_saves_kernel"]


def test_traffic_is_used_only_for_the_sources_it_was_measured_on(tmp_path):
    good = {"n": 8, "source_hash": bench.kernel_source_hash(), "record": 1.0, "adjoint": 2.0}
    stale = dict(good, source_hash="0" * 16)
    (tmp_path / "good.json").write_text(json.dumps(good))
    (tmp_path / "stale.json").write_text(json.dumps(stale))
    assert bench.load_traffic(str(tmp_path / "good.json"), "x")["adjoint"] == 2.0
    assert bench.load_traffic(str(tmp_path / "stale.json"), "x") is None
    assert bench.load_traffic(str(tmp_path / "absent.json"), "x") is None
