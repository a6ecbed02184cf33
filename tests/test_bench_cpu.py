"""Host logic of bench.py (no GPU): the one-GPU contract, the traffic lookup and its staleness
check against the kernel sources, the V-cycle efficiency figure and the kernel-name keys."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_short_name_strips_namespaces_and_arguments():
    k = "void mg::(anonymous namespace)::k_fused<double, 2, 16, false, 0, 0, false, 2>(mg::(anonymous namespace)::FusedArgs)"
    assert bench.short_name(k) == "k_fused<double, 2, 16, false, 0, 0, false, 2>"


def test_v_cycle_efficiency():
    # 57 B per DoF at 512^3 in 4 ms: 57 * 2^27 / 4e-3 bytes per second
    e = bench.v_cycle_efficiency(512, 4.0)
    assert e["bytes_per_dof"] == 57.0
    assert e["achieved"] == pytest.approx(57.0 * 512 ** 3 / 4e-3 / 1e9)
    assert e["frac"] == pytest.approx(e["achieved"] / 8000.0)


def test_traffic_lookup_and_staleness(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": bench.kernel_source_hash(),
                             "kernels": {"k_x<1>@512": {"bytes_per_launch": 123.0}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("void mg::k_x<1>(int)", 512) == 123.0
    assert bench.measured_traffic("void mg::k_x<1>(int)", 256) is None
    assert bench.measured_traffic("void mg::k_y<1>(int)", 512) is None
    # counters taken on other kernel sources are not reported
    f.write_text(json.dumps({"source_hash": "0" * 16, "kernels": {"k_x<1>@512": {"bytes_per_launch": 123.0}}}))
    assert bench.measured_traffic("void mg::k_x<1>(int)", 512) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.measured_traffic("void mg::k_x<1>(int)", 512) is None



def test_v_cycle_counted(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": bench.kernel_source_hash(),
                             "v_cycle": {"512": {"bytes_per_cycle": 32e9, "cycles": 5}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    r = bench.v_cycle_counted(512, 4.0)
    assert r["bytes_per_cycle"] == pytest.approx(32e9)
    assert r["achieved"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(1.0)
    assert r["over_algorithmic"] == pytest.approx(32e9 / (57.0 * 512 ** 3))
    assert bench.v_cycle_counted(256, 4.0) is None
    f.write_text(json.dumps({"source_hash": "0" * 16, "v_cycle": {"512": {"bytes_per_cycle": 32e9, "cycles": 5}}}))
    assert bench.v_cycle_counted(512, 4.0) is None


DOWN = "void mg::(anonymous namespace)::k_march<double, 8, false, false, true, false>(mg::(anonymous namespace)::MarchArgs)"
UP = "void mg::(anonymous namespace)::k_march<double, 8, true, true, true, false>(mg::(anonymous namespace)::MarchArgs)"


def _counter_csv(path, counter, rows):
    import csv
    path.mkdir()
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, grid, v) in enumerate(rows):
            w.writerow([i + 1, grid, name, counter, v])


def test_summarize_counters_sums_whole_cycles(tmp_path):
    """Calibration from the 1 GiB copy; a V-cycle is every dispatch from one finest-level down
    pass to the next (coarser down passes included); spans holding a once-per-solve kernel are
    left out."""
    seq = [("__amd_rocclr_copyBuffer", 131072, None), ("void mg::k_source(A)", 99, 7.0),
           (DOWN, 1000, 100.0), (DOWN, 500, 50.0), ("void mg::k_tail<double, true>(A)", 10, 5.0), (UP, 1000, 200.0),
           ("void mg::k_sum_partials(A)", 9, 1.0),
           (DOWN, 1000, 100.0), (DOWN, 500, 50.0), ("void mg::k_tail<double, true>(A)", 10, 5.0), (UP, 1000, 200.0),
           ("void mg::k_sum_partials(A)", 9, 1.0),
           (DOWN, 1000, 100.0), ("void mg::k_shift(A)", 99, 3.0), ("void mg::k_source(A)", 99, 7.0),
           (DOWN, 1000, 100.0)]
    _counter_csv(tmp_path / "f", "FETCH_SIZE", [(k, g, 524288.0 if v is None else v) for k, g, v in seq])
    _counter_csv(tmp_path / "w", "WRITE_SIZE", [(k, g, 1048576.0 if v is None else v / 2) for k, g, v in seq])
    out = tmp_path / "out"
    out.mkdir()
    bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), 512, str(out))
    t = json.loads((out / "traffic.json").read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    vc = t["v_cycle"]["512"]
    assert vc["cycles"] == 2
    assert vc["read_bytes"] == pytest.approx(356.0 * 1024 * 2)
    assert vc["write_bytes"] == pytest.approx(178.0 * 1024)
    k = t["kernels"]["k_march<double, 8, false, false, true, false>@512"]
    assert k["grid"] == 1000 and k["dispatches"] == 4
    assert k["read_bytes"] == pytest.approx(100.0 * 1024 * 2)
    assert (out / "hbm_traffic_c2_512.md").exists()
