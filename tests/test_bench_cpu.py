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
                             "kernels": {"k_a@512": {"bytes_per_launch": 7e9}, "k_b@512": {"bytes_per_launch": 14e9}}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    passes = [{"kernel": "void mg::k_a(int)", "launches": 12}, {"kernel": "void mg::k_b(int)", "launches": 6}]
    r = bench.v_cycle_counted(passes, 6, 512, 4.0)
    # per cycle: (2 x 7 + 1 x 14) GB x 8/7 = 32 GB in 4 ms
    assert r["bytes_per_cycle"] == pytest.approx(32e9)
    assert r["achieved"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(1.0)
    passes.append({"kernel": "void mg::k_c(int)", "launches": 6})
    assert bench.v_cycle_counted(passes, 6, 512, 4.0) is None
