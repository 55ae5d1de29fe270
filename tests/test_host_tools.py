"""Host logic of the measurement tools, on the CPU: the source hash that
decides whether committed counters still describe the code, the parsing of
rocprofv3 CSV output, the calibrated HBM traffic, the profile records bench.py
reads, and the one-GPU guard of bench.py."""
import csv
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

from paper_1806_08741_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_lines_drop_comments_and_blank_lines():
    src = 'int a = 1;  // one\n\n   // only a comment\nconst char* s = "a//b"; // tail\n'
    assert profsum.code_lines(src) == 'int a = 1;\nconst char* s = "a//b";'


def test_every_kernel_class_hashes_existing_sources():
    for k, (pat, files) in profsum.KERNELS.items():
        for f in files:
            assert os.path.exists(os.path.join(profsum.HERE, "csrc", f)), (k, f)
        h = profsum.kernel_source_hash(k)
        assert len(h) == 16 and h == profsum.kernel_source_hash(k)


def test_short_names():
    assert profsum.short_name(
        "void sslic::(anonymous namespace)::sweep_kernel<unsigned char, 2, 3, true>(sslic::Geo)"
    ) == "sweep_kernel<unsigned char, 2, 3, true>"
    assert profsum.short_name("cc_resolve_kernel(int*)") == "cc_resolve_kernel"


def _counter_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_pmc_means_per_dispatch_and_traffic_calibration(tmp_path):
    k = "void sslic::(anonymous namespace)::sweep_kernel<unsigned char, 2, 3, true>(x)"
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>(x)"
    # two sweep dispatches, split over two XCD rows each (values add per dispatch)
    _counter_csv(str(tmp_path / "f" / "a" / "x_counter_collection.csv"),
                 [(1, k, "FETCH_SIZE", 300.0), (1, k, "FETCH_SIZE", 100.0),
                  (2, k, "FETCH_SIZE", 500.0), (2, k, "FETCH_SIZE", 300.0)])
    _counter_csv(str(tmp_path / "w" / "x_counter_collection.csv"),
                 [(1, k, "WRITE_SIZE", 1000.0), (2, k, "WRITE_SIZE", 2000.0)])
    # the copy of 1 MiB reads back 512 KiB of FETCH_SIZE and 1024 KiB of WRITE_SIZE
    _counter_csv(str(tmp_path / "cf" / "x_counter_collection.csv"), [(7, neg, "FETCH_SIZE", 512.0)])
    _counter_csv(str(tmp_path / "cw" / "x_counter_collection.csv"), [(7, neg, "WRITE_SIZE", 1024.0)])
    per = profsum.pmc(str(tmp_path / "f"), "sweep_kernel")
    rec = per["sweep_kernel<unsigned char, 2, 3, true>"]
    assert rec["_dispatches"] == 2 and rec["FETCH_SIZE"] == 600.0
    a = SimpleNamespace(kernel="sweep", workload="w", fetch=str(tmp_path / "f"),
                        write=str(tmp_path / "w"), copy_fetch=str(tmp_path / "cf"),
                        copy_write=str(tmp_path / "cw"), mib=1)
    t = profsum.traffic(a)
    assert t["copy_calibration"]["fetch_factor"] == 2.0
    assert t["copy_calibration"]["write_factor"] == 1.0
    assert t["fetch_bytes_per_launch"] == round(600.0 * 1024 * 2.0)
    assert t["write_bytes_per_launch"] == round(1500.0 * 1024)
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    assert t["source_hash"] == profsum.kernel_source_hash("sweep")


def test_stats_sorted_by_total_time(tmp_path):
    p = tmp_path / "s" / "x_kernel_stats.csv"
    os.makedirs(p.parent)
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["void sslic::a_kernel(int)", 2, 2000, 1000, 10.0])
        w.writerow(["void sslic::b_kernel(int)", 1, 9000, 9000, 90.0])
    rows = profsum.stats(str(tmp_path / "s"))
    assert [r["name"] for r in rows] == ["b_kernel", "a_kernel"]
    assert rows[0]["total_ms"] == 0.009 and rows[1]["mean_us"] == 1.0


def _bench_module():
    sys.path.insert(0, ROOT)
    import importlib
    import bench
    return importlib.reload(bench)


def test_load_profile_only_on_matching_source(tmp_path, monkeypatch):
    bench = _bench_module()
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    good = {"kernel": "sweep", "source_hash": profsum.kernel_source_hash("sweep"),
            "bytes_per_launch": 123}
    with open(tmp_path / "profiles" / "traffic_sweep_wl.json", "w") as fh:
        json.dump(good, fh)
    assert bench.load_traffic("sweep", "wl") == 123
    stale = dict(good, source_hash="0" * 16)
    with open(tmp_path / "profiles" / "traffic_sweep_wl.json", "w") as fh:
        json.dump(stale, fh)
    assert bench.load_traffic("sweep", "wl") is None
    assert bench.load_traffic("sweep", "missing") is None


def test_committed_traffic_records_name_their_kernel_and_workload():
    d = os.path.join(ROOT, "profiles")
    for f in os.listdir(d):
        if f.startswith("traffic_") and f.endswith(".json"):
            with open(os.path.join(d, f)) as fh:
                r = json.load(fh)
            assert f == f"traffic_{r['kernel']}_{r['workload']}.json"
            assert abs(r["bytes_per_launch"] - r["fetch_bytes_per_launch"] - r["write_bytes_per_launch"]) <= 1
            assert r["kernel"] in profsum.KERNELS


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
