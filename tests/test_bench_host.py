"""Host-side pieces of the benchmark's measurement contract (CPU only): the
single-GPU guard, the kernel-name mapping to rocprofv3's demangled names,
the HBM-traffic summary from two counter runs scaled by a device copy, and
the source fingerprint that invalidates a stale traffic record."""
import csv
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def test_rocprof_names():
    assert bench.rocprof_name("eri_tile_2221") == "void jk::k_eri_tile<jk::Eri2221<double>, double>(jk::EriTileArgs)"
    assert bench.rocprof_name("eri_tile_fp32_1010") == "void jk::k_eri_tile<jk::Eri1010<float>, float>(jk::EriTileArgs)"
    assert bench.rocprof_name("digest_c_2110") == "void jk::k_digest_c<2, 1, 1, 0, double, true, false>(jk::DigestArgs)"
    assert bench.rocprof_name("digest_d_2110") == "void jk::k_digest_d4<2, 1, 1, 0, true>(jk::DigestArgs)"
    assert bench.rocprof_name("digest_d_2222") == "void jk::k_digest_d<2, 2, 2, 2, double, true>(jk::DigestArgs)"
    assert (bench.rocprof_name("digest_d_fp32_2221", g16=False)
            == "void jk::k_digest_d<2, 2, 2, 1, float, false>(jk::DigestArgs)")


def _counter_dir(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, value) in enumerate(rows):
            w.writerow([i, name, counter, value])


def test_pmc_summary_scales_each_counter_by_the_copy(tmp_path):
    copy_mib = 64
    target = bench.rocprof_name("eri_tile_2221")
    copy = "__amd_rocclr_copyBuffer"
    # as on MI355X, the copy reads as a little over half its size in
    # FETCH_SIZE and in full in WRITE_SIZE
    fetch_copy = copy_mib * 1024 / 2 + 15.0
    _counter_dir(str(tmp_path / "F"), "FETCH_SIZE",
                 [(copy, fetch_copy), (target, 1000.0), (target, 1200.0), ("other", 5.0)])
    _counter_dir(str(tmp_path / "W"), "WRITE_SIZE",
                 [(copy, copy_mib * 1024), (target, 300.0), (target, 500.0)])
    out = tmp_path / "t.json"
    bench.pmc_summary(str(tmp_path / "F"), str(tmp_path / "W"), "eri_tile_2221", copy_mib, str(out))
    rec = json.loads(out.read_text())
    sf = copy_mib * 1024 / fetch_copy
    assert abs(rec["FETCH_SIZE"]["copy_scale"] - sf) < 1e-12
    assert abs(rec["WRITE_SIZE"]["copy_scale"] - 1.0) < 1e-12
    assert abs(rec["FETCH_SIZE"]["bytes_per_launch"] - 1100.0 * 1024 * sf) < 1e-6
    assert abs(rec["WRITE_SIZE"]["bytes_per_launch"] - 400.0 * 1024) < 1e-6
    assert abs(rec["hbm_bytes_per_launch"] - (1100.0 * 1024 * sf + 400.0 * 1024)) < 1e-6
    assert rec["FETCH_SIZE"]["dispatches"] == 2
    assert rec["source_sha256"] == bench.kernel_sources_sha256()


def test_traffic_record_is_ignored_once_the_sources_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    rec = {"kernel": "eri_tile_2221", "source_sha256": bench.kernel_sources_sha256(),
           "hbm_bytes_per_launch": 123.0}
    (tmp_path / "eri_tile_2221_large620_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("eri_tile_2221", "large") == 123.0
    assert bench.measured_traffic("eri_tile_2221", "medium") is None
    rec["source_sha256"] = "0" * 64
    (tmp_path / "eri_tile_2221_large620_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("eri_tile_2221", "large") is None
    assert bench.measured_traffic("digest_c_0000", "large") is None
