"""Host-side logic of bench.py: kernel-name parsing, the counter summary and
its calibration, the source-hash guard on stored traffic, the one-GPU rule."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("full,short", [
    ("bec::(anonymous namespace)::dir_write_kernel(bec::PwParams, bec::DirArgs)", "dir_write_kernel"),
    ("void bec::(anonymous namespace)::fft_pass_kernel<128, 16, 8, 4, 4, 256, true, 0>(bec::FftPassArgs)",
     "fft_pass_kernel<128, 16, 8, 4, 4, 256, true, 0>"),
    ("bec::(anonymous namespace)::reduce_final_kernel(bec::(anonymous namespace)::RedSeg, "
     "bec::(anonymous namespace)::RedSeg, bec::(anonymous namespace)::RedSeg)", "reduce_final_kernel"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_kernel_short_name(full, short):
    assert bench.kernel_short_name(full) == short


def _csv(path, rows):
    cols = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w") as f:
        f.write(",".join(f'"{c}"' for c in cols) + "\n")
        for r in rows:
            f.write(",".join(f'"{x}"' for x in r) + "\n")


def test_pmc_summary_scales_by_the_copy_calibration(tmp_path):
    k = "bec::(anonymous namespace)::dir_write_kernel(bec::PwParams, bec::DirArgs)"
    _csv(tmp_path / "f.csv", [(k, "FETCH_SIZE", 100.0), (k, "FETCH_SIZE", 300.0)])
    _csv(tmp_path / "w.csv", [(k, "WRITE_SIZE", 50.0), (k, "WRITE_SIZE", 50.0)])
    # a 1 MiB copy that reads 512 KiB and writes 1024 KiB by the counters
    _csv(tmp_path / "cf.csv", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0)])
    _csv(tmp_path / "cw.csv", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0)])
    out = bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                            str(tmp_path / "cw.csv"), 1, out_path=str(tmp_path / "t.json"))
    assert out["fetch_factor"] == pytest.approx(2.0) and out["write_factor"] == pytest.approx(1.0)
    d = out["kernels"]["dir_write_kernel"]
    assert d["fetch_bytes"] == pytest.approx(200.0 * 1024 * 2.0)
    assert d["write_bytes"] == pytest.approx(50.0 * 1024)
    assert d["dispatches"] == 2
    assert json.load(open(tmp_path / "t.json"))["source_hash"] == bench.kernel_source_hash()


def test_stored_traffic_is_dropped_when_kernel_sources_change(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    good = {"source_hash": bench.kernel_source_hash(),
            "kernels": {bench.LABEL_KERNEL["dir_write"]: {"bytes_per_launch": 7.0}}}
    path.write_text(json.dumps(good))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.traffic_from_profiles("dir_write") == 7.0
    assert bench.traffic_from_profiles("fft_x_kspace") is None
    path.write_text(json.dumps(dict(good, source_hash="0" * 16)))
    assert bench.traffic_from_profiles("dir_write") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
