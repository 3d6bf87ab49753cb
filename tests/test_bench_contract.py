"""Host-side rules of bench.py that need no GPU: a request for more than one
GPU exits with a message, and the measured HBM traffic is reported only for
the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_needs_matching_kernel_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pmc_traffic.json").write_text(json.dumps({
        "k_trace_batch": {"source_hash": "aaaa", "bytes_per_launch": 123},
        "k_recon_batch": {"source_hash": "bbbb", "bytes_per_launch": 456},
    }))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "aaaa")
    assert bench.load_traffic("k_trace_batch") == 123
    assert bench.load_traffic("k_recon_batch") is None     # measured on other sources
    assert bench.load_traffic("k_other") is None
    (prof / "pmc_traffic.json").write_text("not json")
    assert bench.load_traffic("k_trace_batch") is None


def test_kernel_source_hash_tracks_both_kernels():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.kernel_source_hash()


def test_roofline_peaks_are_the_published_ones():
    assert bench.HBM_PEAK_GBS == 8000.0
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one non-packed FP32 op per lane
    assert abs(bench.VALU_PEAK_GOPS - 39321.6) < 1e-6
