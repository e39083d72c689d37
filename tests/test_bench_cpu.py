"""Host-side checks of bench.py that need no GPU: it refuses more than one
GPU before touching one, its roofline line follows the per-clause-counter
byte model, and the HBM traffic figure is used only while the kernel sources
still hash to the value recorded beside the counters."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_byte_model():
    # 2.56e11 attempts in 4 launches of 345 ms: 185.5 G attempts/s
    kt = {"attempts": 2.56e11, "ms": 4 * 345.0, "launches": 4}
    a = 0.25
    r = bench.ksat_roofline(kt, 495000, a, traffic=123.0)
    deg = 4 * 495000 / 50000  # k M / N
    assert r["mean_degree"] == pytest.approx(39.6)
    assert r["bytes_per_attempt"] == pytest.approx((deg + 1) * (1 + a))
    rate = 2.56e11 / 1.38
    assert r["kernel_attempts_per_s"] == pytest.approx(rate)
    assert r["achieved"] == pytest.approx(rate * (deg + 1) * (1 + a) / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["traffic"] == 123.0
    assert r["algorithmic_bytes_per_launch"] == pytest.approx((deg + 1) * (1 + a) * 2.56e11 / 4)
    assert r["kernel_ms_per_launch"] == pytest.approx(345.0)


def test_counter_bytes_follow_the_source_hash(tmp_path, monkeypatch):
    srcs = "include/nmc.h"
    h = hashlib.sha256(open(os.path.join(ROOT, srcs), "rb").read()).hexdigest()
    good = tmp_path / "good.md"
    good.write_text(f"counter_bytes_per_sweep: 1234\nkernel_sources: {srcs}\nkernel_sources_sha256: {h}\n")
    monkeypatch.setattr(bench, "KSAT_PROFILE", str(good))
    assert bench.counter_bytes_per_sweep() == 1234.0
    stale = tmp_path / "stale.md"
    stale.write_text(f"counter_bytes_per_sweep: 1234\nkernel_sources: {srcs}\nkernel_sources_sha256: {'0' * 64}\n")
    monkeypatch.setattr(bench, "KSAT_PROFILE", str(stale))
    assert bench.counter_bytes_per_sweep() is None
    monkeypatch.setattr(bench, "KSAT_PROFILE", str(tmp_path / "missing.md"))
    assert bench.counter_bytes_per_sweep() is None
