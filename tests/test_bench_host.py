"""Host logic of bench.py (CPU only): the one-GPU contract and the lookup of
copy-calibrated traffic, which is reported only while the kernel sources match
the ones the counters were taken with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_measured_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    digest = bench.kernel_sources_digest("faber")
    f = tmp_path / "hbm_traffic.txt"
    f.write_text("# header\n"
                 f"faber layered2d_1001x501 f32 3.6e+07 {digest}\n"
                 f"krylov_arnoldi layered2d_1001x501 f32 8.5e+08 {'0' * 64}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("faber", "layered2d_1001x501", "f32") == 3.6e7
    # counters taken with other sources: not reported
    assert bench.measured_traffic("krylov_arnoldi", "layered2d_1001x501", "f32") is None
    # no line for this workload or dtype
    assert bench.measured_traffic("faber", "layered2d_1001x501", "f64") is None
    assert bench.measured_traffic("faber", "homog2d_101", "f32") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("faber", "layered2d_1001x501", "f32") is None


def test_kernel_sources_digest_depends_on_the_class_sources():
    a = bench.kernel_sources_digest("krylov_arnoldi")
    b = bench.kernel_sources_digest("faber")
    assert len(a) == 64 and len(b) == 64 and a != b
    assert a == bench.kernel_sources_digest("krylov_arnoldi")
