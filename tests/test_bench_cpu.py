"""bench.py's host-side contract, on the CPU: the one-GPU guard, the roofline
arithmetic and the rule that a counter-measured traffic figure is reported only
for the push sources and launch shape it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_roofline_of():
    import bench
    tim = {"push_ms": 2.0, "push_launches": 10}
    roof = bench.roofline_of(1.6e9, tim, "k_push_f64")
    assert roof["avg_launch_us"] == 200.0
    assert abs(roof["achieved"] - 8000.0) < 1e-9 and abs(roof["frac"] - 1.0) < 1e-12
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    json.dumps(roof)


def test_traffic_only_for_matching_sources_and_shape(tmp_path, monkeypatch):
    import bench
    f = tmp_path / "traffic.txt"
    good = bench.push_source_hash()
    f.write_text(f"kernel: k_push_f64<128, 2, 1>\npush_shape: 128:2:nt\nsource_sha256: {good}\n"
                 "traffic_bytes_per_launch: 1234\n\n  notes: indented lines are prose\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic((128, 2, True)) == 1234.0
    assert bench.measured_traffic((256, 2, True)) is None          # another launch shape
    assert bench.measured_traffic((128, 2, False)) is None
    f.write_text(f.read_text().replace(good, "0" * 64))
    assert bench.measured_traffic((128, 2, True)) is None          # other push sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic((128, 2, True)) is None


def test_traffic_files_are_keyed_by_their_own_sources(tmp_path):
    """The FP32-bulk and batched push summaries are keyed by those kernels' sources."""
    import bench
    f = tmp_path / "t32.txt"
    f.write_text(f"push_shape: 128:4:nt\nsource_sha256: {bench.push_source_hash(bench.PUSH32_SOURCES)}\n"
                 "traffic_bytes_per_launch: 99\n")
    assert bench.measured_traffic((128, 4, True), str(f), bench.PUSH32_SOURCES) == 99.0
    assert bench.measured_traffic((128, 4, True), str(f), bench.BATCH_SOURCES) is None
    assert bench.push_source_hash(bench.PUSH32_SOURCES) != bench.push_source_hash(bench.PUSH_SOURCES)
