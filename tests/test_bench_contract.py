"""bench.py's contract on the host: the multi-GPU refusal and the rule that
HBM traffic is reported only from counters taken on the same kernel
sources and launch size."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_from_matching_counters(tmp_path):
    import bench

    srcs = bench.GRAD_SOURCES
    text = "".join(open(os.path.join(ROOT, "paper_2508_15743_amd", "csrc", f)).read() for f in srcs)
    sha = hashlib.sha256(text.encode()).hexdigest()[:16]
    prof = tmp_path / "p.txt"
    prof.write_text(f"note\ntraffic_launch_batch 4096\ntraffic_bytes_per_launch 1.5e+12\nsource_sha256_16 {sha}  (x)\n")
    assert bench.measured_traffic(4096, str(prof), srcs, "traffic_launch_batch") == 1.5e12
    assert bench.measured_traffic(2048, str(prof), srcs, "traffic_launch_batch") is None
    prof.write_text(f"traffic_launch_batch 4096\ntraffic_bytes_per_launch 1.5e+12\nsource_sha256_16 {'0' * 16}\n")
    assert bench.measured_traffic(4096, str(prof), srcs, "traffic_launch_batch") is None
    assert bench.measured_traffic(4096, str(tmp_path / "missing.txt"), srcs, "traffic_launch_batch") is None
