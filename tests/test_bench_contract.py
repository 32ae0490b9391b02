"""bench.py on the host: it refuses more than one GPU, and it reports the profiled HBM
traffic of a kernel only while the kernel sources hash to the ones the counters were taken
on (a stale figure is reported as null)."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def _sources_sha():
    import bench
    h = hashlib.sha256()
    for name in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1302_2132_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def test_traffic_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    import bench
    summary = tmp_path / "traffic.md"
    summary.write_text("# traffic\n\ntraffic_bytes_per_launch k_tile2<double,0>: 48587070\n"
                       f"kernel_sources_sha: {_sources_sha()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARIES", (str(tmp_path / "missing.md"), str(summary)))
    assert bench._profiled_traffic("k_tile2<double,0>") == 48587070.0
    assert bench._profiled_traffic("k_tile2<double,4>") is None          # not profiled
    summary.write_text("traffic_bytes_per_launch k_tile2<double,0>: 48587070\nkernel_sources_sha: 0123456789abcdef\n")
    assert bench._profiled_traffic("k_tile2<double,0>") is None          # sources changed since
