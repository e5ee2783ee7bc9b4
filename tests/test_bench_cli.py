"""bench.py on the CPU: more than one GPU is refused with a message (the path is
single-GPU), before anything touches a device, for every workload; the counter
summaries behind a line's `traffic` count only for the source they were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("workload", ["video", "batch", "fw", "prox"])
def test_more_than_one_gpu_is_refused(workload):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--workload", workload],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_summary_counts_only_for_the_source_it_was_taken_on(tmp_path):
    """The bench line's `traffic` comes from a committed counter summary only while
    the kernel's source hashes to the value recorded with it; any edit makes it null."""
    bench = _bench_module()
    src = tmp_path / "kernel.hip"
    src.write_text("__global__ void k() {}\n")
    summ = tmp_path / "traffic.md"
    summ.write_text("notes\ntraffic_bytes_per_launch: 123456\nsources_sha256: "
                    f"{bench.source_hash([str(src)])}\n")
    assert bench.measured_traffic(str(summ), [str(src)]) == 123456.0
    src.write_text("__global__ void k() { }\n")
    assert bench.measured_traffic(str(summ), [str(src)]) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), [str(src)]) is None


@pytest.mark.parametrize("which", ["sweep", "fw"])
def test_committed_traffic_summaries_parse(which):
    """Each committed summary holds one byte count, at least the kernel's algorithmic
    bytes (76,800 x 200 FP32 read once), and a SHA-256 of its sources."""
    bench = _bench_module()
    path = bench.TRAFFIC_FILE if which == "sweep" else bench.FW_TRAFFIC_FILE
    lines = dict(l.split(":", 1) for l in open(path).read().splitlines()
                 if l.startswith(("traffic_bytes_per_launch:", "sources_sha256:", "sweep_sources_sha256:")))
    assert float(lines["traffic_bytes_per_launch"]) >= 4 * 76800 * 200
    digest = (lines.get("sources_sha256") or lines["sweep_sources_sha256"]).strip()
    assert len(digest) == 64 and int(digest, 16) >= 0
