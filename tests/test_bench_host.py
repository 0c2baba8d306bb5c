"""Host-side logic of bench.py (no GPU): the one-GPU rule and the traffic
arithmetic behind the roofline's `traffic` figure."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_copy_calibrated_counter_bytes():
    b = _bench()
    fetch, write = b.MEASURED_TRAFFIC["column/0"]
    # FETCH_SIZE reads half of what a plain copy moves in, WRITE_SIZE all of what it writes
    assert b.measured_traffic("column", 0) == (2.0 * fetch + 1.0 * write) * 1024
    assert b.measured_traffic("column", 99) is None
    # every measured shape is within 10 % of its algorithmic bytes (2048^2 complex64:
    # column pass 2 x 32 MiB, row pass 2 x 32 MiB + 16 MiB of FP32 potential)
    alg = {"column": 2 * 32 << 20, "row": (2 * 32 + 16) << 20}
    for key in b.MEASURED_TRAFFIC:
        if key == "sources_sha256":
            continue
        kind, var = key.split("/")
        t = b.measured_traffic(kind, int(var))
        assert 0.9 * alg[kind] < t < 1.1 * alg[kind], key


def test_sources_fingerprint_covers_the_pass_sources():
    b = _bench()
    fp = b.sources_fingerprint()
    assert len(fp) == 64 and fp == b.sources_fingerprint()
    for f in b.TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1012_3911_amd", "csrc", f)), f
