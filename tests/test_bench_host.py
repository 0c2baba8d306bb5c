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
    fetch, write = b.MEASURED_TRAFFIC["c64"]["column/0"]
    # FETCH_SIZE reads half of what a plain copy moves in, WRITE_SIZE all of what it writes
    assert b.measured_traffic("c64", "column", 0) == (2.0 * fetch + 1.0 * write) * 1024
    assert b.measured_traffic("c64", "column", 99) is None
    assert b.measured_traffic("c256", "column", 0) is None
    # every measured shape moves its algorithmic bytes to within -10 % / +40 % (2048^2:
    # column pass reads and writes the state, row pass also reads the potential; complex64
    # 8 B per point and FP32 potential, complex128 16 B and FP64; narrow complex128
    # column shapes write up to 41 % more than the state, i.e. 25 % more in total; the
    # pipelined shapes that spill registers (never chosen by the autotuner) up to 31 %)
    for dtype, sb, vb in (("c64", 8, 4), ("c128", 16, 8)):
        npts = 2048 * 2048
        alg = {"column": 2 * sb * npts, "row": (2 * sb + vb) * npts}
        for key in b.MEASURED_TRAFFIC[dtype]:
            kind, var = key.split("/")
            t = b.measured_traffic(dtype, kind, int(var))
            assert 0.9 * alg[kind] < t < 1.4 * alg[kind], (dtype, key)


def test_sources_fingerprint_covers_the_pass_sources():
    b = _bench()
    fp = b.sources_fingerprint()
    assert len(fp) == 64 and fp == b.sources_fingerprint()
    for f in b.TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1012_3911_amd", "csrc", f)), f
