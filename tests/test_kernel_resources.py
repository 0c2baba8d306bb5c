"""The tile shapes the benchmark times compile without a stack frame.

The autotuner leaves out any shape whose kernel has private (scratch)
memory, since it reads that as a register spill. A transform that calls a
helper at run time instead of folding it (for instance a recursive
constexpr function used as an ordinary call argument) gets a small stack
frame and no spill. The shape then silently drops out of tuning. This
test compiles the timed shapes of the 2048^2 complex128 and complex64
paths, the 4096^2 path and the reverse sweep for gfx950. It checks that each
has a zero private segment and makes no call. CPU only: hipcc
cross-compiles, and nothing runs on a GPU."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# k_xpass<R, N, RAD, THREADS, WPE, NS, PAD, LATE, PRE>,
# k_colpass<R, N, RAD, C, WPE, NS, CHI, VGRAD, PRE>, k_colpipe<R, N, RAD, C, WPE, ORDER>
KERNELS = [
    "k_xpass<double, 2048, 8, 256, 1, 1, false, true, true>",      # 2048^2 c128 rows
    "k_colpipe<double, 2048, 16, 4, 2, 2>",                        # 2048^2 c128 columns
    "k_xpass<double, 2048, 8, 256, 1, 2, false, true, true>",      # reverse sweep rows
    "k_colpass<double, 2048, 16, 2, 1, 2, false, false, true>",    # reverse sweep columns
    "k_xpass<double, 4096, 16, 256, 1, 1, true, false, true>",     # 4096^2 c128 rows
    "k_colpass<double, 4096, 16, 2, 1, 1, false, false, true>",    # 4096^2 c128 columns
    "k_xpass<float, 2048, 16, 128, 4, 1, true, true, false>",      # 2048^2 c64 rows
    "k_colpass<float, 2048, 16, 8, 1, 1, false, false, false>",    # 2048^2 c64 columns
]


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_timed_shapes_have_no_stack_frame(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text('#include "pass_kernels.h"\nvoid *kernel_addresses[] = {\n' +
                   "".join("    (void *)&sfo::%s,\n" % k for k in KERNELS) + "};\n")
    asm = tmp_path / "probe.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1012_3911_amd", "csrc"), "--cuda-device-only", "-S", str(src),
           "-o", str(asm)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    text = asm.read_text()
    # per-kernel metadata: name, private segment size
    found = re.findall(r"\.name:\s+(_Z\S+)\n(?:.*\n)*?\s+\.private_segment_fixed_size:\s+(\d+)", text)
    kernels = {n: int(p) for n, p in found if not n.endswith(".kd")}
    assert len(kernels) == len(KERNELS), sorted(kernels)
    for name, priv in kernels.items():
        assert priv == 0, (name, priv)
    assert "s_swappc" not in text
