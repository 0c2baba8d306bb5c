"""Build the HIP library libsfo.so for gfx950 in-tree with hipcc.

Each translation unit is compiled to an object in parallel, then linked
into paper_1012_3911_amd/libsfo.so.  Packed FP32 instructions are disabled
for all device code (-packed-fp32-ops off)."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsfo.so")
SOURCES = ["sfo_kernels.hip", "sfo_row.hip", "sfo_col.hip", "sfo_dirac.hip", "sfo_batch.hip", "sfo_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="sfo_build_") as tmp:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            # hipcc's host pass does not know the packed-fp32 feature flag: harmless
            lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if p.returncode != 0:
                failed.append(src)
                sys.stderr.write("\n".join(lines) + "\n")
            elif verbose and lines:
                print("\n".join(lines))
        if failed:
            raise RuntimeError("hipcc failed for: " + ", ".join(failed))
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp_lib] + objs
        subprocess.check_call(cmd)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
