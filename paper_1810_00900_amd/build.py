"""Build the HIP library libtorgbs.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtorgbs.so")
SOURCES = ["csrc/tor_api.hip", "csrc/tor_kernels.hip", "csrc/tor_kernels_disp.hip", "csrc/tor_kernels_info.hip",
           "csrc/tor_kernels_qd.hip",
           "csrc/gbs_sampler.hip", "csrc/tor_async.hip", "csrc/tor_invert.hip", "csrc/tor_gather.hip",
           "csrc/tor_pserver.hip", "csrc/tor_fused.hip"]

# -ffp-contract=off: the double-double error-free transformations must not be
# fused into FMAs by the compiler (explicit fma() calls are kept).
# -packed-fp32-ops: no packed FP32 instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")


def build(verbose: bool = False, out: str = LIB) -> str:
    """Compile every source to an object in parallel (one hipcc per source),
    then link the shared library."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    with tempfile.TemporaryDirectory(prefix="torgbs_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[hipcc(), *FLAGS, *inc, "-c", os.path.join(HERE, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        _run([hipcc(), *FLAGS, *objs, "-o", out + ".tmp"], verbose)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
