"""Compile libswe.so for gfx950 in-tree (hipcc; no JIT cache, no torch extension machinery)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libswe.so")

SOURCES = ["swe_mesh.cpp", "swe_api.cpp", "swe_batch.cpp", "swe_tune.cpp", "swe_launch.cpp",
           "swe_kernels.hip", "swe_kernels_fast.hip", "swe_adjoint.hip", "swe_static.hip"]
HEADERS = ["swe_internal.h", "swe_device_math.h"]

# Contraction off: every product and sum rounds on its own, in the order the sources write
# it.  Packed FP32 instructions are disabled for every kernel.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode}): {' '.join(cmd[-3:])}")
    noise = [ln for ln in (r.stdout + r.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "target-feature" not in ln]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")


def build(out: str = LIB, verbose: bool = False, extra=(), jobs: int = 8) -> str:
    """Compile every source to an object (in parallel, in a temporary folder), then link."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    cc = hipcc()
    flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="swe_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[cc, *flags, *extra, "-I", INCLUDE, "-I", CSRC, "-c", "-o", o,
                 os.path.join(CSRC, s)] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(cmds)))) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp", *objs], verbose)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
