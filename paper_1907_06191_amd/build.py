"""Build libdgd.so in-tree with hipcc for gfx950.

    python -m paper_1907_06191_amd.build

compiles every source under csrc/ into paper_1907_06191_amd/libdgd.so.
All device code is built with packed-FP32 instruction selection disabled.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgd.so")
ARCH = os.environ.get("DGD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = True, jobs: int = 8) -> str:
    """Compile each source to an object in _build/ (in parallel), then link."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    procs = []
    t0 = time.time()
    for src in sources():
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"]
        cmd = [hipcc(), *FLAGS, *lang, "-c", src, "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    while procs:
        _wait(procs.pop(0), verbose)
    tmp = LIB + ".tmp"
    # roctx: named ranges around the solve's phases for rocprofv3 traces
    cmd = [hipcc(), *FLAGS, "-shared", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


def _wait(item, verbose):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{text}")
    if verbose and text.strip():
        # keep warnings visible, minus hipcc's note about the packed-fp32 feature on the host pass
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    build()
