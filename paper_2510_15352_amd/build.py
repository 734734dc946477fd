"""Build the HIP library libgsmi.so for gfx950 in-tree with hipcc.

Every source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops) and linked into one
shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsmi.so")
SOURCES = ["k_project.hip", "k_sort.hip", "k_raster.hip", "k_backward.hip", "k_upsample.hip",
           "k_probe.hip", "runtime.hip"]
ARCH = "gfx950"


def hip_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
            "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]


def build(jobs: int = 4, verbose: bool = False) -> str:
    """Compile every source (always) and link libgsmi.so; returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    procs = []
    objs = []
    for s in srcs:
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, *hip_flags(), "-x", "hip", "-c", os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[[i for i, (_, p) in enumerate(procs) if p.poll() is None][0]][1].wait()
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((s, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for s, text in failed:
            sys.stderr.write(f"--- {s}\n{text}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(hipcc)), "lib")
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{rocm_lib}", f"-Wl,-rpath,{rocm_lib}", "-lrocprofiler-sdk-roctx"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
