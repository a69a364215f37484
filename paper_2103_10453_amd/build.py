"""Build libplse.so (HIP kernels for gfx950 + host orchestrator) in-tree.

Every source is compiled with hipcc for gfx950 only; packed-FP32 instruction
selection is disabled.  Objects go to _build/ next to the sources.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libplse.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["k_plits.hip", "k_plits_lean.hip", "k_init.hip", "k_evo.hip", "k_measure.hip",
           "host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = False
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        noise = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"hipcc failed on {src}:\n" + "\n".join(noise) + "\n")
        elif verbose and noise:
            sys.stderr.write("\n".join(noise) + "\n")
    if failed:
        raise RuntimeError("libplse build failed")
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    build_example()
    return OUT


EXAMPLE_SRC = os.path.join(HERE, "examples", "plse_solve.c")
EXAMPLE = os.path.join(HERE, "examples", "plse_solve")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_example() -> str:
    """The plain-C command-line driver of the C ABI (gcc, no HIP device code)."""
    include = os.path.join(os.path.dirname(HERE), "include")
    tmp = EXAMPLE + ".tmp"
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-I", include,
                           "-I", os.path.join(ROCM, "include"), EXAMPLE_SRC, "-o", tmp,
                           "-L", HERE, "-lplse", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                           "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
