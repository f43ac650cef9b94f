"""Build libcpf.so (HIP for gfx950) in-tree with hipcc.

The kernel sources are compiled once per chain length the library serves
(CPF_NJ = 7 and 8 joints, each into its own namespace); the host sources
once.  Every HIP source is compiled with packed FP32 instructions disabled;
the host pass prints a harmless warning that it does not know that target
feature.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcpf.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

KERNEL_SOURCES = ["fk.hip", "dp.hip", "lm.hip"]
HOST_SOURCES = ["capi.cpp", "serve.cpp"]
CHAIN_LENGTHS = (7, 8)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", CSRC, "-I", INCLUDE,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-Wno-unused-function"]


def _compile(src: str, build_dir: str = BUILD, defines=(), nj=None) -> str:
    tag = "" if nj is None else ".nj%d" % nj
    obj = os.path.join(build_dir, os.path.basename(src) + tag + ".o")
    if nj is not None:
        defines = tuple(defines) + ("CPF_NJ=%d" % nj,)
    cmd = ([HIPCC] + COMMON + [f"-D{d}" for d in defines] +
           ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    noise = [ln for ln in (r.stdout + r.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source and link `out`.  `defines` selects diagnostic
    variants (e.g. CPF_PHASE_CYCLES); those are built into their own folder."""
    build_dir = BUILD if not defines else os.path.join(BUILD, "_".join(defines))
    os.makedirs(build_dir, exist_ok=True)
    jobs = [(s, nj) for s in KERNEL_SOURCES for nj in CHAIN_LENGTHS] + [(s, None) for s in HOST_SOURCES]
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda j: _compile(j[0], build_dir, defines, j[1]), jobs))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=LIB)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    a = ap.parse_args()
    build(verbose=True, out=a.out, defines=tuple(a.defines))
