"""Builds libmlsdc_sh.so (HIP for gfx950 + quad-precision host setup) in-tree.

    python -m paper_1805_07923_amd.build

Every call recompiles.  HIP sources are compiled with packed-FP32 ops
disabled; the host set-up file is compiled by the host C++ compiler and
linked against libquadmath.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmlsdc_sh.so")
HIP_SOURCES = ["legendre.hip", "legendre_mixed.hip", "fourier.hip", "spectral.hip", "adjoint.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [["g++", "-O2", "-fPIC", "-std=gnu++17", "-c", os.path.join(SRC, "setup_host.cpp"),
             "-o", os.path.join(BUILD, "setup_host.o")]]
    objs = [os.path.join(BUILD, "setup_host.o")]
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s.replace(".hip", ".o"))
        jobs.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(SRC, s), "-o", o])
        objs.append(o)
    workers = min(len(jobs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(workers) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lquadmath"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
