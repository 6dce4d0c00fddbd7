"""The library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer: every source is compiled with the sanitizers on
its host side only (device code unchanged), linked into the host-check driver
tests/host_check/abi_host_check.cpp (quad-precision set-up routines and the
ABI's argument validation, no GPU needed) and run; any sanitizer report
aborts the run.  Takes about half a minute (the HIP sources are compiled for
gfx950 as well)."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1805_07923_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
HIP_SOURCES = ["legendre", "legendre_mixed", "fourier", "spectral", "adjoint", "api"]
# sanitizers on the host compilation only: each -fsanitize= follows -Xarch_host
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
CPP_SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]


def _run(cmd, cwd):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_host_code_under_asan_ubsan():
    d = tempfile.mkdtemp(prefix="shx_san_")
    try:
        gcc_inc = subprocess.run(["gcc", "-print-file-name=include"], capture_output=True, text=True).stdout.strip()
        jobs = [[HIPCC, "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                 "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"] + HOST_SAN +
                ["-c", os.path.join(SRC, f + ".hip"), "-o", f + ".o"] for f in HIP_SOURCES]
        jobs.append([CLANG, "-O1", "-g", "-fPIC", "-std=gnu++17"] + CPP_SAN +
                    ["-idirafter", gcc_inc, "-c", os.path.join(SRC, "setup_host.cpp"), "-o", "setup_host.o"])
        jobs.append([CLANG, "-O1", "-g", "-std=c++17"] + CPP_SAN +
                    ["-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__", "-c",
                     os.path.join(ROOT, "tests", "host_check", "abi_host_check.cpp"), "-o", "drv.o"])
        with cf.ThreadPoolExecutor(min(8, len(jobs))) as ex:
            list(ex.map(lambda c: _run(c, d), jobs))
        objs = ["drv.o"] + [f + ".o" for f in HIP_SOURCES] + ["setup_host.o"]
        _run([CLANG] + CPP_SAN + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-lquadmath", "-Wl,-rpath,/opt/rocm/lib",
                                         "-o", "abi_host_check"], d)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([os.path.join(d, "abi_host_check")], cwd=d, env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
        assert "host checks passed" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    finally:
        shutil.rmtree(d, ignore_errors=True)
