"""The library's host core (validation, arc compilation, the level
schedule, serving) built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host side only (every report fatal), running the CPU tests of the C
ABI against it: the validators on valid and malformed netlists, arcs and
stimuli, the exports, and a context created where there is no GPU.  The
kernels are linked from the regular build (compiled here when it is
absent).  CPU only; this file builds host code with sanitizers and is not
sent to GPU runs.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_06117_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SOURCES = ("host.cpp", "schedule.cpp", "serve.cpp")


def clang_asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_host_core_under_sanitizers(tmp_path):
    rt = clang_asan_runtime()
    if not rt or not os.path.exists(HIPCC):
        pytest.skip("no clang sanitizer runtime or hipcc")
    from paper_2203_06117_amd import build as B
    host_flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
                  "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    sanitize = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src in HOST_SOURCES:
        obj = str(tmp_path / (src + ".o"))
        r = subprocess.run([HIPCC, "--cuda-host-only", "-x", "hip"] + host_flags + sanitize +
                           ["-c", os.path.join(CSRC, src), "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        objs.append(obj)
    kobj = os.path.join(ROOT, "paper_2203_06117_amd", "_build", "kernels.hip.o")
    if not os.path.exists(kobj):
        kobj = str(tmp_path / "kernels.hip.o")
        r = subprocess.run([HIPCC] + B.FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", kobj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    lib = str(tmp_path / "libgatesim_san.so")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + sanitize + ["-o", lib] + objs + [kobj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    env = dict(os.environ, GATESIM_LIBRARY=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_library_host.py"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
