"""Host-code sanitizer runs (CPU only): the oracle built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven through its
entry points, argument errors included; the C ABI's host code (api.cpp)
rebuilt with the same sanitizers on the host side, linked with the built
kernel objects, and driven through every argument check that rejects a call
before it reaches the GPU.  (The autotuner cache's host code runs under the
same sanitizers in tests/test_tune_cache.py.)"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan):
        pytest.skip("libasan not found")
    lib = str(tmp_path / "liboracle_san.so")
    r = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra",
                        "-Wno-unknown-pragmas", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer", "-o", lib, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"sanitizer build unavailable: {r.stderr[:200]}")
    env = dict(os.environ, SSTEP_ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "native", "oracle_exercise.py")], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "oracle exercised" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


def test_abi_host_code_under_asan_ubsan(tmp_path):
    """api.cpp with -fsanitize=address,undefined on the host side only (the
    device code is unchanged), linked with the kernel objects of the last
    build."""
    build = os.path.join(ROOT, "_build")
    objs = [o for o in glob.glob(os.path.join(build, "*.o")) if not o.endswith("api.cpp.o")]
    rt = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not objs or not rt:
        pytest.skip("no kernel objects from a previous build, or no clang sanitizer runtime")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer"]
    obj = str(tmp_path / "api_san.o")
    lib = str(tmp_path / "libsstep_san.so")
    r = subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fPIC", *san, "-I",
                        os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2512_09642_amd", "csrc"),
                        "-x", "hip", "-c", os.path.join(ROOT, "paper_2512_09642_amd", "csrc", "api.cpp"), "-o", obj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-o", lib, obj, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt[0], ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "native", "abi_exercise.py"), lib], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "abi exercised" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
