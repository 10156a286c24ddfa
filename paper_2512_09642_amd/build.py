"""Build libsstep.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Every translation unit is compiled in parallel into ``_build/`` and linked
into ``paper_2512_09642_amd/libsstep.so``.  ``gram_s.hip`` (the Gram, FGS and
batched launchers of one basis width) is compiled once per width
``-DSSTEP_S=1..32``, widest first, so the heavy instantiations spread over
the workers.  Device code is built with packed FP32 instructions disabled
(``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsstep.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]


PER_WIDTH = "gram_s.hip"
MAX_S = 32


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def units():
    """(source, extra flags, object name) of every compilation, the per-width
    instantiations first (widest first: they take longest)."""
    out = []
    for src in sources():
        if os.path.basename(src) == PER_WIDTH:
            out = [(src, [f"-DSSTEP_S={w}"], f"{PER_WIDTH}.s{w}.o") for w in range(MAX_S, 0, -1)] + out
        else:
            out.append((src, [], os.path.basename(src) + ".o"))
    return out


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return max(os.path.getmtime(h) for h in hs)


def _compile(unit, verbose: bool, incremental: bool = False) -> str:
    src, extra, name = unit
    obj = os.path.join(BUILD, name)
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) > max(os.path.getmtime(src), _headers_mtime()):
            return obj
    cmd = [HIPCC, *CFLAGS, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    """Compile and link the library.  ``incremental`` reuses objects newer
    than their source and every header (a full build compiles everything)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose, incremental), units()))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
