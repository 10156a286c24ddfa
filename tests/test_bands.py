"""The batched two-step basis's band tables and dispatch order (host code, no
GPU).  Builds tests/native/bands_check.cpp against the library's bands.h
with g++ (with AddressSanitizer and UndefinedBehaviorSanitizer when
available) and runs it on the batched workload's 64 systems and on smaller
batches.  The driver checks that each table covers every system's rows and
planes exactly once within one block's threads, that each dispatch order
runs every (band, right-hand side) block exactly once with a band's
right-hand sides together (and a whole system on one XCD when asked), and
that the per-XCD work stays within one unit of the mean."""
import os
import subprocess

import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "bands_check.cpp")
INC = os.path.join(ROOT, "paper_2512_09642_amd", "csrc")


@pytest.fixture(scope="module", params=[False, True], ids=["plain", "asan_ubsan"])
def exe(tmp_path_factory, request):
    out = str(tmp_path_factory.mktemp("bands") / "bands_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-I", INC, SRC, "-o", out]
    if request.param:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if request.param:
            pytest.skip(f"sanitizer build unavailable: {r.stderr[:200]}")
        raise AssertionError(r.stderr)
    return out


def run(exe, dims, nrhs, cus=256):
    text = f"{nrhs} {cus}\n" + "".join(f"{nx} {ny} {nz}\n" for nx, ny, nz in dims)
    r = subprocess.run([exe], input=text, capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and "FAIL" not in r.stdout, r.stdout[-3000:] + r.stderr[-3000:]
    words = r.stdout.split()
    return {words[i]: float(words[i + 1]) for i in range(0, len(words) - 1, 2)}


def test_batched_workload(exe):
    """64 systems of side 32..96, 8 right-hand sides: whole-system ranges,
    work per XCD within 1% of the mean."""
    dims = [pr.dims for pr in gen.config4(0)]
    out = run(exe, dims, 8)
    assert out["longest_range"] == max(d[2] for d in dims)
    assert out["balance_whole"] <= 1.01 and out["balance_short"] <= 1.01, out
    assert out["short"] > out["bands"]


@pytest.mark.parametrize("dims,nrhs", [
    ([(12, 10, 8)], 1),                              # one band, one range
    ([(40, 37, 35), (33, 20, 18), (12, 12, 12)], 2),  # small batch: 16-plane ranges
    ([(341, 9, 40)], 1),                             # rows of 341 points: one row per band
    ([(7, 300, 90), (100, 9, 17), (31, 33, 129)], 3),  # tall, flat, long
])
def test_small_batches(exe, dims, nrhs):
    out = run(exe, dims, nrhs)
    assert out["longest_range"] <= 16


def test_a_row_too_wide_gives_no_table(exe):
    """A row of 342 points leaves no room for a band with its two ring rows."""
    text = "1 256\n342 3 3\n"
    r = subprocess.run([exe], input=text, capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 1 and "tables built" in r.stdout
