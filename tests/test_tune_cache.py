"""The autotuner's on-disk cache (host code, no GPU): a corrupt or foreign
cache file can only cost a re-tune.  Builds tests/native/tune_cache_check.cpp
against the library's cache header with g++ (with AddressSanitizer and
UndefinedBehaviorSanitizer when available) and runs it."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "tune_cache_check.cpp")
INC = os.path.join(ROOT, "paper_2512_09642_amd", "csrc")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("tune_check_san" if sanitize else "tune_check"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-I", INC, SRC, "-o", exe]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return exe if r.returncode == 0 else None, r.stderr


@pytest.mark.parametrize("sanitize", [False, True])
def test_tune_cache_validation(tmp_path, sanitize):
    exe, err = _build(tmp_path, sanitize)
    if exe is None:
        if sanitize:
            pytest.skip(f"sanitizer build unavailable: {err[:200]}")
        raise AssertionError(err)
    r = subprocess.run([exe, str(tmp_path / "tune.json")], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
