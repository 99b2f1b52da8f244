"""The serving scheduler's first-fit range allocator (device-pool carving) on the
host, under AddressSanitizer and UBSan: random allocation/release sequences
against a brute-force model (first fit, coalescing, accounting)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_range_alloc_matches_model(tmp_path):
    exe = str(tmp_path / "range_alloc_check")
    env = {k: v for k, v in os.environ.items() if k != "LD_PRELOAD"}
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_2303_09916_amd", "csrc"),
                    os.path.join(ROOT, "tests", "range_alloc_check.cpp"), "-o", exe], check=True, env=env)
    # the check carries its own (gcc) sanitizer runtime: no preloaded one
    env = {k: v for k, v in os.environ.items() if k != "LD_PRELOAD"}
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr
    assert "match the model" in r.stdout
