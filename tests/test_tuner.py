"""The search's launch tuner (batch and dock keys, candidate plans, fastest-pick
selection, per-device cache, concurrent callers) on the host, under
AddressSanitizer and UBSan, with a scripted measurement in place of trial
launches."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tuner_selection_and_cache(tmp_path):
    exe = str(tmp_path / "tuner_check")
    env = {k: v for k, v in os.environ.items() if k != "LD_PRELOAD"}
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2303_09916_amd", "csrc"),
                    os.path.join(ROOT, "tests", "tuner_check.cpp"), "-o", exe], check=True, env=env)
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr
    assert "as specified" in r.stdout
