"""The batch's host layout (size classes, concatenated support lists, kept-column maps;
paper_2509_13592_amd/csrc/batch_layout.h, the code bccb_batch_create runs) built on its
own with the address and undefined-behaviour sanitizers and driven with ragged batches of
up to 4096 scenes: every array is checked against the scenes it came from, and
inconsistent tables are refused instead of read out of bounds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "batch_layout_check.cpp")
INC = os.path.join(ROOT, "paper_2509_13592_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_batch_layout_under_sanitizers(tmp_path):
    exe = str(tmp_path / "batch_layout_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{INC}", SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
