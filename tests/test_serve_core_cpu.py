"""CPU checks of the serving policy code (serve_core.h): built with g++ here
and with AddressSanitizer/UBSan, run without a GPU."""

from __future__ import annotations

import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_1708_04329_amd", "csrc")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]])
def test_serve_core(flags):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "t")
        subprocess.check_call(["g++", "-std=c++17", *flags, "-I", INC, SRC, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert out.returncode == 0, out.stderr
        assert out.stdout.strip() == "OK"
