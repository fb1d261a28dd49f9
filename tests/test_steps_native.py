"""CPU checks of the word-level BasisCvt steps the GPU kernels apply.

Compiles tests/native/steps_check.cpp (host code only, with the address and
undefined-behaviour sanitizers) against k_steps.h and runs it: one Taylor
step out of place, two steps composed through the lazily read intermediate
array of the step-pair kernel, and the in-register step of segments of at
most 64 bits, each against the step written bit by bit from Alg. 1.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "steps_check.cpp")
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="no host C++ compiler or HIP headers")
def test_word_level_steps(tmp_path):
    exe = str(tmp_path / "steps_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("wide_step", "step_pair", "in_word_step"):
        assert f"ok {name}" in r.stdout
