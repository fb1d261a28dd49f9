"""CPU checks of the host construction of the constant tables.

Compiles tests/native/consts_check.cpp (host code only, with the address and
undefined-behaviour sanitizers) against consts_host.h and runs it: the Cantor
basis continued into GF(2^128) = GF(2^64)[y] / (y^2 + y + v_63), the field
axioms and order of that extension, the m = 128 Encode matrix and its
inverse, and the split of the butterfly multipliers that the m = 128 kernels
apply through window tables.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "consts_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_constant_tables(tmp_path):
    exe = str(tmp_path / "consts_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("basis_recursion", "basis_rank", "field_axioms", "encode_matrix", "butterfly_split",
                 "v63_table"):
        assert f"ok {name}" in r.stdout
