"""CPU checks of the product server's admission policy and arena allocator.

Compiles tests/native/policy_check.cpp (host code only, with the address and
undefined-behaviour sanitizers) against server_policy.h and runs it.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "policy_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_policy_and_arena(tmp_path):
    exe = str(tmp_path / "policy_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("arena_basics", "arena_random", "batches_small_in_order", "large_runs_alone_and_batch_skips_it",
                 "budget_and_starvation", "max_batch_respected", "batch_shrinks_to_fit", "simulated_stream",
                 "resident_runs_alone_at_its_length"):
        assert f"ok {name}" in r.stdout


PLAN_SRC = os.path.join(ROOT, "tests", "native", "plan_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_launch_sizing_rules(tmp_path):
    """plan.h on the CPU, with the sanitizers: the server's reservation for a
    single launch holds the workspace of the single-product path for every
    split of every product length up to 2^37 bits, every routing threshold's
    workspace holds its transform, and the fused path's buffers fit."""
    exe = str(tmp_path / "plan_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", exe, PLAN_SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("ilog2_is_ceiling", "transform_holds_the_product", "server_reservation_holds_the_workspace",
                 "workspace_holds_every_route", "fused_buffers_fit", "schedule_space"):
        assert f"ok {name}" in r.stdout
