"""The launch planner on the CPU under the address and undefined-behaviour
sanitizers: the planning header the library compiles (argument and aliasing
checks, tile geometry, descriptors, batch work lists, workspace sizes) is
built into a harness with g++ and run on randomized jobs -- offsets at and
past the end of the base allocation and next to 2^64, lengths 0 .. 2^36-32
and just past it, unregistered key slots, overlapping buffers, batches of
4096+ messages under every launch shape -- against a plain restatement of
the validation rules and the invariants the kernels rely on (tiles cover
each message exactly once, every partial lies inside the workspace, the
serving loop's admission bound covers a batch's device bytes)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_plan_invariants_under_sanitizers(tmp_path):
    exe = tmp_path / "plan"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "paper_2602_23067_amd", "csrc"),
                    os.path.join(ROOT, "tests", "plan_harness.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=500)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "OK" in out.stdout
