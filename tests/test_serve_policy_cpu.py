"""Serving-loop admission and batching policy on the CPU: the policy header
the library compiles is built into a small harness with g++ and exercised on
randomized arrivals and completions (budget never exceeded, strict arrival
order of admission and batching, batch caps, oversize and queue-full
rejection, full drain)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_policy_invariants(tmp_path):
    exe = tmp_path / "policy"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "paper_2602_23067_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_policy_harness.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "OK" in out.stdout
