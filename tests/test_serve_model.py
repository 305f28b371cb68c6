"""CPU model of the persistent serving kernel (no GPU): the round planner of
paper_1903_12522_amd/csrc/serve_plan.h drives scripted solves (period launches cover every
period exactly, first and last flags, buffer ping-pong, the CG phase order with FP64 refreshes
and the stop at max_iter after a refresh), and the kernel's bounded grid barrier is modelled
with threads (no round starts early; with a spin limit of one poll every thread leaves)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serving_plan_and_barrier_model(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "serve_model")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "cpu_models", "serve_model.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "ok plan" in r.stdout and "ok barrier" in r.stdout
