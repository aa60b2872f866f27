"""Serving policy on the CPU: the scheduling core compiled with g++ against a
fake executor (admission, continuous batching, memory budget, delivery)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_core_policy(tmp_path):
    exe = str(tmp_path / "serve_core_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-pthread", "-Wall",
                           os.path.join(ROOT, "tests", "cpp", "serve_core_test.cpp"),
                           os.path.join(ROOT, "paper_2012_07990_amd", "csrc", "serve_core.cpp"),
                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout


def test_serve_core_under_sanitizers(tmp_path):
    exe = str(tmp_path / "serve_core_tsan")
    try:
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=thread",
                               os.path.join(ROOT, "tests", "cpp", "serve_core_test.cpp"),
                               os.path.join(ROOT, "paper_2012_07990_amd", "csrc", "serve_core.cpp"),
                               "-o", exe], stderr=subprocess.DEVNULL)
    except subprocess.CalledProcessError:
        pytest.skip("thread sanitizer unavailable")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
