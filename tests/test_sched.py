"""CPU test of the ladder server's scheduler (host C++), built with g++ and the sanitizers."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_state_machine(tmp_path):
    exe = str(tmp_path / "test_sched")
    subprocess.check_call([
        "g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
        "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2301_12191_amd", "csrc"),
        os.path.join(ROOT, "tests", "cpp", "test_sched.cpp"),
        os.path.join(ROOT, "paper_2301_12191_amd", "csrc", "mr_sched.cpp"), "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr + res.stdout
    assert "all checks passed" in res.stdout
