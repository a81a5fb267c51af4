"""Host unit test of the serving scheduler (admission by device-memory footprint,
continuous batching of whole coupling splits): builds tests/cpp/test_sched.cpp
with g++ and runs it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_scheduler_policy(tmp_path):
    exe = str(tmp_path / "test_sched")
    src = os.path.join(HERE, "cpp", "test_sched.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
