"""Host unit test of the split-BF16 MFMA coupling plan (tile GEMMs evaluated in
FP64 from the plan reproduce the directly summed T[t][B]): builds
tests/cpp/test_mfma_plan.cpp with g++ and runs it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2105_08722_amd", "csrc")


def test_mfma_plan_reproduces_direct_sum(tmp_path):
    exe = str(tmp_path / "test_mfma_plan")
    srcs = [os.path.join(HERE, "cpp", "test_mfma_plan.cpp"), os.path.join(CSRC, "mfma_plan.cpp"),
            os.path.join(CSRC, "tables.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-fsanitize=address,undefined"] + srcs +
                   ["-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout


def test_gemm_plan_reproduces_direct_sum(tmp_path):
    """The macro-tiled GEMM plan (rows from the first factors, columns w times the
    product of the rest) against the direct sum, N = 3..6, both parities, both
    splits of the 6PCF."""
    exe = str(tmp_path / "test_gemm_plan")
    srcs = [os.path.join(HERE, "cpp", "test_gemm_plan.cpp"), os.path.join(CSRC, "mfma_plan.cpp"),
            os.path.join(CSRC, "tables.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-Werror", "-fsanitize=address,undefined"] + srcs +
                   ["-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
