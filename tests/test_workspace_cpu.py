"""Host logic of the context workspace, compiled with g++ and run on the CPU (no GPU, no HIP):
a buffer that must read as zero is cleared whenever it is reallocated, even when the allocator
returns the released block's address again with stale contents; the device is quiesced before a
block is released; and atlases past the kernels' 32-bit texel addressing are refused."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_22625_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "cpp", "workspace_regrow.cpp")


def test_workspace_growth_and_atlas_limits(tmp_path):
    exe = str(tmp_path / "workspace_regrow")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-fsanitize=address,undefined", "-I", CSRC, SRC, "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "workspace checks passed" in r.stdout
