"""The kernels' exact modulo (Lemire's direct remainder, used for Eq. 1's
'mod V') checked on the CPU against the C++ '%' operator: exhaustively over
all 2^32 numerators for several divisors, and on sampled and edge numerators
for 64-bit keys.  Compiles tests/native/fastmod_check.hip with hipcc (host
code only runs)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fastmod_exhaustive_against_native_modulo(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fastmod_check")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-pthread",
                           "-I", os.path.join(ROOT, "paper_1907_02900_amd", "csrc"),
                           os.path.join(ROOT, "tests", "native", "fastmod_check.hip"), "-o", exe])
    r = subprocess.run([exe], stdout=subprocess.PIPE, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout
