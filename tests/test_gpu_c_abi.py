"""The C ABI from C: tests/cpp/abi_example (built by __graft_entry__.build())
allocates device memory with the HIP runtime, calls lddmm_shoot_grad and
lddmm_solve through include/lddmm.h, and checks the gradient against the
FP64 oracle's C function."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "cpp", "abi_example")


def test_c_program_through_the_abi():
    if not os.path.exists(EXE):
        pytest.fail("tests/cpp/abi_example is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
