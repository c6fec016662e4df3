"""The C ABI from a plain host program (tests/capi_c_check.cpp, built by
__graft_entry__.build()): HIP runtime allocations, the entry points of
include/hisq.h, no Python or torch in the loop, and the C oracle as the arbiter
(Dslash both parities, the multi-RHS epilogue, batched plain and mixed CG,
FP64 and mixed multi-shift, error paths)."""

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "capi_c_check")


def test_c_program_against_the_c_oracle(cuda_device):
    if not os.path.exists(EXE):
        pytest.fail("tests/capi_c_check is not built (run __graft_entry__.build())")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "all C-ABI checks passed" in r.stdout
