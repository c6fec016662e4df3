"""Host-side bounds check of the Dslash kernel's index arithmetic.

tests/index_check.cpp is built with hipcc against the kernel's own index
helpers (host + device functions of csrc/hisq_internal.h) and the library's
launch validation (order_supported), and enumerates every thread of every
accepted launch shape on lattices from 4^4 to the benchmark's 96^3 x 24:
the threads cover each output site once, every one of the 16 hops lands on the
reference neighbour inside [0, Vh), and every link unit read lies inside the
packed buffer.  No GPU is used.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2111_10354_amd")


def test_kernel_indices_stay_in_bounds(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    if not os.path.exists(os.path.join(LIBDIR, "libhisq.so")):
        pytest.fail("libhisq.so is not built (run __graft_entry__.build())")
    exe = tmp_path / "index_check"
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-I", os.path.join(LIBDIR, "csrc"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "index_check.cpp"), "-L", LIBDIR, "-lhisq", f"-Wl,-rpath,{LIBDIR}",
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe), "big"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "96x96x96x24" in r.stdout and "FAILED" not in r.stdout
