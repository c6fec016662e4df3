"""Host-side checks of bench.py: the one-GPU contract and the algorithmic
byte counts its roofline uses (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_link_bytes_per_site():
    """16 links per output site: 18 reals each when whole; the 8 long links as
    two rows (12 reals) plus a 4-byte sign word per site (comp 1) or a complex
    factor each (comp 2)."""
    import bench
    assert bench.link_bytes_per_site("fp64", 0) == 16 * 18 * 8 == 2304
    assert bench.link_bytes_per_site("fp64", 1) == 2304          # FP64 links are always whole
    assert bench.link_bytes_per_site("fp32", 0) == 1152
    assert bench.link_bytes_per_site("fp32", 1) == 8 * 18 * 4 + 8 * 12 * 4 + 4 == 964
    assert bench.link_bytes_per_site("fp32", 2) == 8 * 18 * 4 + 8 * 12 * 4 + 8 * 2 * 4 == 1024
    assert bench.link_bytes_per_site("fp16s", 1) == 8 * 18 * 2 + 8 * 12 * 2 + 4 == 484
    assert bench.link_bytes_per_site("fp16s", 2) == 8 * 18 * 2 + 8 * 12 * 2 + 8 * 2 * 2 == 512
