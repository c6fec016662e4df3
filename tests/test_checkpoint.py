"""Network-weight checkpoints: raw complex128 plus a JSON header (host only)."""

import numpy as np
import pytest

from paper_2111_10354_amd import checkpoint


def test_round_trip(tmp_path):
    ch = (1, 8, 8, 1)
    rng = np.random.default_rng(0)
    w = rng.standard_normal(720) + 1j * rng.standard_normal(720)
    p = str(tmp_path / "net")
    checkpoint.save(p, w, ch, dims=(32, 32, 32, 8), loss=0.4385, seed=7)
    w2, h = checkpoint.load(p)
    assert np.array_equal(w, w2)
    assert h["channels"] == list(ch) and h["num_weights"] == 720 and h["dims"] == [32, 32, 32, 8]
    assert h["loss"] == 0.4385 and h["seed"] == 7
    assert (tmp_path / "net.bin").stat().st_size == 720 * 16


def test_size_checks(tmp_path):
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "a"), np.zeros(10, complex), (1, 2, 1))
    p = str(tmp_path / "b")
    checkpoint.save(p, np.zeros(36, complex), (1, 2, 1))
    with open(p + ".bin", "ab") as f:
        f.write(b"\0" * 16)
    with pytest.raises(ValueError):
        checkpoint.load(p)
    assert checkpoint.num_weights((1, 8, 8, 1)) == 720
