"""Properties of the seeded input generator (shared by oracle and GPU tests)."""

import numpy as np
import pytest

import synth


def test_thin_links_are_su3_and_reproducible():
    dims = (4, 4, 4, 6)
    U = synth.thin_links(dims, 99, 0.5)
    I = np.eye(3)
    assert np.abs(U @ U.conj().transpose(0, 1, 3, 2) - I).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13
    assert np.array_equal(U, synth.thin_links(dims, 99, 0.5))
    assert not np.array_equal(U, synth.thin_links(dims, 98, 0.5))
    # eps sets the distance from the identity: |U - 1| grows with eps
    d3 = np.abs(synth.thin_links(dims, 99, 0.3) - I).mean()
    d5 = np.abs(U - I).mean()
    assert 0 < d3 < d5


def test_haar_su3_unitary_det_one_and_uniform_trace():
    rng = np.random.default_rng(3)
    R = synth.haar_su3(rng, 200000)
    assert np.abs(R @ R.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-13
    # Haar measure on SU(3): E[tr R] = 0, E[|tr R|^2] = 1
    tr = np.trace(R, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.01
    assert abs(np.mean(np.abs(tr) ** 2) - 1) < 0.02


def test_fat_and_long_recipe():
    dims = (4, 4, 6, 4)
    U = synth.thin_links(dims, 99, 0.5)
    F, L, T = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    Fr, Lr = synth.hisq_links(dims, 99, 0.5, fold=False)
    eta = synth.staggered_eta(dims)
    assert np.allclose(F, Fr * eta[:, :, None, None], atol=0)
    assert np.allclose(L, Lr * eta[:, :, None, None], atol=0)
    assert np.allclose(T, U * eta[:, :, None, None], atol=0)
    Lx, Ly, Lz, Lt = dims
    c = synth.site_coords(dims)

    def lex(x):
        return x[0] + Lx * (x[1] + Ly * (x[2] + Lz * x[3]))

    rng = np.random.default_rng(0)
    for s in rng.integers(0, synth.volume(dims), 10):
        for mu in range(4):
            x0 = c[s].copy()
            x1 = x0.copy(); x1[mu] = (x1[mu] + 1) % dims[mu]
            x2 = x0.copy(); x2[mu] = (x2[mu] + 2) % dims[mu]
            want = U[lex(x0), mu] @ U[lex(x1), mu] @ U[lex(x2), mu]
            assert np.allclose(Lr[s, mu], want, atol=1e-14)
    # fat link is 0.6 U + 0.1 R with R in SU(3)
    R = (Fr - 0.6 * U) / 0.1
    assert np.abs(R @ R.conj().transpose(0, 1, 3, 2) - np.eye(3)).max() < 1e-12


def test_parallel_generation_matches_serial():
    dims = (4, 4, 4, 8)
    a = synth.hisq_links(dims, 7, 0.5, workers=1)
    b = synth.hisq_links(dims, 7, 0.5, workers=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_staggered_eta_constant_along_own_direction():
    dims = (4, 6, 4, 8)
    eta = synth.staggered_eta(dims)
    c = synth.site_coords(dims)
    assert np.all(eta[:, 0] == 1)
    assert np.all(eta[:, 1] == (-1.0) ** c[:, 0])
    assert np.all(eta[:, 2] == (-1.0) ** (c[:, 0] + c[:, 1]))
    assert np.all(eta[:, 3] == (-1.0) ** (c[:, 0] + c[:, 1] + c[:, 2]))


def test_sources_live_on_one_parity():
    dims = (4, 4, 4, 4)
    b = synth.gaussian_source(dims, 99, 2, parity=0)
    par = synth.site_parity(dims)
    assert np.all(b[:, par == 1] == 0)
    assert np.all(b[:, par == 0] != 0)
    assert not np.array_equal(b[0], b[1])


def test_shift_ladder():
    s = synth.shifted_ladder(12)
    assert s.shape == (12,) and np.isclose(s[0], 1e-4) and np.isclose(s[-1], 1.0)
    assert np.allclose(np.diff(np.log10(s)), 4 / 11)


def test_bad_dims_rejected():
    with pytest.raises(ValueError):
        synth.free_links((4, 4, 5, 4), 1, 0)
