"""Pins of the HISQ smearing oracle (oracle/smear.py) against facts fixed by
the definitions, not by the oracle's own recursion:

* unit links: X = 9/8 and L = -1/24 with the phases folded, so the smeared
  free field obeys the free-field spectrum with the tree-level Naik
  coefficients (c1, c3) = (9/8, -1/24);
* a field that is non-trivial in one direction only (random diagonal SU(3),
  so all transports across it are trivial): every path of the fat7 (+ Lepage)
  smearing of that direction is the link displaced transversally, and the sum
  is an explicit weighted sum over displacements, written here without the
  staple recursion (level-1 weights (1/2)^(3-k) (1/4)^k for k displaced
  directions; level-2 weights 1, 1/16, 1/32, 1/64 and -1/8 at two steps);
* constant commuting links C_mu: every staple is C_mu, so V = W = C_mu,
  X = 9/8 C_mu and L = -1/24 C_mu^3 (a staple with a missing adjoint would
  leave C_nu^2 behind);
* the U(3) projection equals the polar factor P Q^+ of the singular value
  decomposition V = P S Q^+, is unitary and leaves unitary links alone;
* gauge covariance of every level.
"""

import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import dense, gauge, smear


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _unit(dims):
    return np.broadcast_to(np.eye(3, dtype=complex), (synth.volume(dims), 4, 3, 3)).copy()


@pytest.mark.parametrize("apbc", [False, True])
def test_unit_links_give_tree_level_hisq(apbc):
    dims = (4, 6, 4, 8)
    F, L = smear.hisq_smear(dims, _unit(dims), antiperiodic_t=apbc)
    Ff, Lf = synth.free_links(dims, 9 / 8, -1 / 24, antiperiodic_t=apbc)
    assert np.abs(F - Ff).max() < 1e-15 and np.abs(L - Lf).max() < 1e-15
    # and the smeared free field has the free-field spectrum of the HISQ coefficients
    mass = 0.05
    v, p = synth.plane_wave(dims, [1, 2, 3, 1], [1.0, 0.5j, -0.2], parity=0, antiperiodic_t=apbc)
    lam = dense.free_field_eigenvalue(p, mass, 9 / 8, -1 / 24)
    assert _rel(oracle.normal_op(dims, F, L, mass, v), lam * v) < 1e-13


def _one_direction_field(dims, mu, seed):
    """Identity links except a random diagonal SU(3) field in direction mu."""
    rng = np.random.default_rng(seed)
    V = synth.volume(dims)
    th = rng.uniform(-np.pi, np.pi, (V, 2))
    U = _unit(dims)
    U[:, mu] = 0
    U[:, mu, 0, 0] = np.exp(1j * th[:, 0])
    U[:, mu, 1, 1] = np.exp(1j * th[:, 1])
    U[:, mu, 2, 2] = np.exp(-1j * (th[:, 0] + th[:, 1]))
    return U


def _displaced_sum(dims, A, mu, weight):
    """sum over transverse displacements D of weight(D) A(x + D)."""
    others = [d for d in range(4) if d != mu]
    out = np.zeros_like(A)
    for steps in itertools.product(range(-2, 3), repeat=3):
        w = weight(steps)
        if w == 0:
            continue
        shifted = A
        for d, k in zip(others, steps):
            if k:
                shifted = gauge._roll(dims, shifted, d, k)
        out = out + w * shifted
    return out


def _w_level1(steps):
    if any(abs(k) > 1 for k in steps):
        return 0.0
    k = sum(1 for s in steps if s)
    return 0.5 ** (3 - k) * 0.25 ** k


def _w_level2(steps):
    nz = [s for s in steps if s]
    if len(nz) == 1 and abs(nz[0]) == 2:
        return -1 / 8                     # Lepage: two steps in one direction
    if any(abs(k) > 1 for k in steps):
        return 0.0
    return {0: 1.0, 1: 1 / 16, 2: 2 / 64, 3: 6 / 384}[len(nz)]


@pytest.mark.parametrize("mu", range(4))
def test_one_direction_field_is_an_explicit_displacement_sum(mu):
    dims = (6, 4, 6, 4)
    U = _one_direction_field(dims, mu, 10 + mu)
    V = smear.fat7(dims, U, U, **smear.LEVEL1)
    assert _rel(V[:, mu], _displaced_sum(dims, U[:, mu], mu, _w_level1)) < 1e-14
    X = smear.fat7(dims, U, U, **smear.LEVEL2)
    assert _rel(X[:, mu], _displaced_sum(dims, U[:, mu], mu, _w_level2)) < 1e-14
    # the projection of a diagonal matrix normalises each diagonal entry
    W = smear.u3_project(V)
    d = np.einsum("sii->si", V[:, mu])
    assert _rel(W[:, mu], np.einsum("si,ij->sij", d / np.abs(d), np.eye(3))) < 1e-14


def test_constant_commuting_links():
    dims = (4, 4, 6, 4)
    rng = np.random.default_rng(3)
    U = _unit(dims)
    for mu in range(4):
        a, b = rng.uniform(-np.pi, np.pi, 2)
        U[:, mu] = np.diag([np.exp(1j * a), np.exp(1j * b), np.exp(-1j * (a + b))])
    F, L, V, W = smear.hisq_smear(dims, U, want_levels=True)
    Ff, Lf = smear.fold(dims, 9 / 8 * U, -1 / 24 * (U @ U @ U))
    assert np.abs(V - U).max() < 1e-14 and np.abs(W - U).max() < 1e-14
    assert np.abs(F - Ff).max() < 1e-14 and np.abs(L - Lf).max() < 1e-14


def test_u3_projection_is_the_polar_factor():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((500, 3, 3)) + 1j * rng.standard_normal((500, 3, 3))
    W = smear.u3_project(M)
    P, _, Qh = np.linalg.svd(M)
    # (Gaussian matrices reach condition numbers ~1e3; V^+ V squares them)
    assert np.abs(W - P @ Qh).max() < 1e-10
    assert np.abs(W.conj().swapaxes(1, 2) @ W - np.eye(3)).max() < 1e-10
    assert np.abs(smear.u3_project(W) - W).max() < 1e-10
    # a determinant phase survives (U(3), not SU(3))
    assert np.abs(np.abs(np.linalg.det(W)) - 1).max() < 1e-10
    assert np.abs(np.angle(np.linalg.det(W))).max() > 0.5


@pytest.mark.parametrize("apbc", [False, True])
def test_gauge_covariance_of_every_level(apbc):
    dims = (4, 4, 4, 6)
    U = synth.thin_links(dims, 99, 0.5)
    g = synth.random_gauge_transform(dims)
    Ug = gauge.transform_links(dims, U, g)
    F, L, V, W = smear.hisq_smear(dims, U, antiperiodic_t=apbc, want_levels=True)
    Fg, Lg, Vg, Wg = smear.hisq_smear(dims, Ug, antiperiodic_t=apbc, want_levels=True)
    assert _rel(Vg, gauge.transform_links(dims, V, g)) < 1e-13
    assert _rel(Wg, gauge.transform_links(dims, W, g)) < 1e-13
    assert _rel(Fg, gauge.transform_links(dims, F, g)) < 1e-13
    assert _rel(Lg, gauge.transform_links(dims, L, g, hop=3)) < 1e-13
    # the smeared links are U(3) at level 1 and the long links a multiple of it
    assert np.abs(W.conj().swapaxes(-1, -2) @ W - np.eye(3)).max() < 1e-13
    LL = L.conj().swapaxes(-1, -2) @ L
    assert np.abs(LL - np.eye(3) / 24 ** 2).max() < 1e-15


@pytest.mark.parametrize("dims,apbc", [((4, 4, 4, 6), False), ((6, 4, 8, 4), True)])
def test_patch_smearing_equals_whole_lattice(dims, apbc):
    """The single-site evaluation (patch of radius 5, used to check large
    lattices at sampled sites) gives the whole-lattice result at every site."""
    U = synth.thin_links(dims, 98, 0.7)
    F, L = smear.hisq_smear(dims, U, antiperiodic_t=apbc)
    for site in np.random.default_rng(0).choice(synth.volume(dims), 4, replace=False):
        f, l = smear.hisq_smear_at(dims, U, int(site), antiperiodic_t=apbc)
        assert np.abs(f - F[site]).max() < 1e-13 and np.abs(l - L[site]).max() < 1e-13
