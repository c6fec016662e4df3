"""Pins of the FP64 oracle against facts fixed by the mathematics, not by the oracle.

Each test names the property it checks and the part of the operator a
plausible mistake would break:

* free-field plane waves are eigenvectors of A with the closed-form eigenvalue
  4[m^2 + sum_mu (c1 sin p_mu + c3 sin 3p_mu)^2]   (Naik hop distance, signs of
  the normal operator, phase folding);
* anti-hermiticity D^+ = -D                       (sign / adjoint of backward hops);
* gauge covariance                                (which site's link a hop uses);
* translation by two sites                        (index arithmetic, wrap-around);
* dense 4^4 brute force: linear solve and spectrum (the whole chain);
* the explicit-phase operator equals the folded one (the generator's folding).
"""

import math

import numpy as np
import pytest

import oracle
from oracle import dense, gauge
import synth

COEFFS = [(9 / 8, -1 / 24), (1.0, 0.0), (0.6, 1.0)]


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 8, 4), (8, 6, 4, 10)])
@pytest.mark.parametrize("c1,c3", COEFFS)
@pytest.mark.parametrize("apbc", [False, True])
def test_free_field_plane_waves(dims, c1, c3, apbc):
    F, L = synth.free_links(dims, c1, c3, antiperiodic_t=apbc)
    mass = 0.07
    rng = np.random.default_rng(5)
    for _ in range(4):
        n = [int(rng.integers(0, d)) for d in dims]
        colour = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        v, p = synth.plane_wave(dims, n, colour, parity=0, antiperiodic_t=apbc)
        Av = oracle.normal_op(dims, F, L, mass, v)
        lam = dense.free_field_eigenvalue(p, mass, c1, c3)
        assert _rel(Av, lam * v) < 1e-13


def test_free_field_eigenvalue_closed_form_values():
    # p = (pi/2, 0, 0, 0): sin p = 1, sin 3p = -1
    assert math.isclose(dense.free_field_eigenvalue([math.pi / 2, 0, 0, 0], 0.0, 1.0, 0.0), 4.0)
    assert math.isclose(dense.free_field_eigenvalue([math.pi / 2, 0, 0, 0], 0.5, 1.0, 1.0), 1.0)
    # tree-level Naik coefficients: c1 sin p + c3 sin 3p = p + O(p^5)
    p = 1e-2
    c1, c3 = 9 / 8, -1 / 24
    val = c1 * math.sin(p) + c3 * math.sin(3 * p)
    assert abs((val - p) / p ** 5 + 3 / 40) < 1e-3


def _free_dslash_closed_form(dims, c1, c3, colour, p):
    """(D v)(x) for a plane wave v = e^{ip.x} colour on the other parity and free
    folded links F = c1 eta bc, L = c3 eta bc: a hop of +-1 or +-3 sites along mu
    multiplies by e^{+-ip_mu} or e^{+-3ip_mu} (with an antiperiodic time direction
    the boundary sign cancels against the half-odd momentum), so
    (D v)(x) = 2i sum_mu eta_mu(x) (c1 sin p_mu + c3 sin 3p_mu) e^{ip.x} colour."""
    coef = 2j * (c1 * np.sin(p) + c3 * np.sin(3 * p))
    phase = np.exp(1j * (synth.site_coords(dims) @ p))
    return (synth.staggered_eta(dims) @ coef)[:, None] * phase[:, None] * np.asarray(colour)[None, :]


@pytest.mark.parametrize("dims,apbc", [((4, 4, 4, 4), False), ((6, 4, 4, 10), True), ((8, 6, 4, 10), False)])
@pytest.mark.parametrize("c1,c3", COEFFS)
def test_free_field_dslash_closed_form_at_every_site(dims, apbc, c1, c3):
    """The Dslash itself (not only A) on free-field plane waves, against the
    closed form at every output site of both parities - through the whole-lattice
    operator and through the sampled-site evaluation used at large sizes."""
    F, L = synth.free_links(dims, c1, c3, antiperiodic_t=apbc)
    rng = np.random.default_rng(11)
    par = synth.site_parity(dims)
    for out_par in (0, 1):
        n = [int(rng.integers(0, d)) for d in dims]
        colour = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        v, p = synth.plane_wave(dims, n, colour, parity=1 - out_par, antiperiodic_t=apbc)
        want = _free_dslash_closed_form(dims, c1, c3, colour, p)
        want[par != out_par] = 0
        got = oracle.dslash(dims, F, L, v, out_par)
        assert _rel(got, want) < 1e-13
        sites = np.nonzero(par == out_par)[0]
        got_s = oracle.dslash_sites(dims, F, L, v, sites)
        assert _rel(got_s, want[sites]) < 1e-13


@pytest.mark.parametrize("dims,apbc", [((4, 4, 4, 4), False), ((6, 4, 4, 10), True), ((8, 6, 4, 10), False)])
def test_dslash_sites_equals_dslash_everywhere(dims, apbc):
    """The sampled-site evaluation (which judges the full-size GPU parity) gives
    the whole-lattice operator's value at every site, of either parity, on random
    fields, in any order of the sites."""
    F, L = synth.hisq_links(dims, 99, 0.5, antiperiodic_t=apbc)
    for out_par in (0, 1):
        chi = synth.gaussian_source(dims, 99, 1, parity=1 - out_par, index0=3)[0]
        full = oracle.dslash(dims, F, L, chi, out_par)
        sites = np.random.default_rng(out_par).permutation(synth.volume(dims))
        got = oracle.dslash_sites(dims, F, L, chi, sites)
        # bit for bit: the same sum in the same order (zero on the input's parity)
        assert np.array_equal(got, full[sites])


@pytest.mark.parametrize("dims,apbc", [((4, 4, 4, 4), False), ((6, 4, 4, 8), True)])
def test_anti_hermiticity_random_fields(dims, apbc):
    F, L = synth.hisq_links(dims, 99, 0.5, antiperiodic_t=apbc)
    x = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    y = synth.gaussian_source(dims, 99, 1, parity=0, index0=7)[0]
    Dx = oracle.dslash(dims, F, L, x, 0)    # D_eo x_o
    Dy = oracle.dslash(dims, F, L, y, 1)    # D_oe y_e
    lhs = np.vdot(y, Dx)
    rhs = -np.vdot(Dy, x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # output lives on the requested parity only
    par = synth.site_parity(dims)
    assert np.all(Dx[par == 1] == 0) and np.all(Dy[par == 0] == 0)


def test_dense_operator_is_antihermitian_and_matches_oracle():
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    D = dense.dense_dslash(dims, F, L)
    assert np.abs(D + D.conj().T).max() < 1e-14
    x = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    assert _rel(oracle.dslash(dims, F, L, x, 0), (D @ x.ravel()).reshape(-1, 3)) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 8)])
def test_gauge_covariance(dims):
    F, L = synth.hisq_links(dims, 99, 0.5)
    g = synth.random_gauge_transform(dims)
    chi = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    Fg = gauge.transform_links(dims, F, g, hop=1)
    Lg = gauge.transform_links(dims, L, g, hop=3)
    lhs = oracle.dslash(dims, Fg, Lg, gauge.transform_vector(g, chi), 0)
    rhs = gauge.transform_vector(g, oracle.dslash(dims, F, L, chi, 0))
    assert _rel(lhs, rhs) < 1e-13


def test_plaquette_gauge_invariant_and_free_value():
    dims = (4, 4, 6, 4)
    U = synth.thin_links(dims, 99, 0.5)
    g = synth.random_gauge_transform(dims)
    p0 = gauge.plaquette_per_site(dims, U)
    p1 = gauge.plaquette_per_site(dims, gauge.transform_links(dims, U, g))
    assert np.abs(p0 - p1).max() < 1e-12
    one = np.broadcast_to(np.eye(3, dtype=complex), U.shape).copy()
    assert np.allclose(gauge.plaquette_per_site(dims, one), 18.0)
    # a non-trivial field changes the plaquette (the check above is not vacuous)
    assert np.abs(p0 - 18.0).max() > 1e-2


def test_translation_by_two_sites():
    dims = (6, 4, 4, 8)
    F, L = synth.hisq_links(dims, 99, 0.5)
    chi = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    out = oracle.dslash(dims, F, L, chi, 0)
    for mu in range(4):
        sh = lambda a: gauge._roll(dims, a, mu, 2)  # noqa: E731
        out_s = oracle.dslash(dims, sh(F), sh(L), sh(chi), 0)
        assert _rel(out_s, sh(out)) < 1e-14


@pytest.mark.parametrize("apbc", [False, True])
def test_explicit_phases_match_folded_links(apbc):
    dims = (4, 6, 4, 8)
    Fr, Lr = synth.hisq_links(dims, 99, 0.5, antiperiodic_t=apbc, fold=False)
    Ff, Lf = synth.hisq_links(dims, 99, 0.5, antiperiodic_t=apbc, fold=True)
    chi = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    a = oracle.dslash_phased(dims, Fr, Lr, chi, 1, antiperiodic_t=apbc)
    b = oracle.dslash(dims, Ff, Lf, chi, 1)
    assert _rel(a, b) < 1e-15
    # free field too: unit links with explicit phases = folded free links
    Ffree, Lfree = synth.free_links(dims, 1.1, 0.3, antiperiodic_t=apbc)
    eye = np.broadcast_to(np.eye(3, dtype=complex), Ffree.shape)
    a = oracle.dslash_phased(dims, 1.1 * eye, 0.3 * eye, chi, 1, antiperiodic_t=apbc)
    b = oracle.dslash(dims, Ffree, Lfree, chi, 1)
    assert _rel(a, b) < 1e-15


def test_dense_normal_operator_matches_schur_form():
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    A = dense.dense_normal_op(dims, F, L, 0.1, sigma=0.3)
    e = dense.parity_index(dims, 0)
    b = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    Ab = oracle.normal_op(dims, F, L, 0.1, b, sigma=0.3)
    assert _rel(Ab.ravel()[e], A @ b.ravel()[e]) < 1e-13
    # Hermitian positive definite
    assert np.abs(A - A.conj().T).max() < 1e-13
    assert np.linalg.eigvalsh(A).min() > 4 * 0.1 ** 2


@pytest.mark.parametrize("apbc", [False, True])
def test_dense_free_spectrum(apbc):
    dims = (4, 4, 4, 4)
    mass, c1, c3 = 0.2, 9 / 8, -1 / 24
    F, L = synth.free_links(dims, c1, c3, antiperiodic_t=apbc)
    A = dense.dense_normal_op(dims, F, L, mass)
    ev = np.linalg.eigvalsh(A)
    full = dense.free_field_spectrum(dims, mass, c1, c3, antiperiodic_t=apbc)
    assert np.abs(ev - full[::2]).max() < 1e-12


def test_cg_matches_dense_solve():
    dims = (4, 4, 4, 4)
    mass = 0.1
    F, L = synth.hisq_links(dims, 99, 0.3)
    b = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    x, status, iters, tr = oracle.cg(dims, F, L, mass, b, tol=1e-12)
    assert status == 0 and tr <= 1e-12
    A = dense.dense_normal_op(dims, F, L, mass)
    e = dense.parity_index(dims, 0)
    xd = np.linalg.solve(A, b.ravel()[e])
    kappa = np.linalg.cond(A)
    assert _rel(x.ravel()[e], xd) <= kappa * 1e-12
    assert np.all(x[synth.site_parity(dims) == 1] == 0)
    assert 0 < iters < 2000


def test_true_residual_against_dense():
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.3)
    A = dense.dense_normal_op(dims, F, L, 0.2, sigma=0.05)
    e = dense.parity_index(dims, 0)
    b = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    x = synth.gaussian_source(dims, 99, 1, parity=0, index0=3)[0]
    want = np.linalg.norm(b.ravel()[e] - A @ x.ravel()[e]) / np.linalg.norm(b.ravel()[e])
    got = oracle.true_residual(dims, F, L, 0.2, b, x, sigma=0.05)
    assert abs(got - want) <= 1e-13 * want


def test_multishift_oracle_per_shift_solutions():
    dims = (4, 4, 4, 4)
    mass = 0.05
    F, L = synth.hisq_links(dims, 99, 0.5)
    b = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    shifts = synth.shifted_ladder(4)
    e = dense.parity_index(dims, 0)
    for s, (x, status, iters, tr) in zip(shifts, oracle.multishift_cg(dims, F, L, mass, shifts, b)):
        A = dense.dense_normal_op(dims, F, L, mass, sigma=s)
        res = np.linalg.norm(b.ravel()[e] - A @ x.ravel()[e]) / np.linalg.norm(b)
        assert status == 0 and res <= 1e-10


def test_free_field_solve_closed_form():
    dims = (8, 4, 4, 6)
    mass, c1, c3 = 0.1, 9 / 8, -1 / 24
    F, L = synth.free_links(dims, c1, c3, antiperiodic_t=True)
    v, p = synth.plane_wave(dims, [1, 2, 0, 1], [1, 0.5j, -0.2], parity=0, antiperiodic_t=True)
    x, status, iters, tr = oracle.cg(dims, F, L, mass, v, tol=1e-12)
    lam = dense.free_field_eigenvalue(p, mass, c1, c3)
    assert status == 0
    assert _rel(x, v / lam) < 1e-11
    assert iters <= 3  # one eigenvector: CG ends in one step, plus the true-residual check
