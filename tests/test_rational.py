"""Rational approximation of A^(-1/2) (the rooted-staggered pseudofermion
operator of RHMC): pins of the oracle's Zolotarev construction and of its
partial-fraction application, and the library's host-side coefficients
against the oracle.  No GPU.

Pins that do not reuse the construction being tested:
* Chebyshev alternation: a best relative approximation of type (n, n) has
  2n + 2 alternating extrema of equal size, and any wrong coefficient (a
  misplaced pole, the wrong elliptic argument, a dropped factor) breaks it;
* the exact dense power A^(-1/2) b on a 4^4 lattice, which the partial-fraction
  sum must reproduce within the approximation's own error bound delta
  (|r(l) - l^(-1/2)| <= delta l^(-1/2) for every eigenvalue l in the interval);
* one term with alpha = 1, sigma = 0 and alpha0 = 0 is A^(-1) b.

The library's minimax approximations of other powers (Remez exchange) are
pinned the same way: the alternation count and equal sizes on the oracle's
grid, Zolotarev's closed form at p = -1/2 (the optimum is unique), the
reciprocal and scaling symmetries, the exact dense A^p b on 4^4, and the
heat-bath/action identity phi = A^(1/4) eta, phi^+ A^(-1/2) phi = |eta|^2.
"""

import numpy as np
import pytest

import synth
from oracle import rational as R

CASES = [(1, 10.0), (4, 1e4), (8, 1e6), (12, 1e7)]


@pytest.mark.parametrize("n,ratio", CASES)
def test_oracle_zolotarev_equioscillates(n, ratio):
    lmin = 3e-3
    a0, al, sh, delta = R.zolotarev_inv_sqrt(lmin, lmin * ratio, n)
    ex = R.relative_error_extrema(a0, al, sh, lmin, lmin * ratio)
    assert len(ex) == 2 * n + 2
    assert np.all(np.sign(ex[1:]) != np.sign(ex[:-1]))
    mags = np.abs(ex)
    assert mags.max() / mags.min() - 1 < 1e-5
    assert abs(mags.max() / delta - 1) < 1e-5
    # poles on the negative axis, positive residues: every shifted system is HPD
    assert np.all(np.array(sh) > 0) and np.all(np.diff(sh) > 0) and np.all(np.array(al) > 0) and a0 > 0


def test_oracle_zolotarev_error_falls_with_poles():
    d = [R.zolotarev_inv_sqrt(1e-3, 10.0, n)[3] for n in (2, 4, 6, 8, 10)]
    assert all(b < a for a, b in zip(d, d[1:]))
    # and the bound holds off the grid the construction used
    a0, al, sh, delta = R.zolotarev_inv_sqrt(1e-3, 10.0, 6)
    x = np.exp(np.random.default_rng(0).uniform(np.log(1e-3), np.log(10.0), 5000))
    r = a0 + sum(a / (x + s) for a, s in zip(al, sh))
    assert np.max(np.abs(np.sqrt(x) * r - 1)) <= delta * (1 + 1e-6)


def test_oracle_rational_apply_matches_dense_inverse_sqrt():
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    mass = 0.1
    b = synth.gaussian_source(dims, 7, 1, parity=0)[0]
    exact, lo, hi = R.dense_power(dims, F, L, mass, b, -0.5)
    assert lo >= 4 * mass * mass * (1 - 1e-12)
    a0, al, sh, delta = R.zolotarev_inv_sqrt(lo, hi, 8)
    got = R.rational_apply(dims, F, L, mass, a0, al, sh, b)
    err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    assert err <= delta * (1 + 1e-6) + 1e-10
    # fewer poles: the error grows but stays inside its own bound
    a0, al, sh, delta3 = R.zolotarev_inv_sqrt(lo, hi, 3)
    got3 = R.rational_apply(dims, F, L, mass, a0, al, sh, b)
    err3 = np.linalg.norm(got3 - exact) / np.linalg.norm(exact)
    assert err < err3 <= delta3 * (1 + 1e-6) + 1e-10


def test_oracle_rational_apply_single_pole_is_inverse():
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    mass = 0.1
    b = synth.gaussian_source(dims, 8, 1, parity=0)[0]
    inv, _, _ = R.dense_power(dims, F, L, mass, b, -1.0)
    got = R.rational_apply(dims, F, L, mass, 0.0, [1.0], [0.0], b)
    assert np.linalg.norm(got - inv) / np.linalg.norm(inv) < 1e-10


@pytest.mark.parametrize("n,ratio", CASES + [(16, 1e10)])
def test_library_zolotarev_matches_oracle(n, ratio):
    from paper_2111_10354_amd import hisq
    lmin = 2e-3
    a0, al, sh, delta = hisq.zolotarev_inv_sqrt(lmin, lmin * ratio, n)
    o0, oal, osh, od = R.zolotarev_inv_sqrt(lmin, lmin * ratio, n)
    tol = 1e-6 if ratio > 1e8 else 1e-8
    assert abs(a0 / o0 - 1) < tol
    assert np.max(np.abs(np.array(sh) / osh - 1)) < tol
    assert np.max(np.abs(np.array(al) / oal - 1)) < tol
    assert abs(delta / od - 1) < 1e-5


@pytest.mark.parametrize("args", [(0.0, 1.0, 4), (1.0, 0.5, 4), (1.0, 2.0, 0), (1.0, 2.0, 65), (1e-10, 1e5, 4),
                                  (float("nan"), 1.0, 4)])
def test_library_zolotarev_rejects(args):
    from paper_2111_10354_amd import hisq
    with pytest.raises(hisq.HisqError):
        hisq.zolotarev_inv_sqrt(*args)


def test_golden_zolotarev_coefficients():
    """tests/golden/zolotarev_inv_sqrt_n8.json was written by
    tests/golden/make_golden.py from the oracle alone: the oracle still
    reproduces it, and the library's host routine agrees with it."""
    import json
    import os
    from paper_2111_10354_amd import hisq
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "zolotarev_inv_sqrt_n8.json")
    rec = json.load(open(path))
    o0, oal, osh, od = R.zolotarev_inv_sqrt(rec["lmin"], rec["lmax"], rec["npole"])
    assert o0 == pytest.approx(rec["alpha0"], rel=1e-12)
    assert np.allclose(oal, rec["alpha"], rtol=1e-12) and np.allclose(osh, rec["shift"], rtol=1e-12)
    a0, al, sh, delta = hisq.zolotarev_inv_sqrt(rec["lmin"], rec["lmax"], rec["npole"])
    assert a0 == pytest.approx(rec["alpha0"], rel=1e-9)
    assert np.allclose(al, rec["alpha"], rtol=1e-9) and np.allclose(sh, rec["shift"], rtol=1e-9)
    assert delta == pytest.approx(rec["delta"], rel=1e-5)


# Minimax rational approximations of other powers (the library's Remez exchange).
# The pin is Chebyshev's alternation theorem, the definition of the optimum:
# 2n + 2 alternating extrema of one size, counted by the oracle on a fine grid.
REMEZ_CASES = [(0.25, 1e-4, 40.0, 12), (-0.25, 1e-4, 40.0, 12), (0.125, 1e-5, 60.0, 14),
               (-0.125, 1e-5, 60.0, 10), (0.375, 1e-4, 40.0, 8), (-0.75, 1e-4, 40.0, 16),
               (0.75, 1e-4, 40.0, 12), (0.5, 1e-3, 10.0, 2), (-0.25, 1.0, 10.0, 1),
               (0.05, 1e-4, 40.0, 16), (-0.9, 1e-4, 40.0, 16), (0.25, 1e-6, 100.0, 20),
               (0.125, 1e-8, 64.0, 24), (0.55, 1e-3, 100.0, 1)]


@pytest.mark.parametrize("p,lmin,lmax,n", REMEZ_CASES)
def test_library_remez_equioscillates(p, lmin, lmax, n):
    from paper_2111_10354_amd import hisq
    a0, al, sh, delta = hisq.rational_remez(p, lmin, lmax, n)
    ex = R.relative_error_extrema(a0, al, sh, lmin, lmax, power=p)
    assert len(ex) == 2 * n + 2
    assert np.all(np.sign(ex[1:]) != np.sign(ex[:-1]))
    mags = np.abs(ex)
    # the FP64 coefficients of a positive power cancel against alpha0 near
    # lmin (r(0) ~ 0): their rounding enters the relative error amplified by
    # (|alpha0| + sum |alpha_k| / (lmin + sigma_k)) / r(lmin)
    amp = (abs(a0) + sum(abs(a) / (lmin + s) for a, s in zip(al, sh))) / lmin ** p
    tol = 1e-4 + 64 * np.finfo(np.float64).eps * amp / delta
    assert mags.max() / mags.min() - 1 < tol
    assert abs(mags.max() / delta - 1) < tol
    # negative real poles: every shifted system is HPD; residues of one sign
    sh, al = np.array(sh), np.array(al)
    assert np.all(sh > 0) and np.all(np.diff(sh) > 0) and a0 > 0
    assert np.all(np.sign(al) == -np.sign(p))


@pytest.mark.parametrize("n,ratio", CASES + [(16, 1e10)])
def test_library_remez_inverse_sqrt_is_zolotarev(n, ratio):
    """p = -1/2: the best approximation is unique, so the exchange must land on
    Zolotarev's closed form (the oracle's, from scipy's elliptic functions)."""
    from paper_2111_10354_amd import hisq
    lmin = 2e-3
    a0, al, sh, delta = hisq.rational_remez(-0.5, lmin, lmin * ratio, n)
    o0, oal, osh, od = R.zolotarev_inv_sqrt(lmin, lmin * ratio, n)
    assert abs(a0 / o0 - 1) < 1e-6
    assert np.max(np.abs(np.array(sh) / osh - 1)) < 1e-6
    assert np.max(np.abs(np.array(al) / oal - 1)) < 1e-6
    assert abs(delta / od - 1) < 1e-5


@pytest.mark.parametrize("p", [0.125, 0.25, 0.375])
def test_library_remez_reciprocal_and_scale(p):
    """1/r approximates x^(-p) with error -e/(1+e): the optimal errors for p and
    -p agree to O(delta^2).  x^p on [s a, s b] is s^p (x/s)^p: the shifts scale
    by s, alpha0 by s^p, the residues by s^(p+1), the error not at all."""
    from paper_2111_10354_amd import hisq
    a = hisq.rational_remez(p, 1e-4, 40.0, 12)
    m = hisq.rational_remez(-p, 1e-4, 40.0, 12)
    assert abs(a[3] / m[3] - 1) < 1e-5 + 4 * a[3]
    s = 100.0
    b = hisq.rational_remez(p, 1e-4 * s, 40.0 * s, 12)
    assert b[0] == pytest.approx(a[0] * s ** p, rel=1e-9)
    assert np.allclose(b[2], np.array(a[2]) * s, rtol=1e-9)
    assert np.allclose(b[1], np.array(a[1]) * s ** (p + 1), rtol=1e-9)
    assert b[3] == pytest.approx(a[3], rel=1e-5)


@pytest.mark.parametrize("p,lmin,lmax", [(0.25, 1e-2, 1.0), (-0.25, 1e-3, 1.0), (0.125, 1.0, 100.0),
                                           (-0.75, 1e-2, 1.0)])
def test_library_remez_one_pole_is_the_bruteforce_optimum(p, lmin, lmax):
    """One pole: the optimum of the three-parameter problem, found by direct
    minimisation of the largest error on a grid (no exchange, no alternation),
    is the library's."""
    from paper_2111_10354_amd import hisq
    a0, al, sh, delta = hisq.rational_remez(p, lmin, lmax, 1)
    bd, bq = R.minimax_bruteforce(p, lmin, lmax, 1)
    assert abs(bd / delta - 1) < 1e-5
    assert abs(bq[0] / sh[0] - 1) < 1e-4


@pytest.mark.parametrize("n", [1, 2])
@pytest.mark.parametrize("lmin,lmax", [(1e-2, 1.0), (1e-3, 10.0), (1.0, 100.0)])
def test_oracle_bruteforce_finds_zolotarev_optimum(n, lmin, lmax):
    """Pin of the brute-force minimisation (oracle only): at p = -1/2 the best
    relative approximation is unique and Zolotarev's closed form gives it, so
    direct minimisation of the largest error must land on its error and its
    poles."""
    bd, bq = R.minimax_bruteforce(-0.5, lmin, lmax, n)
    _, _, sh, delta = R.zolotarev_inv_sqrt(lmin, lmax, n)
    assert abs(bd / delta - 1) < 2e-6
    assert np.max(np.abs(bq / np.array(sh) - 1)) < 1e-6


@pytest.mark.parametrize("p,lmin,lmax", [(0.125, 1.0, 100.0), (-0.5, 1e-2, 1.0), (0.375, 1e-2, 1.0)])
def test_library_remez_two_poles_is_the_bruteforce_optimum(p, lmin, lmax):
    """Two poles: direct minimisation of the largest error (five parameters, no
    exchange, no alternation) reaches the library's error and poles, and never
    goes below it (it is an approximation of the same type)."""
    from paper_2111_10354_amd import hisq
    _, _, sh, delta = hisq.rational_remez(p, lmin, lmax, 2)
    bd, bq = R.minimax_bruteforce(p, lmin, lmax, 2)
    assert delta <= bd * (1 + 1e-6)
    assert bd <= delta * (1 + 1e-4)
    assert np.max(np.abs(bq / np.array(sh) - 1)) < 1e-3


@pytest.mark.parametrize("n,ratio", [(24, 1e9), (32, 1e9), (32, 1e12), (40, 1e14)])
def test_library_zolotarev_equioscillates_at_large_ratios(n, ratio):
    """Many poles over many decades: the nodes near the top of the interval
    come from a tiny cn, so they are mirrored from the lower half
    (c_l c_{2n+1-l} = b).  The definition then holds down to the accuracy of
    the lower nodes (~1e-12 relative at b = 1e14: the asin steps of the
    descending Landen sequence amplify rounding as m -> 1), i.e. an error
    curve uneven by ~1e-12 absolute, which the tolerance allows."""
    from paper_2111_10354_amd import hisq
    lmin = 1e-3
    a0, al, sh, delta = hisq.zolotarev_inv_sqrt(lmin, lmin * ratio, n)
    ex = R.relative_error_extrema(a0, al, sh, lmin, lmin * ratio, npts=400001)
    assert len(ex) == 2 * n + 2
    assert np.all(np.sign(ex[1:]) != np.sign(ex[:-1]))
    mags = np.abs(ex)
    tol = 1e-4 + 2e-12 / delta
    assert mags.max() / mags.min() - 1 < tol
    assert abs(mags.max() / delta - 1) < tol


@pytest.mark.parametrize("p,n,ratio", [(-0.25, 24, 1e9), (0.125, 32, 1e12), (-0.125, 40, 1e14)])
def test_library_remez_equioscillates_at_large_ratios(p, n, ratio):
    from paper_2111_10354_amd import hisq
    lmin = 1e-3
    a0, al, sh, delta = hisq.rational_remez(p, lmin, lmin * ratio, n)
    ex = R.relative_error_extrema(a0, al, sh, lmin, lmin * ratio, npts=400001, power=p)
    assert len(ex) == 2 * n + 2
    assert np.all(np.sign(ex[1:]) != np.sign(ex[:-1]))
    mags = np.abs(ex)
    amp = (abs(a0) + sum(abs(a) / (lmin + s) for a, s in zip(al, sh))) / lmin ** p
    tol = 1e-4 + 2e-12 / delta + 64 * np.finfo(np.float64).eps * amp / delta
    assert mags.max() / mags.min() - 1 < tol
    assert abs(mags.max() / delta - 1) < tol


@pytest.mark.parametrize("p,n", [(0.25, 8), (-0.25, 8), (0.125, 6)])
def test_remez_partial_fractions_match_dense_power(p, n):
    """The library's coefficients applied by the oracle (one plain CG per pole)
    reproduce the exact dense A^p b on 4^4 within the approximation's bound:
    |r(l) - l^p| <= delta l^p for every eigenvalue l of A in the interval."""
    from paper_2111_10354_amd import hisq
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    mass = 0.1
    b = synth.gaussian_source(dims, 21, 1, parity=0)[0]
    exact, lo, hi = R.dense_power(dims, F, L, mass, b, p)
    a0, al, sh, delta = hisq.rational_remez(p, lo, hi, n)
    got = R.rational_apply(dims, F, L, mass, a0, al, sh, b)
    err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
    assert err <= delta * (1 + 1e-6) + 1e-10, (err, delta)


def test_oracle_heatbath_action_identity():
    """Rooted-staggered RHMC for two flavours: heat bath phi = A^(1/4) eta, action
    S = phi^+ A^(-1/2) phi, so that S = |eta|^2 for every eta; with rational
    approximations S / |eta|^2 - 1 is bounded by the errors of the two
    approximations (|e1| <= d1 twice, |e2| <= d2 once)."""
    from paper_2111_10354_amd import hisq
    dims = (4, 4, 4, 4)
    F, L = synth.hisq_links(dims, 99, 0.5)
    mass = 0.1
    eta = synth.gaussian_source(dims, 22, 1, parity=0)[0]
    _, lo, hi = R.dense_power(dims, F, L, mass, eta, 1.0)
    h = hisq.rational_remez(0.25, lo, hi, 6)
    a = hisq.rational_remez(-0.5, lo, hi, 6)
    phi = R.rational_apply(dims, F, L, mass, h[0], h[1], h[2], eta)
    psi = R.rational_apply(dims, F, L, mass, a[0], a[1], a[2], phi)
    ratio = np.vdot(phi, psi).real / np.vdot(eta, eta).real
    bound = (1 + h[3]) ** 2 * (1 + a[3]) - 1
    assert abs(ratio - 1) <= bound + 1e-10
    assert abs(ratio - 1) > 1e-12        # the approximations are not exact


@pytest.mark.parametrize("args", [(0.0, 1e-3, 1.0, 4), (0.97, 1e-3, 1.0, 4), (-1.0, 1e-3, 1.0, 4),
                                  (0.25, 1.0, 0.5, 4), (0.25, 1e-3, 1.0, 0), (0.25, 1e-3, 1.0, 65),
                                  (0.25, 1.0, 1.01, 6), (float("nan"), 1e-3, 1.0, 4),
                                  (0.95, 1e-4, 40.0, 16), (-0.25, 1e-6, 1.0, 1)])
def test_library_remez_rejects(args):
    """Out of range, or more poles than double precision can resolve on the
    interval (x^(1/4) with 6 poles on [1, 1.01]), or too few to be of any use
    (one pole over six decades: error above 0.5), or partial fractions that
    lose the approximation to cancellation (x^0.95 over 5.6 decades)."""
    from paper_2111_10354_amd import hisq
    with pytest.raises(hisq.HisqError):
        hisq.rational_remez(*args)


def test_library_remez_random_cases_equioscillate():
    """Random powers, intervals and pole counts (deterministic draw): every
    accepted request returns an approximation that meets the definition on the
    oracle's grid; refused requests are the documented ones."""
    from hypothesis import HealthCheck, given, settings, strategies as st
    from paper_2111_10354_amd import hisq

    @settings(max_examples=30, deadline=None, derandomize=True, suppress_health_check=list(HealthCheck))
    @given(p=st.one_of(st.floats(-0.9, -0.05), st.floats(0.05, 0.6)), lratio=st.floats(0.5, 8.0),
           n=st.integers(1, 12))
    def check(p, lratio, n):
        lmin, lmax = 1e-3, 1e-3 * 10 ** lratio
        try:
            a0, al, sh, delta = hisq.rational_remez(p, lmin, lmax, n)
        except hisq.HisqError as e:
            assert any(w in str(e) for w in ("too many poles", "too few poles", "cancellation")), str(e)
            return
        ex = R.relative_error_extrema(a0, al, sh, lmin, lmax, power=p)
        assert len(ex) == 2 * n + 2, (p, lratio, n)
        assert np.all(np.sign(ex[1:]) != np.sign(ex[:-1]))
        mags = np.abs(ex)
        amp = (abs(a0) + sum(abs(a) / (lmin + s) for a, s in zip(al, sh))) / lmin ** p
        tol = 1e-4 + 2e-12 / delta + 64 * np.finfo(np.float64).eps * amp / delta
        assert mags.max() / mags.min() - 1 < tol, (p, lratio, n, mags.max() / mags.min() - 1)
        assert abs(mags.max() / delta - 1) < tol

    check()
