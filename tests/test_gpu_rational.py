"""GPU rational functions of A (hisq_rational_apply, hisq_spectral_bounds,
with hisq_zolotarev_inv_sqrt and hisq_rational_remez coefficients) against
the oracle: the exact dense A^(-1/2) b on 4^4 within the Zolotarev
error bound, and the oracle's partial-fraction sum (independent CGs per pole)
on larger lattices within the solver tolerance.

Tolerance of the partial-fraction sum: every shifted solve stops at a true
relative residual <= 1e-10, so |x_k - x_k*| <= 1e-10 |b| / (lmin + sigma_k);
summed with the positive residues, the result differs from the exact sum by
at most 1e-10 |b| sum_k alpha_k / (lmin + sigma_k) <= 1e-10 |b| r(lmin), i.e.
about 1e-10 (1 + delta) |b| / sqrt(lmin) - well under 1e-8 relative here.
"""

import numpy as np
import pytest

import oracle.rational as R
import synth
from gpu_util import fields, flush, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, to_cb

pytestmark = pytest.mark.gpu


def run(g, dims, mass, a0, al, sh, b, **kw):
    import torch
    vh = synth.volume(dims) // 2
    bd = to_device(encode(to_cb(dims, b, 0), "fp64"))
    out = torch.full_like(bd, 0x77)
    rc, st = hisq().rational_apply(g, mass, a0, al, sh, bd, out, hisq().solver_params(**kw))
    return rc, st, from_cb(dims, decode(to_host(out), vh, "fp64"), 0)


def test_inverse_sqrt_matches_dense(cuda_device):
    dims = (4, 4, 4, 4)
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    mass = 0.1
    b = synth.gaussian_source(dims, 11, 1, parity=0)[0]
    exact, lo, hi = R.dense_power(dims, F, L, mass, b, -0.5)
    for npole in (4, 10):
        a0, al, sh, delta = hisq().zolotarev_inv_sqrt(lo, hi, npole)
        flush(f"rational 4^4 npole={npole} delta={delta:.2e}")
        rc, st, got = run(g, dims, mass, a0, al, sh, b)
        assert rc == 0, st
        err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        assert err <= delta * (1 + 1e-6) + 1e-8, (npole, err, delta)
        # pseudofermion action b^+ A^(-1/2) b
        s_gpu = np.vdot(b, got).real
        s_exact = np.vdot(b, exact).real
        assert abs(s_gpu / s_exact - 1) <= delta + 1e-8
    g.close()


@pytest.mark.parametrize("sloppy", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("full", [False, True], ids=["compressed", "full"])
def test_partial_fractions_match_oracle(cuda_device, full, sloppy):
    """FP64 multi-shift, and the mixed one (FP32 Krylov iteration, refinement
    with FP32 or FP16S sloppy iterations): the same answer to 1e-8."""
    dims = (8, 8, 8, 8)
    F, L = fields(dims, cfg_id=0, eps=0.3)
    g = make_gauge(dims, F, L, full_links=full)
    mass = 0.05
    lo, hi = hisq().spectral_bounds(g, mass, 200)
    a0, al, sh, delta = hisq().zolotarev_inv_sqrt(lo, 1.05 * hi, 12)
    b = synth.gaussian_source(dims, 12, 1, parity=0)[0]
    flush(f"rational 8^4 bounds [{lo:.3e}, {hi:.3e}] delta={delta:.2e} sloppy {sloppy}")
    rc, st, got = run(g, dims, mass, a0, al, sh, b, sloppy_prec=sloppy)
    assert rc == 0, st
    assert all(s["true_residual"] <= 1e-10 for s in st)
    want = R.rational_apply(dims, F, L, mass, a0, al, sh, b, tol=1e-12)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-8
    g.close()


def test_spectral_bounds_against_dense(cuda_device):
    dims = (4, 4, 4, 4)
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    mass = 0.1
    _, lo, hi = R.dense_power(dims, F, L, mass, synth.gaussian_source(dims, 1, 1, parity=0)[0], 1.0)
    blo, bhi = hisq().spectral_bounds(g, mass, 300)
    assert blo == pytest.approx(4 * mass * mass, rel=1e-15) and blo <= lo * (1 + 1e-12)
    # a Rayleigh quotient never exceeds the top eigenvalue; 300 steps get close
    assert 0.9 * hi <= bhi <= hi * (1 + 1e-12), (bhi, hi)
    g.close()


def test_degenerate_and_invalid(cuda_device):
    import torch
    dims = (4, 4, 4, 4)
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    b = synth.gaussian_source(dims, 13, 1, parity=0)[0]
    # no poles: out = alpha0 b exactly
    rc, st, got = run(g, dims, 0.1, 2.5, [], [], b)
    assert rc == 0 and np.array_equal(got, 2.5 * b)   # b vanishes on odd sites
    bd = to_device(encode(to_cb(dims, b, 0), "fp64"))
    out = torch.empty_like(bd)
    with pytest.raises(hisq().HisqError):   # shift below -4 m^2
        hisq().rational_apply(g, 0.1, 0.0, [1.0], [-0.05], bd, out)
    with pytest.raises(hisq().HisqError):   # in place
        hisq().rational_apply(g, 0.1, 0.0, [1.0], [0.1], bd, bd)
    with pytest.raises(hisq().HisqError):
        hisq().spectral_bounds(g, -0.1, 10)
    g.close()


@pytest.mark.parametrize("flavour", ["light", "strange"])
def test_heatbath_action_identity(cuda_device, flavour):
    """RHMC pseudofermions through the library, with Remez coefficients
    (light: heat bath phi = A^(1/4) eta, action phi^+ A^(-1/2) phi; strange:
    A^(1/8) and A^(-1/4)).  phi matches the oracle's partial-fraction
    sum with the same coefficients, and the action returns |eta|^2 up to the
    two approximation errors.  Tolerance of phi: the residues of a positive
    power are negative and cancel against alpha0, so the solver error is
    amplified by at most sum_k |alpha_k| / (lmin + sigma_k) / lmin^p <= alpha0 /
    lmin^p, a factor ~20 here: at most 2e-9 for solves to 1e-10, under the
    1e-8 asserted."""
    dims = (8, 8, 8, 8)
    F, L = fields(dims, cfg_id=0, eps=0.3)
    g = make_gauge(dims, F, L)
    mass = 0.05
    lo, hi = hisq().spectral_bounds(g, mass, 200)
    hi *= 1.05
    ph, pa = (0.25, -0.5) if flavour == "light" else (0.125, -0.25)
    h = hisq().rational_remez(ph, lo, hi, 12)
    a = hisq().rational_remez(pa, lo, hi, 12)
    eta = synth.gaussian_source(dims, 23, 1, parity=0)[0]
    flush(f"heat bath {flavour} 8^4 [{lo:.2e}, {hi:.2f}] deltas {h[3]:.1e} {a[3]:.1e}")
    rc, st, phi = run(g, dims, mass, h[0], h[1], h[2], eta)
    assert rc == 0 and all(s["true_residual"] <= 1e-10 for s in st), st
    want = R.rational_apply(dims, F, L, mass, h[0], h[1], h[2], eta, tol=1e-12)
    assert np.linalg.norm(phi - want) / np.linalg.norm(want) < 1e-8
    rc, st, psi = run(g, dims, mass, a[0], a[1], a[2], phi)
    assert rc == 0, st
    ratio = np.vdot(phi, psi).real / np.vdot(eta, eta).real
    assert abs(ratio - 1) <= (1 + h[3]) ** 2 * (1 + a[3]) - 1 + 1e-8, (ratio, h[3], a[3])
    g.close()


@pytest.mark.parametrize("sloppy", ["fp64", "fp32", "fp16s"])
def test_batched_sources_match_oracle(cuda_device, sloppy):
    """Four pseudofermion sources through one batched call: each equals the
    oracle's partial-fraction sum to 1e-8, in the caller's order."""
    import torch
    dims = (8, 8, 8, 8)
    F, L = fields(dims, cfg_id=0, eps=0.3)
    g = make_gauge(dims, F, L)
    mass = 0.05
    lo, hi = hisq().spectral_bounds(g, mass, 200)
    a0, al, sh, delta = hisq().rational_remez(0.25, lo, 1.05 * hi, 10)
    vh = synth.volume(dims) // 2
    etas = synth.gaussian_source(dims, 31, 4, parity=0)
    bd = to_device(np.concatenate([encode(to_cb(dims, e, 0), "fp64") for e in etas]))
    out = torch.full_like(bd, 0x77)
    flush(f"batched rational 8^4 4 sources {sloppy}")
    rc, st = hisq().rational_apply_batched(g, mass, 4, a0, al, sh, bd, out, hisq().solver_params(sloppy_prec=sloppy))
    assert rc == 0, st
    assert len(st) == 4 * len(sh) and all(s["true_residual"] <= 1e-10 for s in st)
    got = to_host(out).reshape(4, -1)
    for j in range(4):
        phi = from_cb(dims, decode(got[j], vh, "fp64"), 0)
        want = R.rational_apply(dims, F, L, mass, a0, al, sh, etas[j], tol=1e-12)
        assert np.linalg.norm(phi - want) / np.linalg.norm(want) < 1e-8, j
    # no poles: out_j = alpha0 b_j exactly, for every source
    out.fill_(0x77)
    rc, st = hisq().rational_apply_batched(g, mass, 4, 2.5, [], [], bd, out)
    assert rc == 0 and st == []
    assert np.array_equal(to_host(out).view(np.float64), 2.5 * to_host(bd).view(np.float64))
    g.close()
