"""GPU HISQ smearing (hisq_smear_links) against the FP64 oracle, and the
Dslash and solvers on smeared links, whose Naik links are stored compressed
as two rows and a complex factor (multiples of U(3) matrices).

Tolerances: the smeared links are FP64 on both sides (different summation
order, the U(3) projection by the cubic's closed form on the GPU and by an
eigen-decomposition in the oracle): 1e-12 absolute on entries of size ~1.
Dslash and solves as in the other GPU tests (FP64 1e-13, FP32 1e-6, FP16S
2e-3, true residual 1e-10)."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, spinor_nbytes, to_cb
from oracle import smear

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 1e-6, "fp16s": 2e-3}


def gpu_smear(dims, U, apbc):
    import torch
    t = to_device(np.ascontiguousarray(U))
    fat, lng = torch.empty_like(t), torch.empty_like(t)
    hisq().smear_links(dims, t, fat, lng, antiperiodic_t=apbc)
    return to_host(fat), to_host(lng)


@pytest.mark.parametrize("dims,eps,apbc,tol", [((4, 4, 4, 6), 0.5, False, 1e-12), ((6, 4, 4, 8), 0.7, True, 1e-12),
                                                ((10, 6, 4, 8), 0.5, True, 1e-12), ((8, 8, 8, 8), 1.0, False, 1e-10)])
def test_smear_matches_oracle(cuda_device, dims, eps, apbc, tol):
    """eps = 1.0 gives rough links whose fat7 sums V are far from unitary at some
    sites; there the projection V -> V (V^+ V)^(-1/2) amplifies the rounding of
    V by about cond(V)^2, so two correct evaluations (closed-form cubic against
    an eigen-decomposition) differ by up to ~1e-11."""
    flush(f"smear {dims} eps {eps} apbc {apbc}")
    U = synth.thin_links(dims, 97, eps)
    F, L = gpu_smear(dims, U, apbc)
    # the Naik links are -1/24 times U(3) matrices (relative defect 1e-13)
    LL = L.conj().swapaxes(-1, -2) @ L
    assert np.abs(LL - np.eye(3) / 576).max() < 1e-13 / 576
    Fo, Lo = smear.hisq_smear(dims, U, antiperiodic_t=apbc)
    assert np.abs(F - Fo).max() < tol
    assert np.abs(L - Lo).max() < tol


def test_smeared_free_field_large(cuda_device):
    dims = (48, 48, 48, 12)
    flush("smear free field 48^3x12")
    V = synth.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3))
    F, L = gpu_smear(dims, U, True)
    Ff, Lf = synth.free_links(dims, 9 / 8, -1 / 24, antiperiodic_t=True)
    assert np.abs(F - Ff).max() < 1e-14 and np.abs(L - Lf).max() < 1e-15


@pytest.fixture(scope="module")
def smeared(cuda_device):
    dims = (10, 6, 4, 8)
    U = synth.thin_links(dims, 96, 0.5)
    F, L = smear.hisq_smear(dims, U)
    g = make_gauge(dims, F, L)
    gf = make_gauge(dims, F, L, full_links=True)
    yield dims, F, L, g, gf
    g.close()
    gf.close()


def test_smeared_naik_links_are_kappa_compressed(smeared):
    _, _, _, g, gf = smeared
    assert g.comp_mode == 2 and gf.comp_mode == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("which", ["compressed", "whole"])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_dslash_on_smeared_links(smeared, prec, which, nrhs):
    import torch
    dims, F, L, g, gf = smeared
    h = g if which == "compressed" else gf
    vh = synth.volume(dims) // 2
    srcs = synth.gaussian_source(dims, 96, nrhs, parity=1, index0=5)
    raw = np.concatenate([encode(to_cb(dims, s_, 1), prec) for s_ in srcs])
    inp = to_device(raw)
    nb = spinor_nbytes(prec, vh)
    out = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    hisq().dslash_multi_rhs(h, 0, prec, nrhs, inp, out)
    got = to_host(out)
    for i in range(nrhs):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(got[i * nb:(i + 1) * nb], vh, prec), want) <= TOL[prec], i


def _smeared_solve(smeared, **kw):
    import torch
    dims, F, L, g, _ = smeared
    mass = 0.05
    b = synth.gaussian_source(dims, 96, 1, parity=0, index0=9)[0]
    bd = to_device(encode(to_cb(dims, b, 0), "fp64"))
    x = torch.zeros_like(bd)
    rc, st = hisq().cg_solve(g, mass, 1, bd, x, hisq().solver_params(**kw))
    xf = from_cb(dims, decode(to_host(x), synth.volume(dims) // 2, "fp64"), 0)
    return rc, st[0], oracle.true_residual(dims, F, L, mass, b, xf)


@pytest.mark.parametrize("sloppy", ["fp64", "fp32", "fp16s"])
def test_solve_on_smeared_links(smeared, sloppy):
    """CG on the smeared links to the 1e-10 true residual.  The smeared field is
    well conditioned (about 180 FP64 iterations at m = 0.05), so the iterated
    residual falls by more than five decades per 100 iterations: mixed precision
    keeps the FP64 iteration count only because a reliable update also comes
    whenever the iterated residual has fallen tenfold (with updates every 100
    iterations alone, FP32 needed 26 times the FP64 count and FP16S stalled).
    FP16S rounds every Dslash to ~3e-4, which costs CG some of its
    orthogonality: 1.7 times the FP64 count here."""
    rc, st, res = _smeared_solve(smeared, sloppy_prec=sloppy, fallback=0)
    assert rc == 0 and res <= 1e-10, (rc, res, st)
    if sloppy != "fp64":
        _, st64, _ = _smeared_solve(smeared, sloppy_prec="fp64")
        assert st["iterations"] <= (1.1 if sloppy == "fp32" else 2.0) * st64["iterations"], (st, st64)


def test_reliable_update_by_residual_drop_alone(smeared):
    """With the periodic reliable update pushed out of reach, the tenfold-drop
    trigger alone keeps mixed FP32 CG at the FP64 iteration count; with both off
    the sloppy recurrence runs far past FP32 accuracy and the solve stalls."""
    _, st64, _ = _smeared_solve(smeared, sloppy_prec="fp64")
    rc, st, res = _smeared_solve(smeared, sloppy_prec="fp32", ru_period=100000, fallback=0)
    assert rc == 0 and res <= 1e-10 and st["iterations"] <= 1.1 * st64["iterations"], (st, st64)
    rc, st, res = _smeared_solve(smeared, sloppy_prec="fp32", ru_period=100000, ru_delta=0.0, fallback=0,
                                 max_iter=20 * st64["iterations"])
    assert rc == hisq().NOT_CONVERGED, (rc, st)


def test_smear_full_size_sampled(cuda_device):
    """96^3 x 24 (the benchmark lattice): smeared links at sampled sites against
    the oracle's single-site evaluation, and the Dslash on them (compressed
    Naik links, FP32) at sampled output sites."""
    import torch
    dims = (96, 96, 96, 24)
    flush("smear 96^3x24: thin links")
    U = synth.thin_links(dims, synth.CFG_IDS["c5"], 0.5)
    t = to_device(U)
    fat, lng = torch.empty_like(t), torch.empty_like(t)
    flush("smear 96^3x24: smearing")
    hisq().smear_links(dims, t, fat, lng, antiperiodic_t=False)
    torch.cuda.synchronize()
    del t
    V = synth.volume(dims)
    rng = np.random.default_rng(4)
    sites = rng.choice(V, 3, replace=False)
    for s_ in sites:
        f, l = smear.hisq_smear_at(dims, U, int(s_))
        gf = fat.view(V, 4, 3, 3)[int(s_)].cpu().numpy()
        gl = lng.view(V, 4, 3, 3)[int(s_)].cpu().numpy()
        assert np.abs(gf - f).max() < 1e-12 and np.abs(gl - l).max() < 1e-12, s_
    flush("smear 96^3x24: Dslash on the smeared links")
    g = hisq().Gauge(dims, fat, lng, ("fp32",))
    assert g.comp_mode == 2
    Fh, Lh = to_host(fat), to_host(lng)
    del fat, lng
    torch.cuda.empty_cache()
    chi = synth.gaussian_source(dims, 5, 1, parity=1)[0]
    inp = to_device(encode(to_cb(dims, chi, 1), "fp32"))
    out = torch.empty_like(inp)
    hisq().dslash_eo(g, 0, "fp32", inp, out)
    vh = V // 2
    got = decode(to_host(out), vh, "fp32")
    chi_q = from_cb(dims, decode(to_host(inp), vh, "fp32"), 1)
    par = synth.site_parity(dims)
    even = np.nonzero(par == 0)[0]
    pick = rng.choice(len(even), 256, replace=False)
    want = oracle.dslash_sites(dims, Fh, Lh, chi_q, even[pick])
    assert rel_l2(got[:, pick], want.T) <= 1e-6
    g.close()
