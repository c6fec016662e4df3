"""GPU parity of the single- and multi-RHS Dslash against the FP64 oracle.

Tolerances (relative L2 over the output vector):
* FP64: 1e-13; FP32: 1e-6 -- the stated parity bar of the build;
* FP16S (FP16 links, FP16 values with an FP32 per-site scale, FP32
  arithmetic): 2e-3 -- 2^-12 relative rounding of every link entry and of the
  output, summed over 16 terms, stays near 3e-4; the bar leaves margin.
The oracle is fed exactly the (rounded) input the GPU received, so the error
measured is that of the kernel and of the link/output storage only.  Every
case runs with the long links compressed (two rows stored, the third rebuilt
from unitarity; the default for the unitary Naik links of the workloads) and
with all links stored whole.
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import fields, flush, force_shape, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, spinor_nbytes, to_cb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 1e-6, "fp16s": 2e-3}

# several tiles and a ragged tail (Vh = 480, 960), one exact multiple (2048),
# and a few thousand sites (4096, 6144)
DIMS = [(4, 4, 4, 4), (6, 4, 4, 10), (10, 6, 4, 8), (8, 8, 8, 8), (16, 8, 8, 8), (8, 12, 8, 16)]


@pytest.fixture(scope="module")
def gauges(cuda_device):
    cache = {}

    def get(dims, apbc=False, free=None, full=False):
        key = (dims, apbc, free, full)
        if key not in cache:
            F, L = fields(dims, apbc=apbc, free=free)
            cache[key] = (make_gauge(dims, F, L, full_links=full), F, L)
        return cache[key]

    yield get
    for g, _, _ in cache.values():
        g.close()


def run_dslash(g, dims, F, L, chi_full, parity, prec):
    import torch
    vh = synth.volume(dims) // 2
    raw = encode(to_cb(dims, chi_full, 1 - parity), prec)
    chi_q = from_cb(dims, decode(raw, vh, prec), 1 - parity)
    inp = to_device(raw)
    out = torch.empty(spinor_nbytes(prec, vh), dtype=torch.uint8, device="cuda")
    hisq().dslash_eo(g, parity, prec, inp, out)
    got = decode(to_host(out), vh, prec)
    want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, parity), parity)
    return got, want


@pytest.mark.parametrize("full", [False, True], ids=["compressed", "full"])
@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("parity", [0, 1])
def test_dslash_matches_oracle(gauges, dims, prec, parity, full):
    flush(f"dslash parity dims={dims} prec={prec} parity={parity} full={full}")
    g, F, L = gauges(dims, apbc=(dims[3] % 4 == 2), full=full)
    assert g.compressed == (not full)
    chi = synth.gaussian_source(dims, 99, 1, parity=1 - parity, index0=parity)[0]
    got, want = run_dslash(g, dims, F, L, chi, parity, prec)
    err = rel_l2(got, want)
    assert err <= TOL[prec], err


def test_compression_choice(gauges, cuda_device):
    """Long links are compressed with a sign bit exactly when every one is
    unitary with det +-1, with a complex factor when every one is a positive
    multiple of a unitary matrix, and not at all otherwise."""
    dims = (4, 4, 4, 4)
    g, F, L = gauges(dims)
    assert g.comp_mode == 1
    g2, _, _ = gauges(dims, apbc=True)
    assert g2.comp_mode == 1  # boundary signs make det = -1, still a sign bit
    gf, _, _ = gauges(dims, free=(9 / 8, -1 / 24))
    assert gf.comp_mode == 2  # L = c3 eta 1: a multiple of a unitary matrix
    chi = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    L2 = np.array(L)
    L2[17, 2] *= 1.0 + 1e-9  # one long link scaled: a multiple of a unitary matrix
    L3 = np.array(L)
    L3[17, 2, 0, 1] += 1e-9  # one entry moved off the unitary group
    for Lx, mode in ((L2, 2), (L3, 0)):
        gp = make_gauge(dims, F, Lx)
        assert gp.comp_mode == mode
        for prec in ("fp64", "fp32"):
            got, want = run_dslash(gp, dims, F, Lx, chi, 0, prec)
            assert rel_l2(got, want) <= TOL[prec]
        gp.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_compressed_matches_full(gauges, prec):
    """Same input through both layouts: equal up to the storage rounding of the third row."""
    dims = (10, 6, 4, 8)
    gc, F, L = gauges(dims)
    gw, _, _ = gauges(dims, full=True)
    chi = synth.gaussian_source(dims, 99, 1, parity=0, index0=3)[0]
    a, _ = run_dslash(gc, dims, F, L, chi, 1, prec)
    b, _ = run_dslash(gw, dims, F, L, chi, 1, prec)
    assert rel_l2(a, b) <= TOL[prec], rel_l2(a, b)


def test_fp16s_error_against_unrounded_input(gauges):
    """FP16S end to end, including the quantisation of the input spinor."""
    dims = (8, 8, 8, 8)
    g, F, L = gauges(dims)
    chi = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    got, _ = run_dslash(g, dims, F, L, chi, 0, "fp16s")
    want = to_cb(dims, oracle.dslash(dims, F, L, chi, 0), 0)
    err = rel_l2(got, want)
    flush(f"fp16s end-to-end rel L2 = {err:.3e}")
    assert err <= 3e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dslash_is_deterministic(gauges, prec):
    import torch
    dims = (16, 8, 8, 8)
    g, F, L = gauges(dims)
    vh = synth.volume(dims) // 2
    chi = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    inp = to_device(encode(to_cb(dims, chi, 1), prec))
    outs = []
    for _ in range(3):
        out = torch.empty(spinor_nbytes(prec, vh), dtype=torch.uint8, device="cuda")
        hisq().dslash_eo(g, 0, prec, inp, out)
        outs.append(to_host(out))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_multi_rhs_matches_single(gauges, prec, nrhs):
    import torch
    dims = (10, 6, 4, 8)
    g, F, L = gauges(dims)
    vh = synth.volume(dims) // 2
    srcs = synth.gaussian_source(dims, 99, nrhs, parity=1, index0=10)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    inp = to_device(raw)
    out = torch.empty(spinor_nbytes(prec, vh) * nrhs, dtype=torch.uint8, device="cuda")
    hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, out)
    got = to_host(out).reshape(nrhs, -1)
    nb = spinor_nbytes(prec, vh)
    for i in range(nrhs):
        one = torch.empty(nb, dtype=torch.uint8, device="cuda")
        hisq().dslash_eo(g, 0, prec, inp[i * nb:(i + 1) * nb], one)
        single = to_host(one)
        # same accumulation order per RHS: bitwise equal
        assert np.array_equal(got[i], single), i
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(got[i], vh, prec), want) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_multi_rhs_shifted_epilogue(gauges, prec):
    """out_i = diag_i y_i - D_eo (D_oe y_i) is (A + sigma_i) y_i."""
    import torch
    dims = (8, 8, 8, 8)
    g, F, L = gauges(dims)
    vh = synth.volume(dims) // 2
    nrhs = 4
    mass = 0.1
    sig = [0.0, 1e-3, 0.1, 1.0]
    diag = [4 * mass * mass + s for s in sig]
    ys = synth.gaussian_source(dims, 99, nrhs, parity=0, index0=20)
    raw = np.concatenate([encode(to_cb(dims, y, 0), prec) for y in ys])
    y = to_device(raw)
    nb = spinor_nbytes(prec, vh)
    t = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    out = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    hisq().dslash_multi_rhs(g, 1, prec, nrhs, y, t)
    hisq().dslash_multi_rhs(g, 0, prec, nrhs, t, out, diag=diag, y=y)
    got = to_host(out).reshape(nrhs, -1)
    tol = {"fp64": 1e-13, "fp32": 2e-6, "fp16s": 4e-3}[prec]
    for i in range(nrhs):
        yq = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 0)
        want = to_cb(dims, oracle.normal_op(dims, F, L, mass, yq, sigma=sig[i]), 0)
        assert rel_l2(decode(got[i], vh, prec), want) <= tol


@pytest.mark.parametrize("full", [False, True], ids=["compressed", "full"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_ragged_rhs_tiles(tmp_path, cuda_device, prec, full):
    """17 RHS in tiles of 2, 4, 8 and 16 (the last tile ragged: its missing RHS
    repeat the last one and are never stored), also split over several waves of
    a workgroup, plain and with the (A + sigma_i) epilogue: every shape writes
    exactly what one RHS per thread writes, and nothing beyond the 17 outputs."""
    import torch
    dims = (10, 6, 4, 8)
    F, L = fields(dims)
    g = make_gauge(dims, F, L, full_links=full)
    vh = synth.volume(dims) // 2
    n = 17
    mass = 0.1
    diag = [4 * mass * mass + 0.05 * k * k for k in range(n)]
    srcs = synth.gaussian_source(dims, 97, n, parity=1, index0=30)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    ys = synth.gaussian_source(dims, 97, n, parity=0, index0=40)
    yraw = np.concatenate([encode(to_cb(dims, y, 0), prec) for y in ys])
    inp, y = to_device(raw), to_device(yraw)
    nb = spinor_nbytes(prec, vh)
    guard = 4 * nb

    def run(shape):
        assert force_shape(g, prec, n, 0, shape, tmp_path / f"p{shape[0]}.jsonl") == shape
        assert force_shape(g, prec, n, 1, shape, tmp_path / f"e{shape[0]}.jsonl") == shape
        out = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        epi = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, out)
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, epi, diag=diag, y=y)
        o, e = to_host(out), to_host(epi)
        assert np.all(o[nb * n:] == 0x5A) and np.all(e[nb * n:] == 0x5A)
        return o[:nb * n], e[:nb * n]

    ref, ref_e = run((1, 64, 0))
    tiles = (2, 4) if prec == "fp64" else (2, 4, 8, 16)
    for tile in tiles:
        got, got_e = run((tile, 128, 0))
        assert np.array_equal(got, ref), tile
        assert np.array_equal(got_e, ref_e), tile
    # RHS tiles of a site split over 2 or 4 waves of a workgroup (bits 24-25 of
    # the order), the last workgroup's waves partly past the 17th RHS
    for tile, block, rsl in ((1, 128, 1), (1, 256, 2), (2, 256, 1), (4, 256, 2), (2, 256, 2)):
        got, got_e = run((tile, block, rsl << 24))
        assert np.array_equal(got, ref), (tile, block, rsl)
        assert np.array_equal(got_e, ref_e), (tile, block, rsl)
    for i in range(n):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(ref[i * nb:(i + 1) * nb], vh, prec), want) <= TOL[prec]
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_field_plane_wave_large_lattice(prec):
    """A p = lambda(p) p for a free-field plane wave on 48^3 x 12 (any size holds)."""
    import torch
    dims = (48, 48, 48, 12)
    c1, c3, mass = 9 / 8, -1 / 24, 0.005
    flush(f"free field 48^3x12 {prec}")
    F, L = synth.free_links(dims, c1, c3, antiperiodic_t=True)
    g = make_gauge(dims, F, L, precs=(prec,))
    del F, L
    vh = synth.volume(dims) // 2
    v, p = synth.plane_wave(dims, [3, 7, 1, 2], [0.3, -1j, 0.5 + 0.2j], parity=0, antiperiodic_t=True)
    lam = 4 * (mass ** 2 + np.sum((c1 * np.sin(p) + c3 * np.sin(3 * p)) ** 2))
    y = to_device(encode(to_cb(dims, v, 0), prec))
    nb = spinor_nbytes(prec, vh)
    t = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = torch.empty(nb, dtype=torch.uint8, device="cuda")
    hisq().dslash_eo(g, 1, prec, y, t)
    hisq().dslash_multi_rhs(g, 0, prec, 1, t, out, diag=[4 * mass * mass], y=y)
    got = decode(to_host(out), vh, prec)
    want = lam * decode(to_host(y), vh, prec)
    assert rel_l2(got, want) <= (1e-12 if prec == "fp64" else 2e-6)
    g.close()


def test_rejects_unpacked_precision():
    dims = (4, 4, 4, 4)
    F, L = fields(dims)
    g = make_gauge(dims, F, L, precs=("fp32",))
    import torch
    vh = synth.volume(dims) // 2
    buf = torch.zeros(spinor_nbytes("fp64", vh), dtype=torch.uint8, device="cuda")
    out = torch.zeros_like(buf)
    with pytest.raises(hisq().HisqError) as e:
        hisq().dslash_eo(g, 0, "fp64", buf, out)
    assert e.value.code == hisq().ERR_UNSUPPORTED
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_epilogue_calls_on_two_streams(gauges, prec):
    """Two epilogue calls with different coefficients, issued back to back on two
    streams with no host synchronisation between them: the first call's kernel is
    held back behind a spin on its stream, so without device-side ordering the
    second call's coefficients would reach the first call's kernel.  Both outputs
    must be their own (A + sigma) y against the oracle."""
    import torch
    dims = (8, 8, 8, 8)
    g, F, L = gauges(dims)
    vh = synth.volume(dims) // 2
    mass = 0.1
    nb = spinor_nbytes(prec, vh)
    ys = synth.gaussian_source(dims, 99, 2, parity=0, index0=60)
    raw = np.concatenate([encode(to_cb(dims, y, 0), prec) for y in ys])
    y = to_device(raw)
    t = torch.empty(2 * nb, dtype=torch.uint8, device="cuda")
    hisq().dslash_multi_rhs(g, 1, prec, 2, y, t)
    torch.cuda.synchronize()
    sig = [(0.0, 0.25), (3.0, 0.5)]
    outs = [torch.empty(2 * nb, dtype=torch.uint8, device="cuda") for _ in sig]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        torch.cuda._sleep(50_000_000)   # a bounded spin: the first kernel starts late
        hisq().dslash_multi_rhs(g, 0, prec, 2, t, outs[0], diag=[4 * mass * mass + v for v in sig[0]], y=y,
                                stream=s1)
    with torch.cuda.stream(s2):
        hisq().dslash_multi_rhs(g, 0, prec, 2, t, outs[1], diag=[4 * mass * mass + v for v in sig[1]], y=y,
                                stream=s2)
    torch.cuda.synchronize()
    tol = {"fp64": 1e-13, "fp32": 2e-6}[prec]
    for k, o in enumerate(outs):
        got = to_host(o).reshape(2, -1)
        for i in range(2):
            yq = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 0)
            want = to_cb(dims, oracle.normal_op(dims, F, L, mass, yq, sigma=sig[k][i]), 0)
            assert rel_l2(decode(got[i], vh, prec), want) <= tol, (k, i)


def test_overlapping_stacks_rejected(gauges):
    """A partial overlap of two stacks (out one RHS past in, x overlapping b's
    stack) is refused before any launch, like an exact alias."""
    import torch
    dims = (8, 8, 8, 8)
    g, F, L = gauges(dims)
    vh = synth.volume(dims) // 2
    nb = spinor_nbytes("fp64", vh)
    buf = torch.zeros(3 * nb, dtype=torch.uint8, device="cuda")
    H = hisq()
    cases = [lambda: H.dslash_multi_rhs(g, 0, "fp64", 2, buf[:2 * nb], buf[nb:]),
             lambda: H.dslash_multi_rhs(g, 0, "fp64", 2, buf[nb:], buf[:2 * nb]),
             lambda: H.dslash_multi_rhs(g, 0, "fp64", 1, buf[:nb], buf[2 * nb:], diag=[1.0], y=buf[2 * nb:]),
             lambda: H.dslash_eo(g, 0, "fp64", buf[:nb], buf[nb - 16:2 * nb - 16]),
             lambda: H.cg_solve(g, 0.1, 2, buf[:2 * nb], buf[nb:])]
    for i, call in enumerate(cases):
        with pytest.raises(H.HisqError) as e:
            call()
        assert e.value.code == H.ERR_INVALID and "overlap" in H.last_error(), i


@pytest.mark.parametrize("dims", [(8, 6, 4, 10), (12, 4, 4, 8)])
@pytest.mark.parametrize("full", [False, True], ids=["compressed", "full"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_xrow_staging_shapes(tmp_path, cuda_device, dims, prec, full):
    """Traversal order 3: workgroups of whole x-rows stage their input colour
    vectors in LDS and the x-direction hops read them there.  Every accepted
    block size (whole rows; 8x6x4x10 has rows of 4 even sites and a last
    workgroup past the lattice at block 256, 12x4x4x8 rows of 6, only block 192)
    and RHS tile (9 RHS: ragged tiles) writes exactly what memory order with one
    RHS per thread writes, plain and with the (A + sigma_i) epilogue, and
    nothing past the outputs; the reference is checked against the oracle."""
    import torch
    F, L = fields(dims)
    g = make_gauge(dims, F, L, full_links=full)
    vh = synth.volume(dims) // 2
    lxh = dims[0] // 2
    n = 9
    diag = [0.04 + 0.03 * k for k in range(n)]
    srcs = synth.gaussian_source(dims, 98, n, parity=1, index0=10)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    ys = synth.gaussian_source(dims, 98, n, parity=0, index0=20)
    inp, y = to_device(raw), to_device(np.concatenate([encode(to_cb(dims, v, 0), prec) for v in ys]))
    nb = spinor_nbytes(prec, vh)
    guard = 4 * nb

    def run(shape):
        assert force_shape(g, prec, n, 0, shape, tmp_path / "p.jsonl") == shape
        assert force_shape(g, prec, n, 1, shape, tmp_path / "e.jsonl") == shape
        out = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        epi = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, out)
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, epi, diag=diag, y=y)
        o, e = to_host(out), to_host(epi)
        assert np.all(o[nb * n:] == 0x5A) and np.all(e[nb * n:] == 0x5A)
        return o[:nb * n], e[:nb * n]

    ref, ref_e = run((1, 64, 0))
    tried = 0
    for block in (64, 128, 192, 256):
        if block % lxh:
            continue
        for tile in ((1, 2, 4) if prec == "fp64" else (1, 2, 4, 8)):
            flush(f"x-row {dims} {prec} {'whole' if full else 'compressed'} tile {tile} block {block}")
            got, got_e = run((tile, block, 3))
            assert np.array_equal(got, ref), (tile, block)
            assert np.array_equal(got_e, ref_e), (tile, block)
            tried += 1
    assert tried >= 3
    for i in range(n):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(ref[i * nb:(i + 1) * nb], vh, prec), want) <= TOL[prec]
    g.close()


def test_xrow_staging_in_a_batched_solve(tmp_path, cuda_device):
    """A batched mixed FP32 solve whose Dslash launches use x-row staging."""
    import torch
    dims = (8, 8, 8, 8)
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    mass, n = 0.05, 4
    for epi in (0, 1):
        assert force_shape(g, "fp32", n, epi, (2, 128, 3), tmp_path / f"s{epi}.jsonl") == (2, 128, 3)
    srcs = synth.gaussian_source(dims, 99, n, parity=0, index0=80)
    b = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in srcs]))
    x = torch.zeros_like(b)
    rc, st = hisq().cg_solve(g, mass, n, b, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc == 0, st
    vh = synth.volume(dims) // 2
    xs = to_host(x).reshape(n, -1)
    for i in range(n):
        xi = from_cb(dims, decode(xs[i], vh, "fp64"), 0)
        assert oracle.true_residual(dims, F, L, mass, srcs[i], xi) <= 1e-10, i
    g.close()


@pytest.mark.parametrize("dims", [(10, 6, 4, 8), (8, 6, 4, 10)])
@pytest.mark.parametrize("full", [False, True], ids=["compressed", "full"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_tmarch_shapes(tmp_path, cuda_device, dims, prec, full):
    """Traversal order 4 (t-march): each thread computes K sites of one column,
    t advancing by 2, with the t-direction inputs kept in registers.  Every K
    dividing Lt/2 (10x6x4x8: 1, 2, 4; 8x6x4x10: 1, 5), RHS tile 1, 2, 4 (5 RHS:
    ragged tiles) and split over 1 or 2 waves writes exactly what memory order
    with one RHS per thread writes, plain and with the (A + sigma_i) epilogue,
    and nothing past the outputs; the reference is checked against the oracle."""
    import torch
    F, L = fields(dims)
    g = make_gauge(dims, F, L, full_links=full)
    vh = synth.volume(dims) // 2
    n = 5
    diag = [0.04 + 0.03 * k for k in range(n)]
    srcs = synth.gaussian_source(dims, 98, n, parity=1, index0=30)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    ys = synth.gaussian_source(dims, 98, n, parity=0, index0=40)
    inp, y = to_device(raw), to_device(np.concatenate([encode(to_cb(dims, v, 0), prec) for v in ys]))
    nb = spinor_nbytes(prec, vh)
    guard = 4 * nb

    def run(shape):
        assert force_shape(g, prec, n, 0, shape, tmp_path / "p.jsonl") == shape
        assert force_shape(g, prec, n, 1, shape, tmp_path / "e.jsonl") == shape
        out = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        epi = torch.full((nb * n + guard,), 0x5A, dtype=torch.uint8, device="cuda")
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, out)
        hisq().dslash_multi_rhs(g, 0, prec, n, inp, epi, diag=diag, y=y)
        o, e = to_host(out), to_host(epi)
        assert np.all(o[nb * n:] == 0x5A) and np.all(e[nb * n:] == 0x5A)
        return o[:nb * n], e[:nb * n]

    ref, ref_e = run((1, 64, 0))
    half = dims[3] // 2
    tried = 0
    for k in [k for k in range(1, half + 1) if half % k == 0]:
        for tile, block, rsl in ((1, 64, 0), (2, 128, 0), (4, 256, 0), (1, 128, 1), (2, 256, 1)):
            if prec == "fp64" and tile * (1 << rsl) > 4:
                continue
            shape = (tile, block, 4 | k << 8 | rsl << 24)
            flush(f"t-march {dims} {prec} {'whole' if full else 'compressed'} K {k} tile {tile} block {block} "
                  f"split {1 << rsl}")
            got, got_e = run(shape)
            assert np.array_equal(got, ref), shape
            assert np.array_equal(got_e, ref_e), shape
            tried += 1
    assert tried >= 8
    for i in range(n):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(ref[i * nb:(i + 1) * nb], vh, prec), want) <= TOL[prec]
    g.close()


def test_tmarch_in_a_batched_solve(tmp_path, cuda_device):
    """A batched mixed FP32 solve whose Dslash launches march along t."""
    import torch
    dims = (8, 8, 8, 8)
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    mass, n = 0.05, 4
    shape = (1, 128, 4 | 2 << 8 | 1 << 24)
    for epi in (0, 1):
        assert force_shape(g, "fp32", n, epi, shape, tmp_path / f"s{epi}.jsonl") == shape
    srcs = synth.gaussian_source(dims, 99, n, parity=0, index0=90)
    b = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in srcs]))
    x = torch.zeros_like(b)
    rc, st = hisq().cg_solve(g, mass, n, b, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc == 0, st
    vh = synth.volume(dims) // 2
    xs = to_host(x).reshape(n, -1)
    for i in range(n):
        xi = from_cb(dims, decode(xs[i], vh, "fp64"), 0)
        assert oracle.true_residual(dims, F, L, mass, srcs[i], xi) <= 1e-10, i
    g.close()
