"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (the shapes of the committed tuning table): the FP64, FP32 and
FP16S Dslash on 96^3 x 24 with 1 and 4 right-hand sides, long links whole and
compressed, and the 16-RHS Dslash on 48^3 x 12.  The oracle cannot apply the
operator to 21 million sites in seconds, so every right-hand side is checked
on 256 random output sites plus ~150 sites on the lattice faces, where the
fat and Naik hops wrap around (every direction, coordinates 0-2 and L-3 to
L-1, and corners), which the oracle computes one by one; the
tolerances are those of the small-lattice parity tests (FP64 1e-13, FP32 1e-6,
FP16S 2e-3 relative L2 over the sample, the oracle fed the GPU's rounded
input).
"""

import os
import shutil

import numpy as np
import pytest

import oracle
import synth
from gpu_util import flush, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, parity_sites, rel_l2, spinor_nbytes, to_cb

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2111_10354_amd", "tuning", "gfx950.jsonl")
TOL = {"fp64": 1e-13, "fp32": 1e-6, "fp16s": 2e-3}
NSAMPLE = 256


@pytest.fixture(scope="module")
def tune(tmp_path_factory):
    # a copy: a shape missing from the table is tuned and appended there
    path = tmp_path_factory.mktemp("tune") / "gfx950.jsonl"
    shutil.copy(TABLE, path)
    return str(path)


def face_sites(dims, rng, per_face=6):
    """Even output sites (as parity indices h) where hops wrap around the
    lattice: for every direction, sites whose coordinate is 0, 1, 2, L-3, L-2
    or L-1 (the fat and Naik hops that cross the boundary), plus corners with
    every coordinate on a face."""
    L = np.array(dims)
    edge = lambda n: np.array([0, 1, 2, n - 3, n - 2, n - 1])  # noqa: E731
    pts = []
    for mu in range(4):
        for e in edge(dims[mu]):
            for _ in range(per_face):
                c = rng.integers(0, L)
                c[mu] = e
                pts.append(c)
    for _ in range(16):
        pts.append(np.array([rng.choice(edge(n)) for n in dims]))
    hs = set()
    for c in pts:
        if c.sum() % 2:  # make it even: move along a direction other than the face's, inside the lattice
            nu = int(np.argmax(L))
            c[nu] = (c[nu] + 1) % dims[nu] if c[nu] not in (0, dims[nu] - 1) else c[nu] ^ 1
            if c.sum() % 2:
                c[0] = c[0] ^ 1
        lex = c[0] + dims[0] * (c[1] + dims[1] * (c[2] + dims[2] * c[3]))
        assert (c.sum() % 2) == 0
        hs.add(int(lex) // 2)
    return np.array(sorted(hs))


def sampled_check(g, dims, F, L, prec, nrhs, seed, tune):
    import torch
    vh = synth.volume(dims) // 2
    hisq().autotune(g, prec, nrhs, tune)
    srcs = synth.gaussian_source(dims, seed, nrhs, parity=1)
    raw = [encode(to_cb(dims, s, 1), prec) for s in srcs]
    del srcs
    inp = to_device(np.concatenate(raw))
    nb = spinor_nbytes(prec, vh)
    out = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    if nrhs == 1:
        hisq().dslash_eo(g, 0, prec, inp, out)
    else:
        hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, out)
    got = to_host(out).reshape(nrhs, -1)
    even = parity_sites(dims, 0)
    rng = np.random.default_rng(seed)
    faces = face_sites(dims, rng)
    for i in range(nrhs):
        hs = np.union1d(rng.choice(vh, size=NSAMPLE, replace=False), faces)
        chi_q = from_cb(dims, decode(raw[i], vh, prec), 1)
        want = oracle.dslash_sites(dims, F, L, chi_q, even[hs])
        have = decode(got[i], vh, prec)[:, hs].T
        err = rel_l2(have, want)
        assert err <= TOL[prec], (prec, nrhs, i, err, hisq().dslash_shape(g, prec, nrhs, 0))
    return hisq().dslash_shape(g, prec, nrhs, 0)


@pytest.fixture(scope="module")
def c5_fields():
    c = synth.CONFIGS["c5"]
    flush(f"full-size fields {c['dims']}")
    F, L = synth.hisq_links(c["dims"], synth.CFG_IDS["c5"], c["eps"])
    return c["dims"], F, L


# the headline launch and its variants in the benchmark (FP64 links are always
# stored whole, so the compressed gauge has no FP64 case)
CASES = {True: [("fp32", 1), ("fp64", 1), ("fp16s", 1), ("fp32", 4), ("fp16s", 4)],
         False: [("fp32", 1), ("fp16s", 1), ("fp32", 4), ("fp16s", 4)]}


@pytest.mark.parametrize("full", [True, False], ids=["whole", "compressed"])
def test_c5_dslash_sampled(cuda_device, c5_fields, tune, full):
    dims, F, L = c5_fields
    g = make_gauge(dims, F, L, full_links=full)
    try:
        assert g.compressed == (not full)
        for prec, nrhs in CASES[full]:
            flush(f"96^3x24 {'whole' if full else 'compressed'} {prec} nrhs={nrhs}")
            shape = sampled_check(g, dims, F, L, prec, nrhs, 100 + nrhs, tune)
            flush(f"  shape {shape} ok")
    finally:
        g.close()


def test_c3_sixteen_rhs_sampled(cuda_device, tune):
    c = synth.CONFIGS["c3"]
    dims = c["dims"]
    F, L = synth.hisq_links(dims, synth.CFG_IDS["c3"], c["eps"])
    g = make_gauge(dims, F, L, precs=("fp32", "fp16s"))
    try:
        for prec in ("fp32", "fp16s"):
            flush(f"48^3x12 {prec} nrhs=16")
            shape = sampled_check(g, dims, F, L, prec, 16, 300, tune)
            flush(f"  shape {shape} ok")
    finally:
        g.close()
