"""Autotuner: chosen shapes keep the Dslash output bit-identical, the JSON
cache round-trips, and a tuned solve still converges."""

import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import fields, force_shape, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, spinor_nbytes, to_cb

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,nrhs", [("fp32", 1), ("fp32", 4), ("fp16s", 3), ("fp64", 2)])
def test_autotune_keeps_output_and_caches(tmp_path, cuda_device, prec, nrhs):
    import torch
    dims = (16, 8, 8, 8)   # (Lx/2 * Ly) % 64 == 0: both tile orders are candidates
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    vh = synth.volume(dims) // 2
    srcs = synth.gaussian_source(dims, 99, nrhs, parity=1, index0=70)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    inp = to_device(raw)
    nb = spinor_nbytes(prec, vh)
    before = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, before)
    cache = tmp_path / "tune.jsonl"
    hisq().autotune(g, prec, nrhs, str(cache))
    shape = hisq().dslash_shape(g, prec, nrhs, 0)
    order, rsplit = shape[2] & 0xffffff, 1 << ((shape[2] >> 24) & 3)
    assert shape[0] <= nrhs and shape[1] in ((64, 128, 192, 256) if order == 3 else (64, 128, 256))
    assert order in (0, 1, 3) or order & 0xff in (2, 4)
    assert rsplit in (1, 2, 4) and shape[1] // rsplit >= 64 and shape[2] >> 26 == 0
    after = torch.empty_like(before)
    hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, after)
    assert np.array_equal(to_host(before), to_host(after))
    lines = [json.loads(line) for line in cache.read_text().splitlines()]
    assert any(f"|n{nrhs}|e0" in rec["key"] for rec in lines)
    # a fresh handle picks the cached shape without timing anything
    g2 = make_gauge(dims, F, L)
    hisq().autotune(g2, prec, nrhs, str(cache))
    assert hisq().dslash_shape(g2, prec, nrhs, 0) == shape
    assert len(cache.read_text().splitlines()) == len(lines)
    # and the output still matches the oracle
    got = to_host(after).reshape(nrhs, -1)
    tol = {"fp64": 1e-13, "fp32": 1e-6, "fp16s": 2e-3}[prec]
    for i in range(nrhs):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(got[i], vh, prec), want) <= tol
    g.close()
    g2.close()


BRICK = [2 | 8 << 8 | 16 << 16, 2 | 16 << 8 | 8 << 16, 2 | 8 << 8 | 4 << 16]


@pytest.mark.parametrize("prec,nrhs,tile", [("fp32", 1, 1), ("fp32", 4, 4), ("fp16s", 3, 2), ("fp64", 2, 2)])
def test_brick_orders_match_memory_order(tmp_path, cuda_device, prec, nrhs, tile):
    """XCD-brick traversal (a permutation of the output sites, with the
    workgroup-to-XCD remap) writes the same bytes as memory order, and the
    oracle's result."""
    import torch
    dims = (16, 16, 16, 8)   # Lx/2 * BY a multiple of 64 for BY in {8, 16}; 2048 tiles
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    vh = synth.volume(dims) // 2
    srcs = synth.gaussian_source(dims, 98, nrhs, parity=1, index0=71)
    raw = np.concatenate([encode(to_cb(dims, s, 1), prec) for s in srcs])
    inp = to_device(raw)
    nb = spinor_nbytes(prec, vh)
    ref = torch.empty(nb * nrhs, dtype=torch.uint8, device="cuda")
    assert force_shape(g, prec, nrhs, 0, (1, 256, 0), tmp_path / "m.jsonl") == (1, 256, 0)
    hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, ref)
    ref_h = to_host(ref)
    for i, order in enumerate(BRICK):
        for block in (64, 256):
            shape = (tile, block, order)
            assert force_shape(g, prec, nrhs, 0, shape, tmp_path / f"b{i}{block}.jsonl") == shape
            out = torch.full_like(ref, 0xAB)
            hisq().dslash_multi_rhs(g, 0, prec, nrhs, inp, out)
            assert np.array_equal(to_host(out), ref_h), shape
    tol = {"fp64": 1e-13, "fp32": 1e-6, "fp16s": 2e-3}[prec]
    got = ref_h.reshape(nrhs, -1)
    for i in range(nrhs):
        chi_q = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 1)
        want = to_cb(dims, oracle.dslash(dims, F, L, chi_q, 0), 0)
        assert rel_l2(decode(got[i], vh, prec), want) <= tol
    g.close()


def test_brick_order_in_solver(tmp_path, cuda_device):
    """A batched mixed-precision solve whose epilogue Dslash (with the fused
    <p, Ap> block partials) runs in XCD-brick order, and with the RHS split over
    the waves of a workgroup, converges to the oracle's true residual."""
    import torch
    dims = (16, 16, 16, 8)
    F, L = fields(dims, cfg_id=0, eps=0.3)
    g = make_gauge(dims, F, L)
    # FP32: the two RHS split over two waves of a workgroup (one RHS each);
    # FP64: both RHS in one wave
    for prec, shape in (("fp32", (1, 256, BRICK[0] | 1 << 24)), ("fp64", (2, 128, BRICK[0]))):
        assert force_shape(g, prec, 2, 1, shape, tmp_path / f"s{prec}.jsonl") == shape
        assert force_shape(g, prec, 2, 0, shape, tmp_path / f"s0{prec}.jsonl") == shape
    mass = 0.1
    srcs = synth.gaussian_source(dims, 1, 2, parity=0, index0=81)
    vh = synth.volume(dims) // 2
    b = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in srcs]))
    x = torch.zeros_like(b)
    rc, st = hisq().cg_solve(g, mass, 2, b, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc == 0, st
    xs = to_host(x).reshape(2, -1)
    for i in range(2):
        xi = from_cb(dims, decode(xs[i], vh, "fp64"), 0)
        assert oracle.true_residual(dims, F, L, mass, srcs[i], xi) <= 1e-10
    g.close()


def test_tuned_batched_solve_converges(cuda_device):
    import torch
    dims = (16, 8, 8, 8)
    F, L = fields(dims, cfg_id=0, eps=0.3)
    g = make_gauge(dims, F, L)
    hisq().autotune(g, "fp32", 3)
    mass = 0.1
    srcs = synth.gaussian_source(dims, 0, 3, parity=0, index0=80)
    vh = synth.volume(dims) // 2
    b = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in srcs]))
    x = torch.zeros_like(b)
    rc, st = hisq().cg_solve(g, mass, 3, b, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc == 0
    xs = to_host(x).reshape(3, -1)
    for i in range(3):
        xi = from_cb(dims, decode(xs[i], vh, "fp64"), 0)
        assert oracle.true_residual(dims, F, L, mass, srcs[i], xi) <= 1e-10
    g.close()
