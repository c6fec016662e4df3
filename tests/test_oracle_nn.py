"""Pins of the FP64 network oracle (oracle/nn.py).

* identity weights give the identity map on even vectors;
* one layer with forward weights +1 and backward weights -1 is the naive
  staggered operator, i.e. the (separately pinned) Dslash oracle with fat
  links = thin links and no Naik term;
* gauge covariance and linearity of the network;
* the analytic gradient against central finite differences of the loss, on
  the real and on the imaginary part of sampled weights of every layer;
* the function class: a three-layer network's even-site output is fitted
  exactly by the identity plus the 56 two-hop paths, so the least-squares
  optimum over those features bounds the loss of every such network.
"""

import numpy as np
import pytest

import oracle
from oracle import gauge, nn
import synth


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 4, 6)
    _, _, U = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    return dims, np.ascontiguousarray(U)


def _even(dims, k=0):
    return synth.gaussian_source(dims, 99, 1, parity=0, index0=k)[0]


def test_identity_weights(small):
    dims, U = small
    rng = np.random.default_rng(0)
    ws = nn.init_weights([1, 8, 8, 1], rng, scale_identity=1.0, noise=0.0)
    r = _even(dims)
    out, _ = nn.forward(dims, U, ws, r)
    assert np.allclose(out, r, atol=1e-15)


def test_naive_staggered_special_case(small):
    dims, U = small
    W = np.zeros((nn.NPATH, 1, 1), complex)
    W[1:5] = 1.0
    W[5:9] = -1.0
    r = _even(dims)
    y = nn.layer_forward(dims, U, r[:, None, :], W)[:, 0, :]
    want = oracle.dslash(dims, U, np.zeros_like(U), r, 1)
    assert np.abs(y - want).max() < 1e-13


def test_gauge_covariance_and_linearity(small):
    dims, U = small
    rng = np.random.default_rng(1)
    ws = nn.init_weights([1, 3, 3, 1], rng, noise=0.3)
    r1, r2 = _even(dims, 1), _even(dims, 2)
    g = synth.random_gauge_transform(dims)
    Ug = gauge.transform_links(dims, U, g, hop=1)
    out, _ = nn.forward(dims, U, ws, r1)
    outg, _ = nn.forward(dims, Ug, ws, gauge.transform_vector(g, r1))
    assert np.abs(outg - gauge.transform_vector(g, out)).max() < 1e-13 * np.abs(out).max()
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    lhs, _ = nn.forward(dims, U, ws, a * r1 + b * r2)
    o2, _ = nn.forward(dims, U, ws, r2)
    assert np.abs(lhs - (a * out + b * o2)).max() < 1e-12 * np.abs(lhs).max()


def test_gradient_matches_finite_differences(small):
    dims, U = small
    rng = np.random.default_rng(2)
    ws = nn.init_weights([1, 3, 2, 1], rng, scale_identity=0.5, noise=0.3)
    # pairs (A v, v) with the fat/long field of the same lattice
    F, L = synth.hisq_links(dims, 99, 0.5)
    pairs = []
    for k in range(2):
        v = _even(dims, 10 + k)
        pairs.append((oracle.normal_op(dims, F, L, 0.3, v), v))
    L0, grads = nn.loss_and_grad(dims, U, ws, pairs)
    h = 1e-6
    for li in range(len(ws)):
        for _ in range(3):
            p, a, b = (rng.integers(0, s) for s in ws[li].shape)
            for unit in (1.0, 1j):
                wp = [w.copy() for w in ws]
                wm = [w.copy() for w in ws]
                wp[li][p, a, b] += h * unit
                wm[li][p, a, b] -= h * unit
                fd = (nn.loss_and_grad(dims, U, wp, pairs)[0] - nn.loss_and_grad(dims, U, wm, pairs)[0]) / (2 * h)
                an = grads[li][p, a, b].real if unit == 1.0 else grads[li][p, a, b].imag
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (li, p, a, b, unit, fd, an)


def test_adjoint_paths_are_adjoints(small):
    dims, U = small
    x = synth.gaussian_source(dims, 99, 1, parity=0, index0=5)[0] + synth.gaussian_source(dims, 99, 1, parity=1)[0]
    y = synth.gaussian_source(dims, 99, 1, parity=1, index0=6)[0] + synth.gaussian_source(dims, 99, 1, parity=0,
                                                                                            index0=7)[0]
    for p in range(nn.NPATH):
        lhs = np.vdot(y, nn.transport(dims, U, x, p))
        rhs = np.vdot(nn.transport(dims, U, y, nn.adjoint_path(p)), x)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_three_layer_networks_span_two_hop_stencils(small):
    """Any three-layer network restricted to even sites is a combination of the
    identity and the 56 two-hop paths: fitting its outputs is exact."""
    dims, U = small
    rng = np.random.default_rng(11)
    ws = nn.init_weights([1, 3, 2, 1], rng, scale_identity=0.7, noise=0.4)
    pairs = []
    for k in range(3):
        w = _even(dims, 20 + k)
        pairs.append((w, nn.forward(dims, U, ws, w)[0]))
    loss, c, scalar = nn.stencil_optimum(dims, U, pairs)
    assert loss < 1e-24, loss
    assert scalar > 1e-3
    # one layer reaches only the identity on even sites (a single hop lands on odd ones)
    ws1 = nn.init_weights([1, 1], rng, scale_identity=0.7, noise=0.4)
    w = _even(dims, 30)
    out = nn.forward(dims, U, ws1, w)[0]
    coef = np.vdot(w, out) / np.vdot(w, w)
    assert np.linalg.norm(out - coef * w) < 1e-12 * np.linalg.norm(out)


def test_stencil_optimum_bounds_any_network(small):
    dims, U = small
    F, L, _ = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    mass = 0.2
    pairs = []
    for k in range(3):
        v = _even(dims, 40 + k)
        pairs.append((oracle.normal_op(dims, F, L, mass, v), v))
    best, c, scalar = nn.stencil_optimum(dims, U, pairs)
    assert best <= scalar
    rng = np.random.default_rng(5)
    for noise in (0.0, 0.05, 0.3):
        ws = nn.init_weights([1, 4, 4, 1], rng, scale_identity=0.1, noise=noise)
        Lnet, _ = nn.loss_and_grad(dims, U, ws, pairs)
        assert Lnet >= best * (1 - 1e-12)
