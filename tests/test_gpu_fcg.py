"""Flexible CG with the network preconditioner, checked by the FP64 oracle.

Whatever the network, the answer is defined without it: every solve must end
with a true relative residual |b - A x| / |b| <= 1e-10, which the oracle's own
operator recomputes on the host, and the solution must agree with the
oracle's CG solution within the conditioning bound.  Iteration counts are
reported, not matched (the network's effect on them is not unique).
"""

import numpy as np
import pytest

import oracle
from oracle import nn
import synth
from gpu_util import flush, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, to_cb

pytestmark = pytest.mark.gpu

TOL = 1e-10
RES_SLACK = 1.0  # the solvers stop at 0.9 tol: no slack for the oracle


@pytest.fixture(scope="module")
def lat(cuda_device):
    import torch
    dims = (8, 8, 8, 8)
    F, L, U = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    g = make_gauge(dims, F, L, precs=("fp64", "fp32"))
    hisq().gauge_set_thin(g, torch.from_numpy(np.ascontiguousarray(U)).cuda())
    yield dims, F, L, U, g
    g.close()


def make_net(g, channels, seed=0, noise=0.0, scale=1.0):
    ws = nn.init_weights(list(channels), np.random.default_rng(seed), scale_identity=1.0, noise=noise)
    w = np.concatenate([x.ravel() for x in ws])
    net = hisq().Net(g, channels, w)
    if scale != 1.0:
        w = net.get_weights()
        w[: 9 * channels[1] * channels[0]] *= scale  # first layer carries the scale
        net.set_weights(w)
    return net


def fcg(g, dims, mass, srcs, net, x0=None, **kw):
    import torch
    vh = synth.volume(dims) // 2
    n = len(srcs)
    b = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in srcs]))
    if x0 is None:
        x = torch.zeros_like(b)
    else:
        x = to_device(np.concatenate([encode(to_cb(dims, s, 0), "fp64") for s in x0]))
        kw["warm_start"] = 1
    prm = hisq().solver_params(precond=net, **kw)
    rc, st = hisq().cg_solve(g, mass, n, b, x, prm)
    xs = to_host(x).reshape(n, -1)
    return rc, st, [from_cb(dims, decode(xs[i], vh, "fp64"), 0) for i in range(n)]


def check_solution(dims, F, L, mass, b, x, st):
    assert st["true_residual"] <= TOL, st
    res = oracle.true_residual(dims, F, L, mass, b, x)
    assert res <= TOL * RES_SLACK, res
    xo, _, _, _ = oracle.cg(dims, F, L, mass, b, tol=1e-12)
    assert rel_l2(x, xo) <= 1e-7


@pytest.mark.parametrize("mass", [0.1, 0.02])
def test_fcg_scaled_identity(lat, mass):
    dims, F, L, U, g = lat
    net = make_net(g, (1, 8, 8, 1), scale=1.0 / (4 * mass * mass + 6.0))
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=7)[0]
    flush(f"fcg 8^4 m={mass} scaled identity")
    rc, st, (x,) = fcg(g, dims, mass, [b], net)
    assert rc == 0 and st[0]["fallback_used"] == 0, st
    assert st[0]["reliable_updates"] >= 1
    check_solution(dims, F, L, mass, b, x, st[0])
    net.close()


def test_fcg_untrained_random_network(lat):
    """A non-Hermitian, non-trained network: the flexible form must still converge."""
    dims, F, L, U, g = lat
    mass = 0.05
    net = make_net(g, (1, 8, 8, 1), seed=4, noise=0.3, scale=0.1)
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=8)[0]
    flush("fcg 8^4 random network")
    rc, st, (x,) = fcg(g, dims, mass, [b], net)
    assert rc in (0, 3), st
    check_solution(dims, F, L, mass, b, x, st[0])
    net.close()


def test_fcg_zero_network_falls_back(lat):
    """N = 0 makes every search direction vanish: breakdown, then plain FP64 CG."""
    dims, F, L, U, g = lat
    mass = 0.1
    net = hisq().Net(g, (1, 2, 1), np.zeros(9 * 2 + 9 * 2, np.complex128))
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=9)[0]
    flush("fcg 8^4 zero network -> fallback")
    rc, st, (x,) = fcg(g, dims, mass, [b], net)
    assert rc == 3 and st[0]["status"] == 3 and st[0]["fallback_used"] == 1, st
    check_solution(dims, F, L, mass, b, x, st[0])
    # without the fallback the breakdown is reported as such
    rc2, st2, _ = fcg(g, dims, mass, [b], net, fallback=0)
    assert rc2 == 2 and st2[0]["fallback_used"] == 0, st2
    net.close()


def test_fcg_two_rhs_and_warm_start(lat):
    dims, F, L, U, g = lat
    mass = 0.05
    net = make_net(g, (1, 4, 1), scale=1.0 / 6.0)
    bs = synth.gaussian_source(dims, 99, 2, parity=0, index0=10)
    flush("fcg 8^4 two rhs")
    rc, st, xs = fcg(g, dims, mass, list(bs), net)
    assert rc == 0, st
    for b, x, s in zip(bs, xs, st):
        check_solution(dims, F, L, mass, b, x, s)
    # restarting from the converged solutions needs (almost) no iterations
    rc, st2, xs2 = fcg(g, dims, mass, list(bs), net, x0=xs)
    assert rc == 0 and all(s["iterations"] <= 10 for s in st2), st2
    for b, x, s in zip(bs, xs2, st2):
        check_solution(dims, F, L, mass, b, x, s)
    net.close()


def test_fcg_iteration_cap(lat):
    dims, F, L, U, g = lat
    net = make_net(g, (1, 2, 1), scale=1.0 / 6.0)
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=11)[0]
    rc, st, _ = fcg(g, dims, 0.01, [b], net, max_iter=20, fallback=0)
    assert rc == 1 and st[0]["status"] == 1 and st[0]["iterations"] <= 20 + 10, st
    net.close()


def test_mixed_cg_reports_no_fallback(lat):
    """The plain mixed solve reports fallback_used = 0 when it converges alone."""
    import torch
    dims, F, L, U, g = lat
    b = to_device(encode(to_cb(dims, synth.gaussian_source(dims, 99, 1, parity=0, index0=12)[0], 0), "fp64"))
    x = torch.zeros_like(b)
    rc, st = hisq().cg_solve(g, 0.1, 1, b, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc == 0 and st[0]["fallback_used"] == 0


def test_multishift_rejects_network(lat):
    import torch
    dims, F, L, U, g = lat
    net = make_net(g, (1, 2, 1))
    b = to_device(encode(to_cb(dims, synth.gaussian_source(dims, 99, 1, parity=0)[0], 0), "fp64"))
    x = torch.zeros(2, *b.shape, dtype=b.dtype, device=b.device)
    with pytest.raises(Exception):
        hisq().multishift_cg(g, 0.1, [0.0, 0.1], b, x, hisq().solver_params(precond=net))
    net.close()


def test_training_reaches_the_stencil_optimum_without_a_cg_gain(lat):
    """What training buys, against two fixed points the oracle computes on the same
    pairs: the best multiple of the identity and the best even-site stencil of the
    network's function class (identity plus the 56 two-hop paths, least squares).
    Training must close the gap between them from far above (the start is the
    identity / 6, loss 3.4).  The solve is then pinned on both sides: flexible CG
    with the starting network (a multiple of the identity, plus 1e-3 noise)
    must take plain CG's iteration count within 5 % (it iterates in FP32), and
    with the trained network at most 1.25 times it.
    Measured: 2119 (trained) against 1788 (plain), 1.19 times; the oracle's own
    FP64 flexible CG with the exact least-squares stencil needs 2056 against
    1783.  The network's optimum does not precondition A, so no gain is
    asserted: the test guards the training and the solve cost."""
    import torch
    dims, F, L, U, g = lat
    mass, B = 0.02, 16
    vh = synth.volume(dims) // 2
    vs = synth.gaussian_source(dims, 99, B, parity=0, index0=200)
    avs = [oracle.normal_op(dims, F, L, mass, v) for v in vs]
    av_raw = np.concatenate([encode(to_cb(dims, a, 0), "fp32") for a in avs])
    v_raw = np.concatenate([encode(to_cb(dims, v, 0), "fp32") for v in vs])
    q = lambda raw, i: from_cb(dims, decode(raw[i * 24 * vh:(i + 1) * 24 * vh], vh, "fp32"), 0)  # noqa: E731
    best, _, scalar = nn.stencil_optimum(dims, U, [(q(av_raw, i), q(v_raw, i)) for i in range(B)])
    start = make_net(g, (1, 8, 8, 1), seed=2, noise=1e-3, scale=1.0 / (4 * mass * mass + 6.0))
    net = make_net(g, (1, 8, 8, 1), seed=2, noise=1e-3, scale=1.0 / (4 * mass * mass + 6.0))
    av_d, v_d = to_device(av_raw), to_device(v_raw)
    l0 = net.loss_grad(B, av_d, v_d, want_grad=False)[0]
    for _ in range(400):
        net.train_step(B, av_d, v_d, 3e-3)
    l1 = net.loss_grad(B, av_d, v_d, want_grad=False)[0]
    closed = (scalar - l1) / (scalar - best)
    flush(f"loss start {l0:.4f} trained {l1:.5f}; oracle optimum: scalar {scalar:.5f} stencil {best:.5f}; "
          f"gap closed {closed:.2f}")
    assert l1 >= best * (1 - 1e-3)
    assert closed >= 0.9, closed
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=300)[0]
    rc, st, (x,) = fcg(g, dims, mass, [b], net)
    assert rc == 0, st
    check_solution(dims, F, L, mass, b, x, st[0])
    rc0, st0, (x0,) = fcg(g, dims, mass, [b], start)
    assert rc0 == 0, st0
    check_solution(dims, F, L, mass, b, x0, st0[0])
    bd = to_device(encode(to_cb(dims, b, 0), "fp64"))
    xd = torch.zeros_like(bd)
    rc2, st2 = hisq().cg_solve(g, mass, 1, bd, xd, hisq().solver_params())
    assert rc2 == 0
    it_t, it_0, it_p = st[0]["iterations"], st0[0]["iterations"], st2[0]["iterations"]
    flush(f"iterations: flexible CG + trained network {it_t}, + starting network {it_0}, plain CG {it_p}")
    assert abs(it_0 - it_p) <= 0.05 * it_p, (it_0, it_p)
    assert it_t <= 1.25 * it_p, (it_t, it_p)
    net.close()
    start.close()


def test_checkpoint_restores_the_network(lat, tmp_path):
    """Weights saved after training and loaded into a fresh network give the
    same preconditioner output bit for bit."""
    import torch
    from paper_2111_10354_amd import checkpoint
    dims, F, L, U, g = lat
    net = make_net(g, (1, 4, 1), seed=3, noise=0.2, scale=0.2)
    vs = synth.gaussian_source(dims, 99, 2, parity=0, index0=400)
    raw = to_device(np.concatenate([encode(to_cb(dims, v, 0), "fp32") for v in vs]))
    for _ in range(3):
        net.train_step(2, raw, raw, 1e-3)
    checkpoint.save(str(tmp_path / "n"), net.get_weights(), (1, 4, 1), dims=dims, steps=3)
    w, h = checkpoint.load(str(tmp_path / "n"))
    net2 = hisq().Net(g, tuple(h["channels"]), w)
    half = raw.numel() // 2
    a, b = torch.empty_like(raw[:half]), torch.empty_like(raw[:half])
    hisq().precond_apply(g, net, raw[:half], a)
    hisq().precond_apply(g, net2, raw[:half], b)
    assert torch.equal(a, b)
    net.close()
    net2.close()


def test_nan_network_falls_back(lat):
    """A network that returns NaN (corrupted weights) breaks the flexible CG,
    which hands the solve to plain FP64 CG."""
    dims, F, L, U, g = lat
    net = make_net(g, (1, 2, 1))
    w = net.get_weights()
    w[3] = np.nan
    net.set_weights(w)
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=13)[0]
    rc, st, (x,) = fcg(g, dims, 0.1, [b], net)
    assert rc == 3 and st[0]["fallback_used"] == 1, st
    check_solution(dims, F, L, 0.1, b, x, st[0])
    net.close()


def test_solver_failure_statuses(lat):
    """Host-forced failures end every kernel normally and come back as statuses."""
    import torch
    dims, F, L, U, g = lat
    b = synth.gaussian_source(dims, 99, 1, parity=0, index0=14)[0]
    bd = to_device(encode(to_cb(dims, b, 0), "fp64"))
    x = torch.zeros_like(bd)
    rc, st = hisq().cg_solve(g, 0.1, 1, bd, x, hisq().solver_params(max_iter=1))
    assert rc == 1 and st[0]["status"] == 1 and st[0]["iterations"] <= 1
    bad = bd.clone()
    bad.view(torch.float64)[5] = float("nan")
    x.zero_()
    rc, st = hisq().cg_solve(g, 0.1, 1, bad, x, hisq().solver_params(sloppy_prec="fp32"))
    assert rc in (1, 2) and st[0]["status"] in (1, 2), st
