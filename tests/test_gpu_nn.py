"""GPU network kernels against the FP64 network oracle (oracle/nn.py).

The channel mixing runs on BF16 matrix cores with FP32 accumulation, so the
bars are BF16-sized: forward rel. L2 <= 3e-2, loss <= 2e-2 relative, gradient
rel. L2 <= 5e-2 (BF16 has an 8-bit significand: 2^-9 relative rounding per
operand, a few layers and ~150-term sums).
"""

import numpy as np
import pytest

import oracle
from oracle import gauge, nn
import synth
from gpu_util import hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, to_cb

pytestmark = pytest.mark.gpu


def setup(dims, channels, seed=0, noise=0.2, scale_identity=0.7):
    import torch
    F, L, U = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    U = np.ascontiguousarray(U)
    g = make_gauge(dims, F, L, precs=("fp64", "fp32"))
    hisq().gauge_set_thin(g, torch.from_numpy(U).cuda())
    rng = np.random.default_rng(seed)
    ws = nn.init_weights(list(channels), rng, scale_identity=scale_identity, noise=noise)
    net = hisq().Net(g, channels, np.concatenate([w.ravel() for w in ws]))
    return g, net, F, L, U, ws


def apply_gpu(g, net, dims, r):
    import torch
    vh = synth.volume(dims) // 2
    inp = to_device(encode(to_cb(dims, r, 0), "fp32"))
    out = torch.empty_like(inp)
    hisq().precond_apply(g, net, inp, out)
    return from_cb(dims, decode(to_host(out), vh, "fp32"), 0), \
        from_cb(dims, decode(encode(to_cb(dims, r, 0), "fp32"), vh, "fp32"), 0)


@pytest.mark.parametrize("dims,channels", [((4, 4, 4, 4), (1, 8, 8, 1)), ((6, 4, 4, 8), (1, 4, 1)),
                                           ((8, 8, 8, 8), (1, 8, 8, 1)), ((4, 6, 4, 4), (1, 2, 8, 1)),
                                           ((6, 6, 6, 6), (1, 3, 5, 1)), ((6, 4, 6, 6), (1, 8, 8, 8, 1))])
def test_forward_matches_oracle(cuda_device, dims, channels):
    g, net, F, L, U, ws = setup(dims, channels)
    r = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    got, rq = apply_gpu(g, net, dims, r)
    want, _ = nn.forward(dims, U, ws, rq)
    assert rel_l2(got, want) <= 3e-2, rel_l2(got, want)
    net.close()
    g.close()


def test_identity_network(cuda_device):
    dims = (4, 4, 4, 6)
    g, net, F, L, U, ws = setup(dims, (1, 8, 8, 1), noise=0.0, scale_identity=1.0)
    r = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    got, rq = apply_gpu(g, net, dims, r)
    assert rel_l2(got, rq) <= 4e-3
    net.close()
    g.close()


def test_gauge_covariance(cuda_device):
    import torch
    dims = (4, 4, 4, 4)
    g, net, F, L, U, ws = setup(dims, (1, 4, 1), noise=0.3)
    gt = synth.random_gauge_transform(dims)
    r = synth.gaussian_source(dims, 99, 1, parity=0)[0]
    out, rq = apply_gpu(g, net, dims, r)
    Ug = np.ascontiguousarray(gauge.transform_links(dims, U, gt, hop=1))
    hisq().gauge_set_thin(g, torch.from_numpy(Ug).cuda())
    outg, _ = apply_gpu(g, net, dims, gauge.transform_vector(gt, rq))
    assert rel_l2(outg, gauge.transform_vector(gt, out)) <= 3e-2
    net.close()
    g.close()


@pytest.mark.parametrize("channels", [(1, 8, 8, 1), (1, 2, 1), (1, 3, 7, 1)])
def test_loss_and_gradient_match_oracle(cuda_device, channels):
    dims = (4, 4, 4, 6)
    g, net, F, L, U, ws = setup(dims, channels, seed=3, noise=0.3, scale_identity=0.5)
    mass = 0.3
    vs = synth.gaussian_source(dims, 99, 3, parity=0, index0=40)
    vh = synth.volume(dims) // 2
    avs = [oracle.normal_op(dims, F, L, mass, v) for v in vs]
    av_raw = np.concatenate([encode(to_cb(dims, a, 0), "fp32") for a in avs])
    v_raw = np.concatenate([encode(to_cb(dims, v, 0), "fp32") for v in vs])
    loss, grad = net.loss_grad(3, to_device(av_raw), to_device(v_raw))
    q = lambda raw, i: from_cb(dims, decode(raw[i * 24 * vh:(i + 1) * 24 * vh], vh, "fp32"), 0)  # noqa: E731
    pairs = [(q(av_raw, i), q(v_raw, i)) for i in range(3)]
    L0, grads = nn.loss_and_grad(dims, U, ws, pairs)
    assert abs(loss - L0) <= 2e-2 * L0, (loss, L0)
    want = np.concatenate([gw.ravel() for gw in grads])
    assert rel_l2(grad, want) <= 5e-2, rel_l2(grad, want)
    net.close()
    g.close()


def test_training_reduces_loss(cuda_device):
    dims = (8, 8, 8, 8)
    g, net, F, L, U, ws = setup(dims, (1, 8, 8, 1), seed=5, noise=1e-3, scale_identity=1.0)
    import torch
    mass = 0.2
    B = 8
    vs = synth.gaussian_source(dims, 99, B, parity=0, index0=100)
    vh = synth.volume(dims) // 2
    v_raw = to_device(np.concatenate([encode(to_cb(dims, v, 0), "fp32") for v in vs]))
    av = torch.empty_like(v_raw)
    t = torch.empty_like(v_raw)
    hisq().dslash_multi_rhs(g, 1, "fp32", B, v_raw, t)
    hisq().dslash_multi_rhs(g, 0, "fp32", B, t, av, diag=[4 * mass * mass] * B, y=v_raw)
    # start from N = (1 / mean diagonal) * identity
    w = net.get_weights()
    w[0] = 1.0 / (4 * mass * mass + 16 * 0.4)
    net.set_weights(w)
    l0 = net.loss_grad(B, av, v_raw, want_grad=False)[0]
    losses = [net.train_step(B, av, v_raw, 3e-3) for _ in range(40)]
    l1 = net.loss_grad(B, av, v_raw, want_grad=False)[0]
    assert np.isfinite(l1) and l1 < 0.8 * l0, (l0, l1, losses[::8])
    net.close()
    g.close()


def test_thin_links_out_of_fp16_range_rejected(cuda_device):
    import torch
    dims = (4, 4, 4, 4)
    F, L, U = synth.hisq_links(dims, 99, 0.5, want_thin=True)
    g = make_gauge(dims, F, L, precs=("fp64",))
    bad = np.array(U)
    bad[5, 2, 1, 1] = 1e6
    with pytest.raises(Exception):
        hisq().gauge_set_thin(g, torch.from_numpy(bad).cuda())
    hisq().gauge_set_thin(g, torch.from_numpy(np.ascontiguousarray(U)).cuda())
    g.close()
