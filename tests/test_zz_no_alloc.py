"""hisq_dslash_multi_rhs_noalloc, the no-allocation form of the multi-RHS
Dslash with the (A + sigma_i) epilogue, through the C ABI: its output equals
hisq_dslash_multi_rhs's bit for bit and the FP64 oracle's within the parity
tolerances, on two calls in a row (the second smaller), and it allocates no
device memory."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import fields, hisq, make_gauge, to_device, to_host
from layout import decode, encode, from_cb, rel_l2, spinor_nbytes, to_cb

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 2e-6, "fp16s": 4e-3}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s"])
def test_noalloc_matches_multi_rhs_and_oracle(cuda_device, prec):
    import torch
    H = hisq()
    dims = (10, 6, 4, 8)          # Vh = 960: several tiles and a ragged tail
    F, L = fields(dims)
    g = make_gauge(dims, F, L)
    vh = synth.volume(dims) // 2
    nb = spinor_nbytes(prec, vh)
    mass = 0.1
    bytes0 = g.device_bytes()
    for call, (n, idx) in enumerate(((6, 70), (2, 90))):   # the second call is smaller
        print(f"noalloc {prec} call {call}: nrhs {n}", flush=True)
        sig = [0.01 * (k + 1) * (call + 1) for k in range(n)]
        diag = [4 * mass * mass + v for v in sig]
        ys = synth.gaussian_source(dims, 99, n, parity=0, index0=idx)
        raw = np.concatenate([encode(to_cb(dims, v, 0), prec) for v in ys])
        y = to_device(raw)
        t = torch.empty(n * nb, dtype=torch.uint8, device="cuda")
        H.dslash_multi_rhs_noalloc(g, 1, prec, n, y, t)
        t_ref = torch.empty_like(t)
        H.dslash_multi_rhs(g, 1, prec, n, y, t_ref)
        a = torch.empty_like(t)
        b = torch.empty_like(t)
        H.dslash_multi_rhs_noalloc(g, 0, prec, n, t, a, diag=diag, y=y)
        H.dslash_multi_rhs(g, 0, prec, n, t, b, diag=diag, y=y)
        ta, tr, ga, gb = to_host(t), to_host(t_ref), to_host(a), to_host(b)
        assert np.array_equal(ta, tr)
        assert np.array_equal(ga, gb)
        for i in range(n):
            yq = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, prec), 0)
            want = to_cb(dims, oracle.normal_op(dims, F, L, mass, yq, sigma=sig[i]), 0)
            assert rel_l2(decode(ga[i * nb:(i + 1) * nb], vh, prec), want) <= TOL[prec], (call, i)
    assert g.device_bytes() == bytes0
    g.close()


def test_noalloc_needs_no_handle_buffer_and_rejects_oversize(cuda_device):
    """80 right-hand sides with coefficients: more than the handle's own
    coefficient buffer holds, which hisq_dslash_multi_rhs would grow; the
    no-allocation form leaves the handle's device memory as it was.  Beyond
    HISQ_NOALLOC_MAX_RHS it refuses before any launch."""
    import torch
    H = hisq()
    dims = (4, 4, 4, 4)
    F, L = fields(dims)
    g = make_gauge(dims, F, L, precs=("fp64",))
    vh = synth.volume(dims) // 2
    nb = spinor_nbytes("fp64", vh)
    mass = 0.2
    n = 80
    ys = synth.gaussian_source(dims, 98, n, parity=0)
    raw = np.concatenate([encode(to_cb(dims, v, 0), "fp64") for v in ys])
    y = to_device(raw)
    t = torch.empty(n * nb, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(t)
    sig = np.linspace(0.0, 1.0, n)
    before = g.device_bytes()
    H.dslash_multi_rhs_noalloc(g, 1, "fp64", n, y, t)
    H.dslash_multi_rhs_noalloc(g, 0, "fp64", n, t, out, diag=list(4 * mass * mass + sig), y=y)
    got = to_host(out)
    assert g.device_bytes() == before
    for i in (0, 41, n - 1):
        yq = from_cb(dims, decode(raw[i * nb:(i + 1) * nb], vh, "fp64"), 0)
        want = to_cb(dims, oracle.normal_op(dims, F, L, mass, yq, sigma=float(sig[i])), 0)
        assert rel_l2(decode(got[i * nb:(i + 1) * nb], vh, "fp64"), want) <= 1e-13
    big = 4097
    assert big > 4096
    bufs = [torch.zeros(big * nb, dtype=torch.uint8, device="cuda") for _ in range(3)]
    with pytest.raises(H.HisqError) as e:
        H.dslash_multi_rhs_noalloc(g, 0, "fp64", big, bufs[0], bufs[1], diag=[1.0] * big, y=bufs[2])
    assert e.value.code == H.ERR_INVALID and "HISQ_NOALLOC_MAX_RHS" in H.last_error()
    g.close()
