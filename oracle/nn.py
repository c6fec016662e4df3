"""FP64 reference of the gauge-covariant preconditioner network (test infrastructure).

A stack of linear, gauge-covariant layers on the full lattice (the L-CNN
construction of Favoni et al. 2022, used as a multigrid-free preconditioner
by Lehner and Wettig 2023).  Layer with C_in -> C_out complex channels:

    y_a(x) = sum_b [ W0_ab psi_b(x)
                     + sum_mu ( Wf_mu,ab U_mu(x)       psi_b(x + mu)
                              + Wb_mu,ab U_mu(x - mu)^+ psi_b(x - mu) ) ]

with complex weights and the thin links U (staggered phases and boundary
signs folded in, as for the operator).  There is no bias and no activation.
The network maps an even-site vector r to an even-site vector: r is embedded
in the full lattice with zeros on odd sites, passed through the layers
(channels 1 -> C -> ... -> 1) and the output is projected back to even sites.

Weights of one layer: complex array [9, C_out, C_in], path index
0 = identity, 1 + mu = forward hop along mu, 5 + mu = backward hop along mu.

Loss over a batch of pairs (A v_i, v_i):  L = (1/B) sum_i |N(A v_i) - v_i|^2 / |v_i|^2.
Gradients use the convention G(z) = dL/dRe z + i dL/dIm z.
"""

from __future__ import annotations

import numpy as np

NPATH = 9


def _roll(dims, a, mu, k):
    """a(x + k mu) for arrays indexed by lexicographic site first."""
    Lx, Ly, Lz, Lt = dims
    shaped = a.reshape(Lt, Lz, Ly, Lx, *a.shape[1:])
    return np.roll(shaped, -k, axis=3 - mu).reshape(a.shape)


def transport(dims, U, psi, path):
    """(T_path psi)(x) for psi of shape [V, 3] (or [V, C, 3])."""
    if path == 0:
        return psi.copy()
    if path <= 4:
        mu = path - 1
        nb = _roll(dims, psi, mu, +1)                      # psi(x + mu)
        return np.einsum("sab,s...b->s...a", U[:, mu], nb)
    mu = path - 5
    Ub = _roll(dims, U[:, mu], mu, -1)                     # U_mu(x - mu)
    nb = _roll(dims, psi, mu, -1)                          # psi(x - mu)
    return np.einsum("sba,s...b->s...a", Ub.conj(), nb)


def adjoint_path(path):
    """T_p^+ = T_{adjoint_path(p)}: forward and backward hops swap."""
    if path == 0:
        return 0
    return path + 4 if path <= 4 else path - 4


def layer_forward(dims, U, psi, W):
    """psi: [V, C_in, 3], W: [9, C_out, C_in] -> [V, C_out, 3]."""
    V = psi.shape[0]
    out = np.zeros((V, W.shape[1], 3), np.complex128)
    for p in range(NPATH):
        t = transport(dims, U, psi, p)                     # [V, C_in, 3]
        out += np.einsum("ab,sbc->sac", W[p], t)
    return out


def layer_backward(dims, U, psi, W, g):
    """Given G(y) = g [V, C_out, 3], return (G(psi) [V, C_in, 3], G(W) [9, C_out, C_in])."""
    gpsi = np.zeros_like(psi)
    gW = np.zeros_like(W)
    for p in range(NPATH):
        t = transport(dims, U, psi, p)
        gW[p] = np.einsum("sac,sbc->ab", g, t.conj())
        h = np.einsum("ab,sac->sbc", W[p].conj(), g)      # W^H applied to the gradient
        gpsi += transport(dims, U, h, adjoint_path(p))
    return gpsi, gW


def embed_even(dims, r_even_full):
    """[V, 3] vector (zero on odd sites) -> [V, 1, 3] first-layer input."""
    return r_even_full[:, None, :].copy()


def even_mask(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return (((x + y + z + t) & 1) == 0).ravel()


def forward(dims, U, weights, r):
    """Network output on even sites (zero on odd sites), r: [V, 3] even vector.
    Returns (out [V, 3], activations list)."""
    acts = [embed_even(dims, r)]
    for W in weights:
        acts.append(layer_forward(dims, U, acts[-1], W))
    out = acts[-1][:, 0, :].copy()
    out[~even_mask(dims)] = 0
    return out, acts


def loss_and_grad(dims, U, weights, pairs):
    """pairs: list of (Av, v), each [V, 3] even vectors.  Returns (L, [G(W_l)])."""
    B = len(pairs)
    grads = [np.zeros_like(W) for W in weights]
    L = 0.0
    em = even_mask(dims)
    for Av, v in pairs:
        out, acts = forward(dims, U, weights, Av)
        nv2 = float(np.vdot(v, v).real)
        d = out - v
        L += float(np.vdot(d, d).real) / nv2 / B
        g = (2.0 / (B * nv2)) * d                          # G(out) on even sites
        g[~em] = 0
        g = g[:, None, :]
        for l in range(len(weights) - 1, -1, -1):
            g, gW = layer_backward(dims, U, acts[l], weights[l], g)
            grads[l] += gW
    return L, grads


def init_weights(channels, rng, scale_identity=1.0, noise=1e-3):
    """Weights for channel counts e.g. [1, 8, 8, 1]: identity path of channel 0
    carries scale_identity through every layer, all other entries N(0, noise)."""
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = noise * (rng.standard_normal((NPATH, cout, cin)) + 1j * rng.standard_normal((NPATH, cout, cin)))
        W[0, 0, 0] += scale_identity
        ws.append(W)
    return ws


# --------------------------------------------------------------------------
# The function class of a two- or three-layer network.  Every path through
# three nearest-neighbour layers has 0, 1, 2 or 3 hops; from an even input
# only the 0- and 2-hop paths end on even sites, and a hop followed by its
# own reverse is the identity (unitary thin links).  So N restricted to even
# sites lies in the span of the identity and the 56 distinct transported
# two-hop paths T_b T_a, and the best loss any such network can reach on a
# set of pairs is a linear least-squares problem over those 57 features.

def two_hop_paths():
    """(first, second) path indices of the 56 distinct two-hop paths."""
    out = []
    for a in range(1, NPATH):
        for b in range(1, NPATH):
            if b == adjoint_path(a):
                continue
            out.append((a, b))
    return out


def two_hop_features(dims, U, r):
    """[57, V, 3]: r and T_b T_a r for every distinct two-hop path (a then b)."""
    first = {a: transport(dims, U, r, a) for a in range(1, NPATH)}
    feats = [r.copy()]
    for a, b in two_hop_paths():
        feats.append(transport(dims, U, first[a], b))
    return np.stack(feats)


def stencil_optimum(dims, U, pairs):
    """Least loss over the even-site span of the 57 features:
    min_c (1/B) sum_i |sum_k c_k f_k(A v_i) - v_i|^2 / |v_i|^2 (even sites).
    Returns (loss, c, scalar_loss) where scalar_loss is the optimum of c I alone."""
    em = even_mask(dims)
    rows, rhs = [], []
    for Av, v in pairs:
        nv = np.sqrt(float(np.vdot(v, v).real))
        f = two_hop_features(dims, U, Av)[:, em, :].reshape(57, -1)
        rows.append(f.T / nv)
        rhs.append(v[em].ravel() / nv)
    M = np.concatenate(rows)
    y = np.concatenate(rhs)
    c, *_ = np.linalg.lstsq(M, y, rcond=None)
    res = M @ c - y
    B = len(pairs)
    m0 = M[:, 0]
    c0 = np.vdot(m0, y) / np.vdot(m0, m0)
    r0 = m0 * c0 - y
    return float(np.vdot(res, res).real) / B, c, float(np.vdot(r0, r0).real) / B
