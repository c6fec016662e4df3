"""Dense-matrix form of the operator on tiny lattices, and the free-field spectrum.

Test infrastructure (see the package docstring).  Pure-Python site loops: only
meant for lattices of a few hundred sites (4^4 gives 768 x 768).
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def _lex(dims, c):
    Lx, Ly, Lz, _ = dims
    return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))


def dense_dslash(dims, fat, lng) -> np.ndarray:
    """The full-lattice operator as a (3V, 3V) matrix, entry by entry from
    (D chi)(x) = sum_mu [F_mu(x) chi(x+mu) - F_mu(x-mu)^+ chi(x-mu)
                         + L_mu(x) chi(x+3mu) - L_mu(x-3mu)^+ chi(x-3mu)]
    (phases folded into F and L).  Hops that land on the same site add up."""
    V = int(np.prod(dims))
    D = np.zeros((3 * V, 3 * V), np.complex128)
    for c in itertools.product(*[range(L) for L in dims]):
        c = (c[0], c[1], c[2], c[3])
        s = _lex(dims, c)
        for mu in range(4):
            for k, U in ((1, fat), (3, lng)):
                fw = list(c)
                fw[mu] = (c[mu] + k) % dims[mu]
                bw = list(c)
                bw[mu] = (c[mu] - k) % dims[mu]
                f, b = _lex(dims, fw), _lex(dims, bw)
                D[3 * s:3 * s + 3, 3 * f:3 * f + 3] += U[s, mu]
                D[3 * s:3 * s + 3, 3 * b:3 * b + 3] -= U[b, mu].conj().T
    return D


def parity_index(dims, parity: int) -> np.ndarray:
    """Component indices (3*site + colour) of the sites of one parity, site-ordered."""
    V = int(np.prod(dims))
    Lx, Ly, Lz, _ = dims
    s = np.arange(V)
    x = s % Lx
    y = (s // Lx) % Ly
    z = (s // (Lx * Ly)) % Lz
    t = s // (Lx * Ly * Lz)
    sites = s[((x + y + z + t) & 1) == parity]
    return (3 * sites[:, None] + np.arange(3)[None, :]).ravel()


def dense_normal_op(dims, fat, lng, mass: float, sigma: float = 0.0) -> np.ndarray:
    """A_ee = (D^+ D)_ee + 4 m^2 + sigma built from the dense D (not from -D_eo D_oe)."""
    D = dense_dslash(dims, fat, lng)
    e = parity_index(dims, 0)
    DtD = D.conj().T @ D
    return DtD[np.ix_(e, e)] + (4 * mass * mass + sigma) * np.eye(len(e))


def free_field_eigenvalue(p, mass: float, c1: float, c3: float) -> float:
    """Eigenvalue of A on the even-site plane wave of momentum p (free field):
    4 [m^2 + sum_mu (c1 sin p_mu + c3 sin 3 p_mu)^2]."""
    p = np.asarray(p, float)
    return 4.0 * (mass ** 2 + float(np.sum((c1 * np.sin(p) + c3 * np.sin(3 * p)) ** 2)))


def free_field_spectrum(dims, mass: float, c1: float, c3: float, antiperiodic_t: bool = False):
    """Sorted eigenvalues of the full-lattice D^+D + 4m^2 for the free field:
    one value per lattice momentum, each with colour multiplicity 3."""
    axes = []
    for mu, L in enumerate(dims):
        if mu == 3 and antiperiodic_t:
            axes.append([(2 * n + 1) * math.pi / L for n in range(L)])
        else:
            axes.append([2 * math.pi * n / L for n in range(L)])
    vals = [free_field_eigenvalue(p, mass, c1, c3) for p in itertools.product(*axes)]
    return np.sort(np.repeat(vals, 3))
