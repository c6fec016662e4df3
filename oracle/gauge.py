"""Gauge transformations and the plaquette (test infrastructure).

The plaquette follows the functor example printed in the paper (Sec. 2,
Listing 1): for every site, the sum over mu < nu of the real trace of the
closed 1x1 path U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+.
"""

from __future__ import annotations

import numpy as np


def _roll(dims, a, mu, k):
    """a(x + k mu) for an array indexed by lexicographic site first."""
    Lx, Ly, Lz, Lt = dims
    shaped = a.reshape(Lt, Lz, Ly, Lx, *a.shape[1:])
    axis = 3 - mu
    return np.roll(shaped, -k, axis=axis).reshape(a.shape)


def transform_links(dims, U, g, hop: int = 1):
    """U_mu(x) -> g(x) U_mu(x) g(x + hop*mu)^+ for links spanning `hop` sites."""
    out = np.empty_like(U)
    for mu in range(4):
        gf = _roll(dims, g, mu, hop)
        out[:, mu] = g @ U[:, mu] @ gf.conj().transpose(0, 2, 1)
    return out


def transform_vector(g, v):
    """chi(x) -> g(x) chi(x)."""
    return np.einsum("sab,sb->sa", g, v)


def plaquette_per_site(dims, U) -> np.ndarray:
    out = np.zeros(U.shape[0])
    for nu in range(1, 4):
        for mu in range(nu):
            Unu_xmu = _roll(dims, U[:, nu], mu, 1)
            Umu_xnu = _roll(dims, U[:, mu], nu, 1)
            P = U[:, mu] @ Unu_xmu @ Umu_xnu.conj().transpose(0, 2, 1) @ U[:, nu].conj().transpose(0, 2, 1)
            out += np.real(np.trace(P, axis1=1, axis2=2))
    return out
