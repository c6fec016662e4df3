"""HISQ link smearing (test infrastructure): the fat and Naik links of the
HISQ action (Follana et al., Phys. Rev. D 75 (2007) 054502; the action the
paper's code simulates, Sec. 1), built from thin links in plain FP64 numpy.

Definitions (unfolded links: no staggered phases, periodic gauge field):

* staple operator along nu, both orientations, applied to a field A of
  links in direction mu, transporting with links T:
      S_nu[A]_mu(x) = T_nu(x) A_mu(x+nu) T_nu(x+mu)^+
                    + T_nu(x-nu)^+ A_mu(x-nu) T_nu(x-nu+mu);
  the two-step (Lepage) form replaces T_nu(x) by T_nu(x) T_nu(x+nu) and the
  shift nu by 2 nu;
* fat7 smearing F[A, T]_mu = c1 A_mu + c3 sum_nu S_nu[A] + c5 sum_{nu,rho} S_rho[S_nu[A]]
  + c7 sum_{nu,rho,sigma} S_sigma[S_rho[S_nu[A]]] (+ cL sum_nu S2_nu[A]), every
  direction different from mu and from each other, every ordering summed;
  the product form prod_{nu != mu} (1 + delta_nu^2 / 4) gives c1 = 1/8,
  c3 = 1/16, c5 = 1/64 per ordered pair, c7 = 1/384 per ordered triple;
* level 1: V = F[U, U] with (1/8, 1/16, 1/64, 1/384), no Lepage term;
* U(3) projection: W = V (V^+ V)^(-1/2) (eigen-decomposition of V^+ V);
* level 2: X = F[W, W] with c1 = 1, c3 = 1/16, c5 = 1/64, c7 = 1/384 and the
  Lepage term cL = -1/8: two fat7 smearings carry twice the O(a^2) error of
  one, so the Lepage coefficient is twice the one-smearing value -1/16, and
  the one-link term takes 1/8 (fat7) + 6/8 (Lepage) + 1/8 (Naik) so that
  c1 sin p + c3 sin 3p has unit slope;
* Naik link: L_mu(x) = cN W_mu(x) W_mu(x+mu) W_mu(x+2mu), cN = -1/24 (no
  mass correction);
* phases and boundary signs folded at the end: X_mu(x) eta_mu(x) (-1 if
  mu = t and t + 1 >= Lt, antiperiodic), L_mu(x) eta_mu(x) (-1 if mu = t and
  t + 3 >= Lt).
Unit links give X = 9/8 and L = -1/24.  Shares no code with the HIP library.
"""

from __future__ import annotations

import itertools

import numpy as np

from .gauge import _roll

LEVEL1 = dict(c1=1 / 8, c3=1 / 16, c5=1 / 64, c7=1 / 384, cL=0.0)
LEVEL2 = dict(c1=1.0, c3=1 / 16, c5=1 / 64, c7=1 / 384, cL=-1 / 8)
NAIK = -1 / 24


def _dag(a):
    return a.conj().swapaxes(-1, -2)


def staple(dims, T, A, mu, nu, dist=1):
    """S_nu[A]_mu (dist 1) or its two-step Lepage form (dist 2); A is [V,3,3]."""
    Tn = T[:, nu]
    if dist == 1:
        up = Tn                                              # x -> x+nu
    else:
        up = Tn @ _roll(dims, Tn, nu, 1)                     # x -> x+2nu
    fwd = up @ _roll(dims, A, nu, dist) @ _dag(_roll(dims, up, mu, 1))
    down = _roll(dims, up, nu, -dist)                        # link from x-dist*nu to x
    bwd = _dag(down) @ _roll(dims, A, nu, -dist) @ _roll(dims, down, mu, 1)
    return fwd + bwd


def fat7(dims, A, T, c1, c3, c5, c7, cL=0.0):
    """The fat7 (+ Lepage) smearing of the links A with transport links T."""
    out = np.empty_like(A)
    for mu in range(4):
        others = [d for d in range(4) if d != mu]
        acc = c1 * A[:, mu]
        for nu in others:
            s1 = staple(dims, T, A[:, mu], mu, nu)
            acc = acc + c3 * s1
            if cL:
                acc = acc + cL * staple(dims, T, A[:, mu], mu, nu, dist=2)
            for rho in others:
                if rho == nu:
                    continue
                s2 = staple(dims, T, s1, mu, rho)
                acc = acc + c5 * s2
                for sig in others:
                    if sig in (nu, rho):
                        continue
                    acc = acc + c7 * staple(dims, T, s2, mu, sig)
        out[:, mu] = acc
    return out


def u3_project(V):
    """W = V (V^+ V)^(-1/2) for every 3x3 matrix of V."""
    Q = _dag(V) @ V
    w, E = np.linalg.eigh(Q)
    return V @ (E * (1.0 / np.sqrt(w))[..., None, :]) @ _dag(E)


def naik(dims, W, cN=NAIK):
    out = np.empty_like(W)
    for mu in range(4):
        out[:, mu] = cN * W[:, mu] @ _roll(dims, W[:, mu], mu, 1) @ _roll(dims, W[:, mu], mu, 2)
    return out


def fold(dims, X, L, antiperiodic_t=False):
    """Staggered phases eta_mu(x) and the time boundary signs folded into X and L."""
    Lx, Ly, Lz, Lt = dims
    c = np.array(list(itertools.product(range(Lt), range(Lz), range(Ly), range(Lx))))[:, ::-1]
    eta = np.ones((len(c), 4))
    eta[:, 1] = np.where(c[:, 0] & 1, -1.0, 1.0)
    eta[:, 2] = np.where((c[:, 0] + c[:, 1]) & 1, -1.0, 1.0)
    eta[:, 3] = np.where((c[:, 0] + c[:, 1] + c[:, 2]) & 1, -1.0, 1.0)
    sx, sl = eta.copy(), eta.copy()
    if antiperiodic_t:
        sx[:, 3] *= np.where(c[:, 3] + 1 >= Lt, -1.0, 1.0)
        sl[:, 3] *= np.where(c[:, 3] + 3 >= Lt, -1.0, 1.0)
    return X * sx[:, :, None, None], L * sl[:, :, None, None]


PATCH_RADIUS = 5


def hisq_smear_at(dims, U, site, antiperiodic_t=False):
    """(fat, long) [4,3,3] at one lexicographic site, phases folded, from the
    patch of thin links within PATCH_RADIUS steps of it in every direction.

    The fat link at x depends on W within two steps (the Lepage paths) and one
    step ahead along its own direction, and each W on U within one step (plus
    one ahead); the Naik link on W at x, x + mu, x + 2mu.  No path from x leaves
    the patch, so smearing the patch as a periodic lattice of extent 11 gives
    the full lattice's values at its centre (for any lattice extents)."""
    R = PATCH_RADIUS
    P = 2 * R + 1
    Lx, Ly, Lz, Lt = dims
    c0 = np.array([site % Lx, (site // Lx) % Ly, (site // (Lx * Ly)) % Lz, site // (Lx * Ly * Lz)])
    d = np.arange(-R, R + 1)
    t, z, y, x = np.meshgrid((c0[3] + d) % Lt, (c0[2] + d) % Lz, (c0[1] + d) % Ly, (c0[0] + d) % Lx,
                             indexing="ij")
    lex = (x + Lx * (y + Ly * (z + Lz * t))).ravel()
    pd = (P, P, P, P)
    Up = U[lex]
    W = u3_project(fat7(pd, Up, Up, **LEVEL1))
    X = fat7(pd, W, W, **LEVEL2)
    L = naik(pd, W)
    centre = R + P * (R + P * (R + P * R))
    # phases and boundary signs of the site's global coordinates
    eta = np.array([1.0, (-1.0) ** c0[0], (-1.0) ** (c0[0] + c0[1]), (-1.0) ** (c0[0] + c0[1] + c0[2])])
    sx, sl = eta.copy(), eta.copy()
    if antiperiodic_t:
        sx[3] *= -1.0 if c0[3] + 1 >= Lt else 1.0
        sl[3] *= -1.0 if c0[3] + 3 >= Lt else 1.0
    return X[centre] * sx[:, None, None], L[centre] * sl[:, None, None]


def hisq_smear(dims, U, antiperiodic_t=False, want_levels=False):
    """(fat, long) HISQ links from thin links U [V,4,3,3], phases folded; with
    want_levels also the level-1 V and the projected W (unfolded)."""
    V = fat7(dims, U, U, **LEVEL1)
    W = u3_project(V)
    X = fat7(dims, W, W, **LEVEL2)
    L = naik(dims, W)
    F, Lf = fold(dims, X, L, antiperiodic_t)
    return (F, Lf, V, W) if want_levels else (F, Lf)
