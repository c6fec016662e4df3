"""Rational functions of the even-site normal operator A (test infrastructure).

What a rational-approximation solver must return, written from definitions:
* ``rational_apply``: alpha_0 b + sum_k alpha_k (A + sigma_k)^-1 b with every
  shifted system solved by its own plain FP64 CG (the definition of the
  partial-fraction sum; the multi-shift recurrence is not used);
* ``dense_power``: A^p b exactly, from the eigen-decomposition of the dense A
  on a tiny lattice;
* ``zolotarev_inv_sqrt``: Zolotarev's optimal rational approximation of
  x^(-1/2) on [lmin, lmax] (minimax relative error), built from the Jacobi
  elliptic functions of scipy: with k'^2 = 1 - lmin/lmax and K' = K(k'),
  c_l = sn^2 / cn^2 (l K' / (2n + 1)), l = 1..2n, and
  r(x) = D prod_l (x + c_{2l}) / (x + c_{2l-1}) on [1, lmax/lmin], D centring
  the relative error; then partial fractions and rescaling to [lmin, lmax];
* ``relative_error_extrema``: the alternation set of the relative error
  x^(-p) r(x) - 1 on a fine logarithmic grid (p = -1/2 by default; each
  interior extremum read off the parabola through its grid triple), for the
  alternation test: a best approximation of type (n, n) has 2n + 2
  alternating extrema of equal size (Chebyshev).  This is the definition of
  the minimax approximation and the pin of any construction of one, for every
  power; the error is evaluated in extended precision, because for positive
  powers the partial fractions cancel against alpha_0 near x = 0, and
  neighbouring extrema of one sign (one flat peak split by rounding) count
  once.
* ``minimax_bruteforce``: the definition minimised directly for tiny pole
  counts - the largest relative error of c prod (x + z_i) / (x + q_i) against
  x^p over a logarithmic grid, minimised over (log c, log z, log q) through
  smooth L_q norms of growing q and a final Nelder-Mead on the maximum; for
  one and two poles it finds the optimum (pinned against Zolotarev's closed
  form at p = -1/2), for more it gives an upper bound on the optimal error.
Shares no code with the HIP library.
"""

from __future__ import annotations

import numpy as np

from .core import cg
from .dense import dense_normal_op, parity_index


def rational_apply(dims, fat, lng, mass, alpha0, alphas, shifts, b, tol=1e-12):
    """alpha0 b + sum_k alphas[k] (A + shifts[k])^-1 b; b full-lattice (V, 3) on even sites."""
    out = alpha0 * np.asarray(b, dtype=np.complex128)
    for a, s in zip(alphas, shifts):
        x, st, _, _ = cg(dims, fat, lng, mass, b, tol=tol, sigma=float(s))
        if st != 0:
            raise RuntimeError(f"oracle CG for shift {s} did not converge")
        out = out + a * x
    return out


def dense_power(dims, fat, lng, mass, b, p):
    """A^p b (full-lattice (V, 3) in and out, even sites) and A's extreme eigenvalues."""
    A = dense_normal_op(dims, fat, lng, mass)
    w, Q = np.linalg.eigh(A)
    e = parity_index(dims, 0)
    be = np.asarray(b, dtype=np.complex128).ravel()[e]
    ye = Q @ (w ** p * (Q.conj().T @ be))
    out = np.zeros(int(np.prod(dims)) * 3, dtype=np.complex128)
    out[e] = ye
    return out.reshape(-1, 3), float(w[0]), float(w[-1])


def _product(x, c, n):
    r = np.ones_like(x)
    for l in range(n):
        r = r * (x + c[2 * l + 1]) / (x + c[2 * l])
    return r


def zolotarev_inv_sqrt(lmin, lmax, n):
    """(alpha0, alphas, shifts, delta) with x^(-1/2) ~ alpha0 + sum alphas / (x + shifts)."""
    from scipy.special import ellipj, ellipk
    b = lmax / lmin
    m = 1.0 - 1.0 / b
    K = ellipk(m)
    # the lower half directly; the upper half from the quarter-period shift
    # tn(K - v) tn(v) = 1 / sqrt(1 - m), i.e. c_l c_{2n+1-l} = 1 / (1 - m)
    # (there cn is tiny and ellipj's cn has lost its relative accuracy).  The
    # 1 - m that ellipj sees is the rounded one, so the mirror uses it too:
    # every node then belongs to the same interval [1, 1 / (1 - m)], which
    # differs from [1, b] by the rounding of m (~1e-16 b)
    sn, cn, _, _ = ellipj(np.arange(1, n + 1) * K / (2 * n + 1), m)
    lower = sn ** 2 / cn ** 2
    c = np.concatenate([lower, (1.0 / (1.0 - m)) / lower[::-1]])
    # fine enough that the parabola through a grid triple places each extremum
    # value to ~1e-6 of the error itself (its error is cubic in the spacing)
    x = np.exp(np.linspace(0.0, np.log(b), 8000 * n + 8001))
    f = np.sqrt(x) * _product(x, c, n)
    # refine every interior extremum by a parabola through the grid triple
    lo, hi = [f[0], f[-1]], [f[0], f[-1]]
    i = np.arange(1, len(f) - 1)
    for k in i[((f[i] - f[i - 1]) * (f[i + 1] - f[i])) <= 0]:
        u = np.log(x[k - 1:k + 2])
        cf = np.polyfit(u, f[k - 1:k + 2], 2)
        if cf[0] != 0:
            uv = -cf[1] / (2 * cf[0])
            if u[0] <= uv <= u[2]:
                xv = np.exp(uv)
                fv = float(np.sqrt(xv) * _product(np.array([xv]), c, n)[0])
                lo.append(fv)
                hi.append(fv)
        lo.append(f[k])
        hi.append(f[k])
    fmin, fmax = min(lo), max(hi)
    D = 2.0 / (fmin + fmax)
    delta = (fmax - fmin) / (fmax + fmin)
    p = c[0::2]
    num = c[1::2]
    res = np.empty(n)
    for l in range(n):
        # one ratio per factor: the separate products overflow for many poles
        others = np.delete(p, l)
        res[l] = D * (num[-1] - p[l]) * np.prod((num[:-1] - p[l]) / (others - p[l]))
    s = np.sqrt(lmin)
    return D / s, res * s, p * lmin, float(delta)


def relative_error_extrema(alpha0, alphas, shifts, lmin, lmax, npts=200001, power=-0.5):
    """Values of x^(-power) r(x) - 1 at its alternation points on [lmin, lmax] (ends included)."""
    ld = np.longdouble
    x = np.exp(np.linspace(np.log(ld(lmin)), np.log(ld(lmax)), npts, dtype=ld))
    r = ld(alpha0) + sum(ld(a) / (x + ld(s)) for a, s in zip(alphas, shifts))
    e = r * x ** ld(-power) - 1
    d = np.diff(e)
    k = np.where(np.sign(d[1:]) != np.sign(d[:-1]))[0] + 1
    # the peak value of the parabola through each grid triple: near the ends
    # of the interval the extrema are sharp and the grid value under-reads them
    em, e0, ep = e[k - 1], e[k], e[k + 1]
    curv = ep - 2 * e0 + em
    safe = np.where(curv != 0, curv, 1)
    peak = np.where(curv != 0, e0 - (ep - em) ** 2 / (8 * safe), e0)
    ext = []
    for v in np.concatenate([[e[0]], peak, [e[-1]]]):
        if ext and (ext[-1] > 0) == (v > 0):
            if abs(v) > abs(ext[-1]):
                ext[-1] = v
        else:
            ext.append(v)
    return np.array(ext, dtype=np.float64)


def minimax_bruteforce(p, lmin, lmax, n, npts=4001, restarts=3):
    """(delta, shifts): the smallest max relative error of a type (n, n)
    rational approximation of x^p on [lmin, lmax] that direct minimisation
    finds, and its poles -q_i (as shifts q_i, ascending).

    The largest error is not differentiable, so it is approached through the
    L_q norms of the error on the grid, q = 2, 4, ..., 4096 (each a smooth
    function of the parameters, minimised by BFGS from the previous optimum;
    the L_q norm tends to the maximum as q grows), and then polished by
    Nelder-Mead on the maximum itself.  delta is the maximum of the result's
    error on a grid 50 times finer, so it bounds the error of what was found
    from below by at most the grid's under-reading of a smooth extremum
    (~1e-8 relative)."""
    from scipy.optimize import minimize
    from scipy.special import logsumexp

    def err_on(x):
        lx = np.log(x)

        def err(th):
            lc, lz, lq = th[0], th[1:n + 1], th[n + 1:]
            lr = lc + np.sum(np.log(x[:, None] + np.exp(lz)[None, :]) - np.log(x[:, None] + np.exp(lq)[None, :]),
                             axis=1)
            return np.expm1(lr - p * lx)
        return err

    x = np.exp(np.linspace(np.log(lmin), np.log(lmax), npts))
    err = err_on(x)

    def max_err(th):
        return float(np.max(np.abs(err(th))))

    # start: zeros and poles interlaced, evenly spread in log x
    lx = np.log(x)
    t = np.linspace(np.log(lmin), np.log(lmax), 2 * n + 2)[1:-1]
    lq0, lz0 = (t[0::2], t[1::2]) if p < 0 else (t[1::2], t[0::2])
    lc0 = np.mean(p * lx - np.sum(np.log(x[:, None] + np.exp(lz0)) - np.log(x[:, None] + np.exp(lq0)), axis=1))
    th = np.concatenate([[lc0], lz0, lq0])
    for q in 2.0 ** np.arange(1, 13):
        def lq_norm(th, q=q):
            return float((logsumexp(q * np.log(np.abs(err(th)) + 1e-300)) - np.log(npts)) / q)
        th = minimize(lq_norm, th, method="BFGS").x
    for _ in range(restarts):
        th = minimize(max_err, th, method="Nelder-Mead",
                      options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 20000, "maxfev": 40000}).x
    fine = err_on(np.exp(np.linspace(np.log(lmin), np.log(lmax), 50 * (npts - 1) + 1)))
    return float(np.max(np.abs(fine(th)))), np.sort(np.exp(th[n + 1:]))
