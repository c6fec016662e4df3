// Rational functions of the even-site normal operator A = (D^+ D)_ee + 4 m^2,
// the solver-side part of rational hybrid Monte Carlo: a rooted staggered
// pseudofermion action needs A^(-1/2) (two light flavours) applied to a vector,
// and a rational approximation in partial fractions
//     A^(-1/2) ~ alpha_0 + sum_k alpha_k (A + sigma_k)^(-1)
// turns that into one multi-shift CG over the poles sigma_k followed by a
// linear combination.  This file holds
//  * Zolotarev's optimal (minimax relative error) rational approximation of
//    x^(-1/2) on [lmin, lmax] (host code, FP64): with b = lmax / lmin, k' the
//    modulus with k'^2 = 1 - 1/b and K' = K(k'), the numbers
//        c_l = sn^2(l K'/(2n+1); k') / cn^2(l K'/(2n+1); k'),  l = 1 .. 2n,
//    give r(x) = D prod_l (x + c_{2l}) / (x + c_{2l-1}) on [1, b], whose
//    relative error sqrt(x) r(x) - 1 equioscillates 2n + 2 times once D
//    centres it;
//  * the minimax relative approximation of x^p for other powers (x^(1/4) for
//    the heat bath of the same pseudofermions, x^(-1/4) and x^(1/8) for the
//    strange quark) by Remez exchange, started from Zolotarev's solution;
//  * the power-iteration estimate of the top of A's spectrum (the bottom is
//    bounded by 4 m^2 since D^+ D >= 0);
//  * the application alpha_0 b + sum_k alpha_k x_k after the multi-shift solve.

#include <algorithm>
#include <cmath>
#include <vector>

#include "solver_internal.h"

namespace hisq {

// ------------------------------------------------------------------ elliptic functions (host)
// In x87 extended precision: for large b = lmax / lmin the nodes below come
// from cn ~ 1/sqrt(b) computed as cos(phi) near pi/2, whose relative error is
// the working precision divided by cn; in double that limits the nodes to
// ~1e-13 relative at b = 1e12, enough to break the equioscillation of an
// approximation whose error is ~1e-11.
//
// Complete elliptic integral K(m) from the complementary parameter m1 = 1 - m
// (accurate as m -> 1): K = pi / (2 AGM(1, sqrt(m1))).
static long double ellip_k_from_m1(long double m1) {
    long double a = 1.0L, b = sqrtl(m1);
    for (int i = 0; i < 64 && fabsl(a - b) > 1e-20L * a; ++i) {
        const long double t = 0.5L * (a + b);
        b = sqrtl(a * b);
        a = t;
    }
    return 3.14159265358979323846264338327950288L / (2.0L * a);
}

// Jacobi sn and cn of (u | m), m1 = 1 - m, by the descending Landen (AGM)
// sequence: a_{n+1} = (a_n + b_n)/2, b_{n+1} = sqrt(a_n b_n),
// c_{n+1} = (a_n - b_n)/2, then phi_N = 2^N a_N u and
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2; sn = sin phi_0.
static void ellip_sn_cn(long double u, long double m1, long double *sn, long double *cn) {
    constexpr int NMAX = 48;
    long double a[NMAX + 1], c[NMAX + 1];
    long double an = 1.0L, bn = sqrtl(m1);
    a[0] = an;
    c[0] = sqrtl(1.0L - m1);
    int n = 0;
    while (n < NMAX && fabsl(c[n]) > 1e-20L * a[n]) {
        const long double a1 = 0.5L * (an + bn), b1 = sqrtl(an * bn), c1 = 0.5L * (an - bn);
        an = a1;
        bn = b1;
        ++n;
        a[n] = an;
        c[n] = c1;
    }
    long double phi = ldexpl(a[n] * u, n);
    for (int k = n; k > 0; --k) phi = 0.5L * (phi + asinl(c[k] * sinl(phi) / a[k]));
    *sn = sinl(phi);
    *cn = cosl(phi);
}

// sqrt(x) prod_l (x + c_{2l}) / (x + c_{2l-1}) (c 0-based: c[2l+1] / c[2l])
static double zolo_f(double x, const std::vector<double> &c, int n) {
    double f = std::sqrt(x);
    for (int l = 0; l < n; ++l) f *= (x + c[2 * l + 1]) / (x + c[2 * l]);
    return f;
}

// Extremum of zolo_f in [lo, hi] (golden section on log x; sign +1 = max).
static double zolo_extremum(double lo, double hi, const std::vector<double> &c, int n, int sign) {
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = std::log(lo), b = std::log(hi);
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = sign * zolo_f(std::exp(x1), c, n), f2 = sign * zolo_f(std::exp(x2), c, n);
    for (int it = 0; it < 200 && b - a > 1e-14 * std::max(1.0, std::fabs(a)); ++it) {
        if (f1 > f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            f1 = sign * zolo_f(std::exp(x1), c, n);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            f2 = sign * zolo_f(std::exp(x2), c, n);
        }
    }
    return sign * std::max(f1, f2);
}

// c_l = sn^2 / cn^2 (l K' / (2n + 1); k'), l = 1 .. 2n, for the interval [1, b]
// Only l <= n is evaluated: for u near K' cn is tiny and loses its relative
// accuracy.  The upper half follows from the quarter-period shift
// tn(K' - v) = 1 / (sqrt(1 - k'^2) tn(v)), i.e. c_l c_{2n+1-l} = b.
static std::vector<double> zolotarev_nodes(double b, int n) {
    const long double m1 = 1.0L / (long double)b;  // 1 - k'^2
    const long double K = ellip_k_from_m1(m1);
    std::vector<double> c(2 * n);
    for (int l = 1; l <= n; ++l) {
        long double sn, cn;
        ellip_sn_cn(l * K / (2 * n + 1), m1, &sn, &cn);
        const long double t = (sn * sn) / (cn * cn);
        c[l - 1] = (double)t;
        c[2 * n - l] = (double)((long double)b / t);
    }
    return c;
}

int zolotarev_inv_sqrt(double lmin, double lmax, int n, double *alpha0, double *alpha, double *shift,
                       double *delta) {
    const double b = lmax / lmin;
    const std::vector<double> c = zolotarev_nodes(b, n);
    // centre the relative error: D = 2 / (max f + min f) over [1, b], the
    // extrema found on a log grid and refined by golden section (the ends of
    // the interval are extrema too)
    const int NG = 400 * n + 400;
    std::vector<double> xs(NG + 1), fs(NG + 1);
    for (int i = 0; i <= NG; ++i) {
        xs[i] = std::exp(std::log(b) * i / NG);
        fs[i] = zolo_f(xs[i], c, n);
    }
    double fmax = std::max(fs[0], fs[NG]), fmin = std::min(fs[0], fs[NG]);
    for (int i = 1; i < NG; ++i) {
        if (fs[i] >= fs[i - 1] && fs[i] >= fs[i + 1]) fmax = std::max(fmax, zolo_extremum(xs[i - 1], xs[i + 1], c, n, +1));
        if (fs[i] <= fs[i - 1] && fs[i] <= fs[i + 1]) fmin = std::min(fmin, zolo_extremum(xs[i - 1], xs[i + 1], c, n, -1));
    }
    const double D = 2.0 / (fmax + fmin);
    if (delta) *delta = (fmax - fmin) / (fmax + fmin);
    // partial fractions on [1, b]: r(x) = D + sum_l r_l / (x + p_l), p_l = c_{2l-1}
    std::vector<double> p(n), r(n);
    for (int l = 0; l < n; ++l) p[l] = c[2 * l];
    for (int l = 0; l < n; ++l) {
        double v = D;
        for (int j = 0; j < n; ++j) {
            v *= (c[2 * j + 1] - p[l]);
            if (j != l) v /= (p[j] - p[l]);
        }
        r[l] = v;
    }
    // scale to [lmin, lmax]: x^(-1/2) = lmin^(-1/2) (x / lmin)^(-1/2)
    const double s = std::sqrt(lmin);
    *alpha0 = D / s;
    for (int l = 0; l < n; ++l) {
        alpha[l] = r[l] * s;
        shift[l] = p[l] * lmin;
    }
    return HISQ_OK;
}

// ------------------------------------------------------------------ minimax rational approximation of x^p (host)
// Best relative approximation of type (n, n) of x^p on [1, b], kept as a
// product r(x) = c prod_i (x + z_i) / (x + q_i) whose parameters are stored as
// logarithms.  The derivative of log r with respect to log z_i is z_i/(x+z_i),
// a step in log x centred on z_i; with interlaced zeros and poles these steps
// are well separated, so the Newton systems below stay well conditioned in
// FP64 where a solve for partial-fraction coefficients does not.
//
// Chebyshev's alternation theorem characterises the optimum: the relative
// error r(x) x^(-p) - 1 reaches its largest magnitude E at 2n + 2 points with
// alternating signs.  The Remez exchange repeats two steps: solve
// r(x_j) x_j^(-p) = 1 + (-1)^j E on the reference points x_j (Newton on the
// 2n + 1 parameters and E), then move every x_j to the extremum of the new
// error in its bracket.  The start is Zolotarev's solution for p = -1/2 (or its
// reciprocal for p = +1/2), carried along p to the requested power in steps of
// at most 0.05, so every exchange begins next to its answer.
namespace {

struct ProdForm {
    double lc = 0.0;                 // log c
    std::vector<double> lz, lq;      // log zeros, log poles
    std::vector<long double> z, q;   // exp of the above

    void sync() {
        z.resize(lz.size());
        q.resize(lq.size());
        for (size_t i = 0; i < lz.size(); ++i) {
            z[i] = expl((long double)lz[i]);
            q[i] = expl((long double)lq[i]);
        }
    }
};

// log(r(x) x^(-p)) in extended precision: its rounding is the noise floor of
// the alternation test
long double log_ratio(long double x, double p, const ProdForm &r) {
    long double s = (long double)r.lc - (long double)p * logl(x);
    for (size_t i = 0; i < r.z.size(); ++i) s += logl(x + r.z[i]) - logl(x + r.q[i]);
    return s;
}

double rel_err_t(double t, double p, const ProdForm &r) { return (double)expm1l(log_ratio(expl((long double)t), p, r)); }

// the point of [ta, tb] (t = log x) where sgn * error is largest: golden
// section inside, compared with both ends (the interval ends are extremal
// points of the optimum)
double bracket_peak(double ta, double tb, double p, const ProdForm &r, int sgn, double *val) {
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = ta, b = tb, x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = sgn * rel_err_t(x1, p, r), f2 = sgn * rel_err_t(x2, p, r);
    for (int it = 0; it < 56; ++it) {
        if (f1 > f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - g * (b - a);
            f1 = sgn * rel_err_t(x1, p, r);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + g * (b - a);
            f2 = sgn * rel_err_t(x2, p, r);
        }
    }
    double bt = f1 > f2 ? x1 : x2, bf = std::max(f1, f2);
    const double fa = sgn * rel_err_t(ta, p, r), fb = sgn * rel_err_t(tb, p, r);
    if (fa > bf) bt = ta, bf = fa;
    if (fb > bf) bt = tb, bf = fb;
    *val = sgn * bf;
    return bt;
}

// Gaussian elimination with partial pivoting, a row-major m x m, solution in rhs
bool dense_solve(int m, std::vector<double> &a, std::vector<double> &rhs) {
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (std::fabs(a[(size_t)i * m + k]) > std::fabs(a[(size_t)piv * m + k])) piv = i;
        if (!(std::fabs(a[(size_t)piv * m + k]) > 0.0)) return false;
        if (piv != k) {
            for (int j = 0; j < m; ++j) std::swap(a[(size_t)k * m + j], a[(size_t)piv * m + j]);
            std::swap(rhs[k], rhs[piv]);
        }
        for (int i = k + 1; i < m; ++i) {
            const double f = a[(size_t)i * m + k] / a[(size_t)k * m + k];
            if (f == 0.0) continue;
            for (int j = k; j < m; ++j) a[(size_t)i * m + j] -= f * a[(size_t)k * m + j];
            rhs[i] -= f * rhs[k];
        }
    }
    for (int k = m - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int j = k + 1; j < m; ++j) s -= a[(size_t)k * m + j] * rhs[j];
        rhs[k] = s / a[(size_t)k * m + k];
    }
    for (int k = 0; k < m; ++k)
        if (!std::isfinite(rhs[k])) return false;
    return true;
}

// residuals log(r(x_j) x_j^(-p)) - log(1 + (-1)^j E); returns the largest magnitude
double reference_residual(const std::vector<double> &t, double p, const ProdForm &r, double E,
                          std::vector<long double> &g) {
    double mx = 0.0;
    for (size_t j = 0; j < t.size(); ++j) {
        const long double s = (j & 1) ? -1.0L : 1.0L;
        g[j] = log_ratio(expl((long double)t[j]), p, r) - log1pl(s * E);
        mx = std::max(mx, (double)fabsl(g[j]));
    }
    return std::isfinite(mx) ? mx : HUGE_VAL;
}

// Newton with backtracking on the reference points t (logs); false on failure
bool solve_reference(const std::vector<double> &t, double p, ProdForm &r, double &E) {
    const int n = (int)r.lz.size(), m = 2 * n + 2;
    std::vector<long double> g(m);
    std::vector<double> J((size_t)m * m), d(m);
    double res = reference_residual(t, p, r, E, g);
    for (int it = 0; it < 40 && res > 1e-17; ++it) {
        for (int j = 0; j < m; ++j) {
            const long double x = expl((long double)t[j]);
            const double s = (j & 1) ? -1.0 : 1.0;
            double *row = &J[(size_t)j * m];
            row[0] = 1.0;
            for (int i = 0; i < n; ++i) {
                row[1 + i] = (double)(r.z[i] / (x + r.z[i]));
                row[1 + n + i] = (double)(-r.q[i] / (x + r.q[i]));
            }
            row[m - 1] = -s / (1.0 + s * E);
            d[j] = -(double)g[j];
        }
        if (!dense_solve(m, J, d)) return false;
        double lam = 1.0, step = 0.0;
        for (int k = 0; k < m; ++k) step = std::max(step, std::fabs(d[k]));
        ProdForm trial;
        double Et = E, rt = HUGE_VAL;
        bool descent = false;
        for (int bt = 0; bt < 30; ++bt, lam *= 0.5) {
            rt = HUGE_VAL;
            trial.lc = r.lc + lam * d[0];
            trial.lz.resize(n);
            trial.lq.resize(n);
            for (int i = 0; i < n; ++i) {
                trial.lz[i] = r.lz[i] + lam * d[1 + i];
                trial.lq[i] = r.lq[i] + lam * d[1 + n + i];
            }
            Et = E + lam * d[m - 1];
            if (!(std::fabs(Et) < 0.9)) continue;
            trial.sync();
            rt = reference_residual(t, p, trial, Et, g);
            if (rt < res) {
                descent = true;
                break;
            }
            if (lam * step < 1e-15) break;
        }
        if (!descent) break;  // the residual is at its rounding floor
        r = trial;
        E = Et;
        res = rt;
    }
    reference_residual(t, p, r, E, g);
    return std::isfinite(E) && res < 1e-6;
}

// alternating extrema of the error on a log grid over [0, T] (ends included),
// reduced to the m of largest size
bool grid_reference(double T, double p, const ProdForm &r, int m, std::vector<double> &t) {
    const int ng = 64 * m + 1;
    std::vector<double> tg(ng), eg(ng);
    for (int i = 0; i < ng; ++i) {
        tg[i] = T * i / (ng - 1);
        eg[i] = rel_err_t(tg[i], p, r);
    }
    std::vector<std::pair<double, double>> ext;
    for (int i = 0; i < ng; ++i) {
        const bool is_ext = i == 0 || i == ng - 1 || (eg[i] - eg[i - 1]) * (eg[i + 1] - eg[i]) <= 0.0;
        if (!is_ext) continue;
        if (!ext.empty() && (ext.back().second > 0) == (eg[i] > 0)) {
            if (std::fabs(eg[i]) > std::fabs(ext.back().second)) ext.back() = {tg[i], eg[i]};
        } else {
            ext.push_back({tg[i], eg[i]});
        }
    }
    while ((int)ext.size() > m) {
        if (std::fabs(ext.front().second) < std::fabs(ext.back().second)) ext.erase(ext.begin());
        else ext.pop_back();
    }
    if ((int)ext.size() != m) return false;
    t.resize(m);
    for (int j = 0; j < m; ++j) t[j] = ext[j].first;
    return true;
}

// one exchange: every reference point moves to the extremum of its bracket;
// returns false if the signs stop alternating, else the spread max/min - 1
bool exchange(double T, double p, const ProdForm &r, std::vector<double> &t, double *spread, double *emax) {
    const int m = (int)t.size();
    std::vector<double> nt(m), ev(m);
    const int s0 = rel_err_t(t[0], p, r) > 0 ? 1 : -1;
    for (int j = 0; j < m; ++j) {
        const double lo = j == 0 ? 0.0 : 0.5 * (t[j - 1] + t[j]);
        const double hi = j == m - 1 ? T : 0.5 * (t[j] + t[j + 1]);
        const int sgn = (j & 1) ? -s0 : s0;
        nt[j] = bracket_peak(lo, hi, p, r, sgn, &ev[j]);
        if (!(sgn * ev[j] > 0.0)) return false;
    }
    double mx = 0.0, mn = HUGE_VAL;
    for (int j = 0; j < m; ++j) {
        mx = std::max(mx, std::fabs(ev[j]));
        mn = std::min(mn, std::fabs(ev[j]));
    }
    t = nt;
    *spread = mx / mn - 1.0;
    *emax = mx;
    return true;
}

}  // namespace

int remez_power(double power, double lmin, double lmax, int n, double *alpha0, double *alpha, double *shift,
                double *delta) {
    const double b = lmax / lmin, T = std::log(b);
    const int m = 2 * n + 2;
    // start: Zolotarev's x^(-1/2) (poles at the odd nodes), or its reciprocal
    const double p0 = power < 0 ? -0.5 : 0.5;
    const std::vector<double> c = zolotarev_nodes(b, n);
    ProdForm r;
    r.lz.resize(n);
    r.lq.resize(n);
    for (int i = 0; i < n; ++i) {
        const double lo = std::log(c[2 * i]), hi = std::log(c[2 * i + 1]);
        r.lq[i] = p0 < 0 ? lo : hi;
        r.lz[i] = p0 < 0 ? hi : lo;
    }
    r.sync();
    {
        double dmax = -HUGE_VAL, dmin = HUGE_VAL;
        const int ng = 64 * m + 1;
        for (int i = 0; i < ng; ++i) {
            const double d = (double)log_ratio(expl((long double)(T * i / (ng - 1))), p0, r);
            dmax = std::max(dmax, d);
            dmin = std::min(dmin, d);
        }
        r.lc = -0.5 * (dmax + dmin);
    }
    std::vector<double> t;
    if (!grid_reference(T, p0, r, m, t)) {
        set_error("remez: no alternation in the starting approximation");
        return HISQ_ERR_UNSUPPORTED;
    }
    double E = rel_err_t(t[0], p0, r);
    const int ns = std::max(1, (int)std::ceil(std::fabs(power - p0) / 0.05 - 1e-9));
    double spread = HUGE_VAL, emax = 0.0;
    for (int k = 1; k <= ns; ++k) {
        const double pk = p0 + (power - p0) * k / ns;
        const bool last = k == ns;
        double best = HUGE_VAL;
        int stall = 0;
        for (int it = 0; it < 60; ++it) {
            if (!solve_reference(t, pk, r, E) || !exchange(T, pk, r, t, &spread, &emax)) {
                set_error("remez: the exchange lost its alternation");
                return HISQ_ERR_UNSUPPORTED;
            }
            if (spread < (last ? 1e-6 : 1e-2)) break;
            if (spread < best * 0.999) best = spread, stall = 0;
            else if (++stall >= 4) break;
        }
    }
    // the optimum's error is E everywhere on the reference; check the whole
    // interval on a fine grid for an extremum the exchange did not see
    double gmax = emax;
    const int ng = 256 * m + 1;
    for (int i = 0; i < ng; ++i) gmax = std::max(gmax, std::fabs(rel_err_t(T * i / (ng - 1), power, r)));
    if (!(spread < 1e-2) || gmax > emax * (1.0 + 1e-3)) {
        set_error("remez: no equioscillating solution found (too many poles for this interval?)");
        return HISQ_ERR_UNSUPPORTED;
    }
    // partial fractions on [1, b]: r(x) = c + sum_k a_k / (x + q_k),
    // a_k = c prod_i (z_i - q_k) / prod_{i != k} (q_i - q_k)
    std::vector<double> z(n), q(n);
    for (int i = 0; i < n; ++i) {
        z[i] = std::exp(r.lz[i]);
        q[i] = std::exp(r.lq[i]);
    }
    std::sort(q.begin(), q.end());
    const double cc = std::exp(r.lc);
    // x^p on [lmin, lmax] = lmin^p (x / lmin)^p
    const double sp = std::pow(lmin, power);
    *alpha0 = cc * sp;
    for (int k = 0; k < n; ++k) {
        double v = cc;
        for (int i = 0; i < n; ++i) {
            v *= (z[i] - q[k]);
            if (i != k) v /= (q[i] - q[k]);
        }
        alpha[k] = v * sp * lmin;
        shift[k] = q[k] * lmin;
    }
    // for positive powers the terms cancel against alpha0 near x = 0 (r(0) ~ 0):
    // check the form that is returned, with its rounded coefficients, on the
    // reference points and a fine grid
    double pmax = 0.0;
    auto pf_err = [&](double tt) {
        const long double x = (long double)lmin * expl((long double)tt);
        long double v = *alpha0;
        for (int k = 0; k < n; ++k) v += (long double)alpha[k] / (x + (long double)shift[k]);
        pmax = std::max(pmax, (double)fabsl(v * powl(x, -(long double)power) - 1.0L));
    };
    for (int j = 0; j < m; ++j) pf_err(t[j]);
    for (int i = 0; i < ng; ++i) pf_err(T * i / (ng - 1));
    if (!(pmax <= gmax * 1.01)) {
        set_error("remez: the partial fractions lose the approximation to cancellation (power too close to 1 "
                  "for this interval)");
        return HISQ_ERR_UNSUPPORTED;
    }
    if (delta) *delta = std::max(gmax, pmax);
    return HISQ_OK;
}

// ------------------------------------------------------------------ device kernels
// out = alpha0 b + sum_k alpha_k x_k, FP64 spinors [3][vh], x stack [n][3][vh]
__global__ __launch_bounds__(256) void k_rational_combine(int vh, const d2v *__restrict__ b, double alpha0, int n,
                                                          const double *__restrict__ alpha,
                                                          const d2v *__restrict__ xs, d2v *__restrict__ out) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const d2v bv = b[(size_t)c * vh + h];
        double re = alpha0 * bv.x, im = alpha0 * bv.y;
        for (int k = 0; k < n; ++k) {
            const d2v xv = xs[((size_t)k * 3 + c) * vh + h];
            re += alpha[k] * xv.x;
            im += alpha[k] * xv.y;
        }
        out[(size_t)c * vh + h] = d2v{re, im};
    }
}

// deterministic pseudo-random start vector for the power iteration
__global__ __launch_bounds__(256) void k_fill_start(int vh, d2v *v, unsigned seed) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double val[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            unsigned x = (unsigned)(h * 6 + 2 * c + q) * 2654435761u ^ seed;
            x ^= x >> 15;
            x *= 0x2c1b3c6du;
            x ^= x >> 12;
            x *= 0x297a2d39u;
            x ^= x >> 15;
            val[q] = (x & 0xffffff) * (1.0 / 16777216.0) - 0.5;
        }
        v[(size_t)c * vh + h] = d2v{val[0], val[1]};
    }
}

__global__ __launch_bounds__(256) void k_scale_into(int vh, const d2v *__restrict__ src, const double *__restrict__ n2,
                                                    d2v *__restrict__ dst) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    const double f = 1.0 / std::sqrt(*n2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const d2v v = src[(size_t)c * vh + h];
        dst[(size_t)c * vh + h] = d2v{f * v.x, f * v.y};
    }
}

// ------------------------------------------------------------------ host drivers
// nsrc sources (stacks of FP64 spinors): one multi-shift solve for all of
// them (in lockstep in mixed precision), then the combination per source
int rational_apply(hisq_gauge_s *g, double mass, int nsrc, double alpha0, int n, const double *alpha,
                   const double *shift, const double *b, double *out, const hisq_solver_params &prm,
                   hisq_solver_stats *st, hipStream_t s) {
    const int vh = g->geom.vh;
    const size_t s64 = spinor_bytes(F64, vh);
    DevBuf xs, al;
    int rc, worst = HISQ_OK;
    if (n > 0) {
        if ((rc = xs.alloc(s64 * n * (size_t)nsrc)) || (rc = al.alloc(sizeof(double) * n))) return rc;
        worst = multishift_solve_batched(g, mass, nsrc, n, shift, b, (double *)xs.p, prm, st, s);
        if (worst < 0) return worst;
        HISQ_HIP_CHECK(hipMemcpyAsync(al.p, alpha, sizeof(double) * n, hipMemcpyHostToDevice, s));
    }
    for (int j = 0; j < nsrc; ++j)
        hipLaunchKernelGGL(k_rational_combine, dim3((vh + 255) / 256), dim3(256), 0, s, vh,
                           (const d2v *)((const char *)b + s64 * j), alpha0, n, (const double *)al.p,
                           (const d2v *)((const char *)xs.p + s64 * (size_t)n * j), (d2v *)((char *)out + s64 * j));
    HISQ_HIP_CHECK(hipGetLastError());
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    return worst;
}

int spectral_bounds(hisq_gauge_s *g, double mass, int iters, double *lmin, double *lmax, hipStream_t s) {
    if (!g->links[F64][0].p) {
        set_error("spectral bounds: the handle lacks packed FP64 links");
        return HISQ_ERR_UNSUPPORTED;
    }
    const int vh = g->geom.vh;
    const size_t s64 = spinor_bytes(F64, vh);
    const int nbd = nb_dslash(g, F64, F64, F64, 1, true), nbb = blas_blocks(vh);
    DevBuf v, t, av, part, scal, diag;
    int rc;
    if ((rc = v.alloc(s64)) || (rc = t.alloc(s64)) || (rc = av.alloc(s64)) ||
        (rc = part.alloc(sizeof(double) * std::max(nbd, nbb))) || (rc = scal.alloc(2 * sizeof(double))) ||
        (rc = diag.alloc(sizeof(double))))
        return rc;
    const double d = 4.0 * mass * mass;
    HISQ_HIP_CHECK(hipMemcpyAsync(diag.p, &d, sizeof(double), hipMemcpyHostToDevice, s));
    const dim3 grid((vh + 255) / 256);
    hipLaunchKernelGGL(k_fill_start, grid, dim3(256), 0, s, vh, (d2v *)v.p, 0x9e3779b9u);
    launch_norm2(vh, 1, v.p, (double *)part.p, s);
    launch_reduce(RED_STORE, 1, (double *)part.p, nbb, nullptr, (double *)scal.p, s);
    hipLaunchKernelGGL(k_scale_into, grid, dim3(256), 0, s, vh, (const d2v *)v.p, (const double *)scal.p, (d2v *)v.p);
    double rq = 0.0;
    for (int it = 0; it < iters; ++it) {
        // av = A v and the fused partials of Re <v, A v> (the Rayleigh quotient, |v| = 1)
        if ((rc = gauge_dslash(g, 1, F64, F64, F64, 1, v.p, t.p, nullptr, nullptr, nullptr, nullptr, s))) return rc;
        if ((rc = gauge_dslash(g, 0, F64, F64, F64, 1, t.p, av.p, v.p, (const double *)diag.p, (double *)part.p,
                               nullptr, s)))
            return rc;
        launch_reduce(RED_STORE, 1, (double *)part.p, nbd, nullptr, (double *)scal.p + 1, s);
        launch_norm2(vh, 1, av.p, (double *)part.p, s);
        launch_reduce(RED_STORE, 1, (double *)part.p, nbb, nullptr, (double *)scal.p, s);
        hipLaunchKernelGGL(k_scale_into, grid, dim3(256), 0, s, vh, (const d2v *)av.p, (const double *)scal.p,
                           (d2v *)v.p);
        HISQ_HIP_CHECK(hipGetLastError());
    }
    HISQ_HIP_CHECK(hipMemcpyAsync(&rq, (double *)scal.p + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    *lmin = d;
    *lmax = rq;
    return HISQ_OK;
}

}  // namespace hisq
