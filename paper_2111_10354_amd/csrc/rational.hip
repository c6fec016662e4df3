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
//  * the power-iteration estimate of the top of A's spectrum (the bottom is
//    bounded by 4 m^2 since D^+ D >= 0);
//  * the application alpha_0 b + sum_k alpha_k x_k after the multi-shift solve.

#include <algorithm>
#include <cmath>
#include <vector>

#include "solver_internal.h"

namespace hisq {

// ------------------------------------------------------------------ elliptic functions (host)
// Complete elliptic integral K(m) from the complementary parameter m1 = 1 - m
// (accurate as m -> 1): K = pi / (2 AGM(1, sqrt(m1))).
static double ellip_k_from_m1(double m1) {
    double a = 1.0, b = std::sqrt(m1);
    for (int i = 0; i < 64 && std::fabs(a - b) > 1e-17 * a; ++i) {
        const double t = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = t;
    }
    return M_PI / (2.0 * a);
}

// Jacobi sn and cn of (u | m), m1 = 1 - m, by the descending Landen (AGM)
// sequence: a_{n+1} = (a_n + b_n)/2, b_{n+1} = sqrt(a_n b_n),
// c_{n+1} = (a_n - b_n)/2, then phi_N = 2^N a_N u and
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2; sn = sin phi_0.
static void ellip_sn_cn(double u, double m1, double *sn, double *cn) {
    constexpr int NMAX = 48;
    double a[NMAX + 1], c[NMAX + 1];
    double an = 1.0, bn = std::sqrt(m1);
    a[0] = an;
    c[0] = std::sqrt(1.0 - m1);
    int n = 0;
    while (n < NMAX && std::fabs(c[n]) > 1e-17 * a[n]) {
        const double a1 = 0.5 * (an + bn), b1 = std::sqrt(an * bn), c1 = 0.5 * (an - bn);
        an = a1;
        bn = b1;
        ++n;
        a[n] = an;
        c[n] = c1;
    }
    double phi = std::ldexp(a[n] * u, n);
    for (int k = n; k > 0; --k) phi = 0.5 * (phi + std::asin(c[k] * std::sin(phi) / a[k]));
    *sn = std::sin(phi);
    *cn = std::cos(phi);
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

int zolotarev_inv_sqrt(double lmin, double lmax, int n, double *alpha0, double *alpha, double *shift,
                       double *delta) {
    const double b = lmax / lmin;
    const double m1 = 1.0 / b;  // 1 - k'^2
    const double K = ellip_k_from_m1(m1);
    std::vector<double> c(2 * n);
    for (int l = 1; l <= 2 * n; ++l) {
        double sn, cn;
        ellip_sn_cn(l * K / (2 * n + 1), m1, &sn, &cn);
        c[l - 1] = (sn * sn) / (cn * cn);
    }
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
int rational_apply(hisq_gauge_s *g, double mass, double alpha0, int n, const double *alpha, const double *shift,
                   const double *b, double *out, const hisq_solver_params &prm, hisq_solver_stats *st,
                   hipStream_t s) {
    const int vh = g->geom.vh;
    const size_t s64 = spinor_bytes(F64, vh);
    DevBuf xs, al;
    int rc, worst = HISQ_OK;
    if (n > 0) {
        if ((rc = xs.alloc(s64 * n)) || (rc = al.alloc(sizeof(double) * n))) return rc;
        worst = multishift_solve(g, mass, n, shift, b, (double *)xs.p, prm, st, s);
        if (worst < 0) return worst;
        HISQ_HIP_CHECK(hipMemcpyAsync(al.p, alpha, sizeof(double) * n, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_rational_combine, dim3((vh + 255) / 256), dim3(256), 0, s, vh, (const d2v *)b, alpha0, n,
                       (const double *)al.p, (const d2v *)xs.p, (d2v *)out);
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
