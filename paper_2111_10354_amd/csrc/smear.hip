// HISQ link smearing on the GPU in FP64 (the HISQ action of Follana et al.,
// Phys. Rev. D 75 (2007) 054502, which the paper's code simulates, Sec. 1):
//
//   level 1   V = fat7[U]:  c1 U + c3 sum S_nu[U] + c5 sum S_rho[S_nu[U]]
//                           + c7 sum S_sig[S_rho[S_nu[U]]],  (1/8, 1/16, 1/64, 1/384)
//   U(3)      W = V (V^+ V)^(-1/2)
//   level 2   X = fat7[W] with one-link 1 and the Lepage term -1/8 sum S2_nu[W]
//   Naik      L_mu(x) = -1/24 W_mu(x) W_mu(x+mu) W_mu(x+2mu)
//
// S_nu[A]_mu(x) = T_nu(x) A_mu(x+nu) T_nu(x+mu)^+ + T_nu(x-nu)^+ A_mu(x-nu) T_nu(x-nu+mu)
// is the staple of the links A of direction mu transported along +-nu by the
// links T of the level (U, then W); S2 uses two-link transports and shifts.
// Every sum runs over distinct directions different from mu, every ordering.
//
// Fields are full-lattice link fields in the canonical layout [V][4][3][3]
// (or one direction, [V][3][3]); one thread per site.  This runs once per
// gauge field, before the solver: plain FP64 arithmetic on 3x3 matrices, the
// bandwidth of ~150 launches over link fields is its cost.

#include "solver_internal.h"

namespace hisq {

namespace {

struct M3 {
    cx<double> e[9];
};

// Link field view: the matrix of site x is at p + (x * nd + mu) * 18 doubles.
struct LinkView {
    double *p;
    int nd;
    int mu;
    __device__ __forceinline__ M3 at(int64_t x) const {
        const d2v *q = (const d2v *)p + ((size_t)x * nd + mu) * 9;
        M3 m;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const d2v v = q[i];
            m.e[i] = {v.x, v.y};
        }
        return m;
    }
    __device__ __forceinline__ void put(int64_t x, const M3 &m) const {
        d2v *q = (d2v *)p + ((size_t)x * nd + mu) * 9;
#pragma unroll
        for (int i = 0; i < 9; ++i) q[i] = d2v{m.e[i].re, m.e[i].im};
    }
};

__device__ __forceinline__ M3 mul(const M3 &a, const M3 &b) {  // a b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a.e[3 * i + k], b.e[3 * k + j]);
            r.e[3 * i + j] = s;
        }
    return r;
}

__device__ __forceinline__ cx<double> conjc(cx<double> a) { return {a.re, -a.im}; }

__device__ __forceinline__ M3 mul_an(const M3 &a, const M3 &b) {  // a^+ b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, conjc(a.e[3 * k + i]), b.e[3 * k + j]);
            r.e[3 * i + j] = s;
        }
    return r;
}

__device__ __forceinline__ M3 mul_na(const M3 &a, const M3 &b) {  // a b^+
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a.e[3 * i + k], conjc(b.e[3 * j + k]));
            r.e[3 * i + j] = s;
        }
    return r;
}

struct Lat {
    int L[4];
    int64_t V;
    __device__ __forceinline__ void coords(int64_t x, int c[4]) const {
        c[0] = (int)(x % L[0]);
        x /= L[0];
        c[1] = (int)(x % L[1]);
        x /= L[1];
        c[2] = (int)(x % L[2]);
        c[3] = (int)(x / L[2]);
    }
    __device__ __forceinline__ int64_t lex(const int c[4]) const {
        return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
    }
    // site reached from coordinates c by k steps along d (|k| < L[d])
    __device__ __forceinline__ int64_t hop(const int c[4], int d, int k) const {
        int q[4] = {c[0], c[1], c[2], c[3]};
        q[d] = wrap(q[d] + k, L[d]);
        return lex(q);
    }
    __device__ __forceinline__ int64_t hop2(const int c[4], int d1, int k1, int d2, int k2) const {
        int q[4] = {c[0], c[1], c[2], c[3]};
        q[d1] = wrap(q[d1] + k1, L[d1]);
        q[d2] = wrap(q[d2] + k2, L[d2]);
        return lex(q);
    }
};

// S_nu[A]_mu (dist 1) or its two-step form (dist 2) at every site; written to
// `set` (if given) and added with weight `coeff` to `acc` (if given).
__global__ __launch_bounds__(256) void k_staple(Lat lat, LinkView T, LinkView A, int mu, int nu, int dist,
                                                LinkView set, LinkView acc, double coeff) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= lat.V) return;
    int c[4];
    lat.coords(x, c);
    LinkView Tn{T.p, T.nd, nu};
    M3 fwd, bwd;
    if (dist == 1) {
        fwd = mul_na(mul(Tn.at(x), A.at(lat.hop(c, nu, 1))), Tn.at(lat.hop(c, mu, 1)));
        const int64_t xm = lat.hop(c, nu, -1);
        bwd = mul(mul_an(Tn.at(xm), A.at(xm)), Tn.at(lat.hop2(c, nu, -1, mu, 1)));
    } else {
        const M3 up = mul(Tn.at(x), Tn.at(lat.hop(c, nu, 1)));
        const M3 upm = mul(Tn.at(lat.hop(c, mu, 1)), Tn.at(lat.hop2(c, mu, 1, nu, 1)));
        fwd = mul_na(mul(up, A.at(lat.hop(c, nu, 2))), upm);
        const int64_t x2 = lat.hop(c, nu, -2);
        const M3 dn = mul(Tn.at(x2), Tn.at(lat.hop(c, nu, -1)));
        const M3 dnm = mul(Tn.at(lat.hop2(c, nu, -2, mu, 1)), Tn.at(lat.hop2(c, nu, -1, mu, 1)));
        bwd = mul(mul_an(dn, A.at(x2)), dnm);
    }
    M3 s;
#pragma unroll
    for (int i = 0; i < 9; ++i) s.e[i] = {fwd.e[i].re + bwd.e[i].re, fwd.e[i].im + bwd.e[i].im};
    if (set.p) set.put(x, s);
    if (acc.p) {
        M3 a = acc.at(x);
#pragma unroll
        for (int i = 0; i < 9; ++i) a.e[i] = {fma(coeff, s.e[i].re, a.e[i].re), fma(coeff, s.e[i].im, a.e[i].im)};
        acc.put(x, a);
    }
}

// out_mu = coeff * A_mu for all four directions (canonical fields)
__global__ __launch_bounds__(256) void k_scale(int64_t n, const double *__restrict__ a, double *__restrict__ out,
                                               double coeff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one complex entry
    if (i >= n) return;
    const d2v v = ((const d2v *)a)[i];
    ((d2v *)out)[i] = d2v{coeff * v.x, coeff * v.y};
}

// W = V (V^+ V)^(-1/2) in place, every link of a canonical field.  With the
// eigenvalues l_i = s_i^2 of Q = V^+ V (all positive), Q^(-1/2) = f0 + f1 Q +
// f2 Q^2 where the f's interpolate 1/s at the three s_i; in terms of u = sum
// s_i, v = sum_{i<j} s_i s_j, w = prod s_i (so that the denominators carry
// u v - w = (s0+s1)(s0+s2)(s1+s2) > 0 and stay finite for equal eigenvalues):
//   f2 = u / d,  f1 = (2 u v - w - u^3) / d,  f0 = (v (u v - w) - w u^2) / d,
//   d = w (u v - w).
__global__ __launch_bounds__(256) void k_u3_project(int64_t nlinks, double *links) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlinks) return;
    LinkView lv{links, 1, 0};
    const M3 v = lv.at(i);
    const M3 q = mul_an(v, v);
    // eigenvalues of the Hermitian Q: trigonometric solution of the cubic
    const double m = (q.e[0].re + q.e[4].re + q.e[8].re) / 3.0;
    const double k00 = q.e[0].re - m, k11 = q.e[4].re - m, k22 = q.e[8].re - m;
    const cx<double> k01 = q.e[1], k02 = q.e[2], k12 = q.e[5];
    const double n01 = k01.re * k01.re + k01.im * k01.im, n02 = k02.re * k02.re + k02.im * k02.im,
                 n12 = k12.re * k12.re + k12.im * k12.im;
    const double p = (k00 * k00 + k11 * k11 + k22 * k22 + 2.0 * (n01 + n02 + n12)) / 6.0;
    // det K for Hermitian K: real
    const cx<double> t = cmul(cmul(k01, k12), conjc(k02));
    const double detk = k00 * k11 * k22 + 2.0 * t.re - k00 * n12 - k11 * n02 - k22 * n01;
    double l[3];
    if (p <= 1e-300) {
        l[0] = l[1] = l[2] = m;
    } else {
        const double sp = sqrt(p);
        double r = detk / (2.0 * p * sp);
        r = fmin(1.0, fmax(-1.0, r));
        const double phi = acos(r) / 3.0;
        const double tpi3 = 2.0943951023931954923;  // 2 pi / 3
        l[0] = m + 2.0 * sp * cos(phi);
        l[1] = m + 2.0 * sp * cos(phi + tpi3);
        l[2] = m + 2.0 * sp * cos(phi - tpi3);
    }
    const double s0 = sqrt(fmax(l[0], 0.0)), s1 = sqrt(fmax(l[1], 0.0)), s2 = sqrt(fmax(l[2], 0.0));
    const double u = s0 + s1 + s2, vv = s0 * s1 + s0 * s2 + s1 * s2, w = s0 * s1 * s2;
    const double uvw = u * vv - w, d = w * uvw;
    const double f2 = u / d, f1 = (2.0 * u * vv - w - u * u * u) / d, f0 = (vv * uvw - w * u * u) / d;
    const M3 q2 = mul(q, q);
    M3 r;
#pragma unroll
    for (int e = 0; e < 9; ++e)
        r.e[e] = {f1 * q.e[e].re + f2 * q2.e[e].re, f1 * q.e[e].im + f2 * q2.e[e].im};
    r.e[0].re += f0;
    r.e[4].re += f0;
    r.e[8].re += f0;
    const M3 wc = mul(v, r);
    // one Newton-Schulz step towards the polar factor, W <- W (3 - W^+ W) / 2:
    // where V is badly conditioned the closed form leaves W unitary only to
    // ~eps cond(V)^2; the step squares that defect
    const M3 ww = mul_an(wc, wc);
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = {-0.5 * ww.e[e].re, -0.5 * ww.e[e].im};
    r.e[0].re += 1.5;
    r.e[4].re += 1.5;
    r.e[8].re += 1.5;
    lv.put(i, mul(wc, r));
}

__device__ __forceinline__ double eta_sign(const int c[4], int mu) {
    int e = 0;
    for (int d = 0; d < mu; ++d) e += c[d];
    return (e & 1) ? -1.0 : 1.0;
}

// L_mu(x) = cN W_mu(x) W_mu(x+mu) W_mu(x+2mu), with eta_mu(x) and the time
// boundary sign (t + 3 >= Lt) folded in
__global__ __launch_bounds__(256) void k_naik(Lat lat, LinkView W, double *lng, double cn, int apbc) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= lat.V) return;
    int c[4];
    lat.coords(x, c);
    for (int mu = 0; mu < 4; ++mu) {
        LinkView Wm{W.p, 4, mu};
        const M3 p = mul(mul(Wm.at(x), Wm.at(lat.hop(c, mu, 1))), Wm.at(lat.hop(c, mu, 2)));
        double sg = cn * eta_sign(c, mu);
        if (apbc && mu == 3 && c[3] + 3 >= lat.L[3]) sg = -sg;
        M3 o;
#pragma unroll
        for (int e = 0; e < 9; ++e) o.e[e] = {sg * p.e[e].re, sg * p.e[e].im};
        LinkView{lng, 4, mu}.put(x, o);
    }
}

// X_mu(x) *= eta_mu(x) (and -1 where the t link crosses an antiperiodic boundary)
__global__ __launch_bounds__(256) void k_fold(Lat lat, double *fat, int apbc) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= lat.V) return;
    int c[4];
    lat.coords(x, c);
    for (int mu = 0; mu < 4; ++mu) {
        double sg = eta_sign(c, mu);
        if (apbc && mu == 3 && c[3] + 1 >= lat.L[3]) sg = -sg;
        if (sg > 0) continue;
        LinkView lv{fat, 4, mu};
        M3 m = lv.at(x);
#pragma unroll
        for (int e = 0; e < 9; ++e) m.e[e] = {-m.e[e].re, -m.e[e].im};
        lv.put(x, m);
    }
}

// One fat7 (+ Lepage) smearing of the canonical field A with transports T into
// the canonical field `out`, using two one-direction temporaries.
int fat7(const Lat &lat, double *A, double *T, double *out, double *t1, double *t2, const double c[5],
         hipStream_t s) {
    const dim3 grid((unsigned)((lat.V + 255) / 256)), blk(256);
    const LinkView none{nullptr, 1, 0};
    hipLaunchKernelGGL(k_scale, dim3((unsigned)((lat.V * 36 + 255) / 256)), blk, 0, s, lat.V * 36, A, out, c[0]);
    for (int mu = 0; mu < 4; ++mu) {
        const LinkView Am{A, 4, mu}, Om{out, 4, mu}, Tv{T, 4, 0}, T1{t1, 1, 0}, T2{t2, 1, 0};
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            hipLaunchKernelGGL(k_staple, grid, blk, 0, s, lat, Tv, Am, mu, nu, 1, T1, Om, c[1]);
            if (c[4] != 0.0) hipLaunchKernelGGL(k_staple, grid, blk, 0, s, lat, Tv, Am, mu, nu, 2, none, Om, c[4]);
            for (int rho = 0; rho < 4; ++rho) {
                if (rho == mu || rho == nu) continue;
                hipLaunchKernelGGL(k_staple, grid, blk, 0, s, lat, Tv, T1, mu, rho, 1, T2, Om, c[2]);
                for (int sig = 0; sig < 4; ++sig) {
                    if (sig == mu || sig == nu || sig == rho) continue;
                    hipLaunchKernelGGL(k_staple, grid, blk, 0, s, lat, Tv, T2, mu, sig, 1, none, Om, c[3]);
                }
            }
        }
    }
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

}  // namespace

int smear_links(const int dims[4], const double *thin, double *fat, double *lng, unsigned flags, hipStream_t s) {
    Lat lat;
    for (int i = 0; i < 4; ++i) lat.L[i] = dims[i];
    lat.V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    const int apbc = (flags & HISQ_SMEAR_ANTIPERIODIC_T) ? 1 : 0;
    const size_t one = (size_t)lat.V * 9 * 16;  // one direction of a link field
    DevBuf w, t1, t2;
    int rc;
    if ((rc = w.alloc(4 * one)) || (rc = t1.alloc(one)) || (rc = t2.alloc(one))) return rc;
    double *W = (double *)w.p;
    static const double level1[5] = {1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0};
    static const double level2[5] = {1.0, 1.0 / 16, 1.0 / 64, 1.0 / 384, -1.0 / 8};
    if ((rc = fat7(lat, const_cast<double *>(thin), const_cast<double *>(thin), W, (double *)t1.p, (double *)t2.p,
                   level1, s)))
        return rc;
    hipLaunchKernelGGL(k_u3_project, dim3((unsigned)((4 * lat.V + 255) / 256)), dim3(256), 0, s, 4 * lat.V, W);
    if ((rc = fat7(lat, W, W, fat, (double *)t1.p, (double *)t2.p, level2, s))) return rc;
    const dim3 grid((unsigned)((lat.V + 255) / 256)), blk(256);
    hipLaunchKernelGGL(k_naik, grid, blk, 0, s, lat, LinkView{W, 4, 0}, lng, -1.0 / 24, apbc);
    hipLaunchKernelGGL(k_fold, grid, blk, 0, s, lat, fat, apbc);
    HISQ_HIP_CHECK(hipGetLastError());
    // the temporaries are freed on return: wait for the kernels that use them
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    return HISQ_OK;
}

}  // namespace hisq
