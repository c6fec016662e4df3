// Vector kernels of the CG family: fused updates with FP64 partial norms,
// deterministic two-stage reductions, precision conversions and the per-RHS
// scalar recurrences kept in device memory (so a chunk of iterations can be
// replayed from a captured graph without host round trips).
//
// Every per-site kernel runs one thread per site and one grid row per
// right-hand side; the per-block partial sums are reduced by a single block
// per RHS in a fixed order, so results are bitwise reproducible.

#include "solver_internal.h"

namespace hisq {

template <class T>
__device__ __forceinline__ T wave_sum64(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of one double per thread over the block, in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wave_sum64(v);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double reduce_partials(const double *part, int nb) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    return block_sum(s);
}

__device__ __forceinline__ bool finite(double v) { return v == v && fabs(v) <= 1.7e308; }

// ---------------------------------------------------------------- scalar steps
// alpha_i = rho_i / Re<p_i, A p_i>
__global__ void k_reduce_alpha(const double *__restrict__ part, int nb, CgState *st) {
    const int r = blockIdx.x;
    CgState &S = st[r];
    if (S.flag != CG_RUNNING) {
        if (threadIdx.x == 0) S.xpend = 0;
        return;
    }
    const double pap = reduce_partials(part + (size_t)r * nb, nb);
    if (threadIdx.x == 0) {
        S.pap = pap;
        if (!(pap > 0.0) || !finite(pap)) {
            S.flag = CG_BREAKDOWN;
            S.xpend = 0;
        } else {
            S.alpha = S.rho / pap;
            S.xpend = 1;
        }
    }
}

// rho_new = |r|^2; decide: continue (beta), convergence check / reliable
// update due (host attention), or stop at the iteration cap.
__global__ void k_reduce_beta(const double *__restrict__ part, int nb, CgState *st) {
    const int r = blockIdx.x;
    CgState &S = st[r];
    if (S.flag != CG_RUNNING) return;
    const double rr = reduce_partials(part + (size_t)r * nb, nb);
    if (threadIdx.x == 0) {
        S.rho_new = rr;
        S.iter += 1;
        S.since_ru += 1;
        if (!finite(rr)) {
            S.flag = CG_BREAKDOWN;
        } else if (rr <= S.stop2 || (S.ru_period > 0 && S.since_ru >= S.ru_period) || rr <= S.ru_delta2 * S.ru_rho) {
            S.flag = CG_ATTENTION;
        } else if (S.iter >= S.max_iter) {
            S.flag = CG_ATTENTION;
        } else {
            S.beta = rr / S.rho;
            S.rho = rr;
        }
    }
}

// After a reliable update: rho_true = |b - A x|^2.  mode 0: stop if below the
// target, else continue with beta = rho_true / rho.
__global__ void k_reduce_true(const double *__restrict__ part, int nb, CgState *st) {
    const int r = blockIdx.x;
    CgState &S = st[r];
    if (S.flag != CG_ATTENTION) return;
    const double rr = reduce_partials(part + (size_t)r * nb, nb);
    if (threadIdx.x == 0) {
        S.true_rr = rr;
        S.reliable += 1;
        S.since_ru = 0;
        if (!finite(rr)) {
            S.flag = CG_BREAKDOWN;
        } else if (rr <= S.true2) {
            S.flag = CG_DONE;
        } else if (S.iter >= S.max_iter) {
            S.flag = CG_MAXITER;
        } else {
            // the iterated residual claimed convergence but the true one has not
            // followed: aim the iterated residual lower (halve its target), or the
            // solve would crawl along the tolerance one reliable update at a time
            if (S.rho_new <= S.stop2) S.stop2 *= 0.25;
            // resume: the p update of this iteration uses the recomputed residual
            S.rho_new = rr;
            S.beta = rr / S.rho;
            S.rho = rr;
            S.ru_rho = rr;
            S.flag = CG_RESUME;
        }
    }
}

// Initial: rho = |r|^2 for every RHS whose flag is CG_ATTENTION (set by the host).
__global__ void k_reduce_init(const double *__restrict__ part, int nb, CgState *st) {
    const int r = blockIdx.x;
    CgState &S = st[r];
    const double rr = reduce_partials(part + (size_t)r * nb, nb);
    if (threadIdx.x == 0) {
        S.true_rr = rr;
        S.rho = rr;
        S.ru_rho = rr;
        if (!finite(rr)) {
            S.flag = CG_BREAKDOWN;
        } else if (rr <= S.true2) {
            S.flag = CG_DONE;
        } else {
            S.flag = CG_RUNNING;
        }
    }
}

__global__ void k_resume_flags(CgState *st) {
    CgState &S = st[blockIdx.x];
    if (threadIdx.x == 0 && S.flag == CG_RESUME) S.flag = CG_RUNNING;
}

// ---------------------------------------------------------------- per-site kernels
template <int F>
using RT = typename RealOf<F>::T;

// x += alpha p ; r -= alpha q ; partial |r|^2
template <int FX, int FR, int FP, int FQ>
__global__ __launch_bounds__(256) void k_update_xr(Spinor<FX> x, Spinor<FR> r, Spinor<FP> p,
                                                   Spinor<FQ> q, const CgState *__restrict__ st,
                                                   double *__restrict__ part) {
    const int i = blockIdx.y;
    const int nb = gridDim.x;
    if (st[i].flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    typedef RT<FX> R;
    double rr = 0.0;
    if (h < x.vh) {
        const R a = (R)st[i].alpha;
        cx<RT<FX>> xv[3];
        cx<RT<FR>> rv[3];
        cx<RT<FP>> pv[3];
        cx<RT<FQ>> qv[3];
        const Spinor<FX> X = x.rhs(i);
        const Spinor<FR> Rr = r.rhs(i);
        X.load(h, xv);
        Rr.load(h, rv);
        p.rhs(i).load(h, pv);
        q.rhs(i).load(h, qv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += a * (R)pv[c].re;
            xv[c].im += a * (R)pv[c].im;
            rv[c].re -= (RT<FR>)a * (RT<FR>)qv[c].re;
            rv[c].im -= (RT<FR>)a * (RT<FR>)qv[c].im;
            rr += (double)rv[c].re * (double)rv[c].re + (double)rv[c].im * (double)rv[c].im;
        }
        X.store(h, xv);
        Rr.store(h, rv);
    }
    const double s = block_sum(rr);
    if (threadIdx.x == 0) part[(size_t)i * nb + blockIdx.x] = s;
}

// r -= alpha q ; partial |r|^2   (running RHS)
template <int FR, int FQ>
__global__ __launch_bounds__(256) void k_update_r(Spinor<FR> r, Spinor<FQ> q, const CgState *__restrict__ st,
                                                  double *__restrict__ part) {
    const int i = blockIdx.y;
    const int nb = gridDim.x;
    if (st[i].flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (h < r.vh) {
        typedef RT<FR> R;
        const R a = (R)st[i].alpha;
        cx<R> rv[3];
        cx<RT<FQ>> qv[3];
        const Spinor<FR> Rr = r.rhs(i);
        Rr.load(h, rv);
        q.rhs(i).load(h, qv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rv[c].re -= a * (R)qv[c].re;
            rv[c].im -= a * (R)qv[c].im;
            rr += (double)rv[c].re * (double)rv[c].re + (double)rv[c].im * (double)rv[c].im;
        }
        Rr.store(h, rv);
    }
    const double s = block_sum(rr);
    if (threadIdx.x == 0) part[(size_t)i * nb + blockIdx.x] = s;
}

// x += alpha p (if this iteration's alpha is pending), then p = r + beta p
// (if the RHS is still running): x, p and r read once
template <int FX, int FR, int FP>
__global__ __launch_bounds__(256) void k_update_xp(Spinor<FX> x, Spinor<FR> r, Spinor<FP> p,
                                                   const CgState *__restrict__ st) {
    const int i = blockIdx.y;
    const bool upd_x = st[i].xpend != 0, upd_p = st[i].flag == CG_RUNNING;
    if (!upd_x && !upd_p) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= p.vh) return;
    typedef RT<FX> RX;
    typedef RT<FP> RP;
    cx<RP> pv[3];
    const Spinor<FP> P = p.rhs(i);
    P.load(h, pv);
    if (upd_x) {
        const RX a = (RX)st[i].alpha;
        cx<RX> xv[3];
        const Spinor<FX> X = x.rhs(i);
        X.load(h, xv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += a * (RX)pv[c].re;
            xv[c].im += a * (RX)pv[c].im;
        }
        X.store(h, xv);
    }
    if (upd_p) {
        const RP b = (RP)st[i].beta;
        cx<RT<FR>> rv[3];
        r.rhs(i).load(h, rv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pv[c].re = (RP)rv[c].re + b * pv[c].re;
            pv[c].im = (RP)rv[c].im + b * pv[c].im;
        }
        P.store(h, pv);
    }
}

// p = r + beta p   (for RHS whose flag equals `when`)
template <int FR, int FP>
__global__ __launch_bounds__(256) void k_update_p(Spinor<FR> r, Spinor<FP> p,
                                                  const CgState *__restrict__ st, int when) {
    const int i = blockIdx.y;
    if (st[i].flag != when) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= p.vh) return;
    typedef RT<FP> R;
    const R b = (R)st[i].beta;
    cx<RT<FR>> rv[3];
    cx<R> pv[3];
    r.rhs(i).load(h, rv);
    const Spinor<FP> P = p.rhs(i);
    P.load(h, pv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pv[c].re = (R)rv[c].re + b * pv[c].re;
        pv[c].im = (R)rv[c].im + b * pv[c].im;
    }
    P.store(h, pv);
}

// dst = src (format conversion) for RHS whose flag equals `when` (or all if when < 0)
template <int FS, int FD>
__global__ __launch_bounds__(256) void k_convert(Spinor<FS> src, Spinor<FD> dst,
                                                 const CgState *__restrict__ st, int when) {
    const int i = blockIdx.y;
    if (when >= 0 && st[i].flag != when) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= dst.vh) return;
    cx<RT<FS>> a[3];
    cx<RT<FD>> b[3];
    src.rhs(i).load(h, a);
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c] = {(RT<FD>)a[c].re, (RT<FD>)a[c].im};
    dst.rhs(i).store(h, b);
}

// xhi += xs ; xs = 0   (RHS with flag == when)
template <int FS>
__global__ __launch_bounds__(256) void k_accum_zero(Spinor<F64> xhi, Spinor<FS> xs,
                                                    const CgState *__restrict__ st, int when) {
    const int i = blockIdx.y;
    if (st[i].flag != when) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= xhi.vh) return;
    cx<double> a[3];
    cx<RT<FS>> b[3];
    const Spinor<F64> X = xhi.rhs(i);
    const Spinor<FS> S = xs.rhs(i);
    X.load(h, a);
    S.load(h, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c].re += (double)b[c].re;
        a[c].im += (double)b[c].im;
        b[c] = {(RT<FS>)0, (RT<FS>)0};
    }
    X.store(h, a);
    S.store(h, b);
}

// r = b - Ax, partial |r|^2  (RHS with flag == when, or all if when < 0)
__global__ __launch_bounds__(256) void k_residual(Spinor<F64> b, Spinor<F64> ax, Spinor<F64> r,
                                                  const CgState *__restrict__ st, int when,
                                                  double *__restrict__ part) {
    const int i = blockIdx.y;
    const int nb = gridDim.x;
    if (when >= 0 && st[i].flag != when) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (h < r.vh) {
        cx<double> bv[3], av[3];
        b.rhs(i).load(h, bv);
        ax.rhs(i).load(h, av);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            av[c] = {bv[c].re - av[c].re, bv[c].im - av[c].im};
            rr += av[c].re * av[c].re + av[c].im * av[c].im;
        }
        r.rhs(i).store(h, av);
    }
    const double s = block_sum(rr);
    if (threadIdx.x == 0) part[(size_t)i * nb + blockIdx.x] = s;
}

// partial |v|^2 for every RHS
__global__ __launch_bounds__(256) void k_norm2(Spinor<F64> v, double *__restrict__ part) {
    const int i = blockIdx.y;
    const int nb = gridDim.x;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (h < v.vh) {
        cx<double> a[3];
        v.rhs(i).load(h, a);
#pragma unroll
        for (int c = 0; c < 3; ++c) rr += a[c].re * a[c].re + a[c].im * a[c].im;
    }
    const double s = block_sum(rr);
    if (threadIdx.x == 0) part[(size_t)i * nb + blockIdx.x] = s;
}

// final sums into out[i] (no scalar logic)
__global__ void k_reduce_store(const double *__restrict__ part, int nb, double *out) {
    const double s = reduce_partials(part + (size_t)blockIdx.x * nb, nb);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// v = 0 for every RHS (fill kernel: safe inside captured graphs)
template <int F>
__global__ __launch_bounds__(256) void k_zero(Spinor<F> v) {
    const int i = blockIdx.y;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= v.vh) return;
    cx<RT<F>> z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) z[c] = {(RT<F>)0, (RT<F>)0};
    v.rhs(i).store(h, z);
}

// ---------------------------------------------------------------- host wrappers
static inline dim3 site_grid(int vh, int nrhs) { return dim3((vh + 255) / 256, nrhs); }
int blas_blocks(int vh) { return (vh + 255) / 256; }

#define SPIN(F, ptr) spinor_view<F>((void *)(ptr), vh)

template <int FX, int FR, int FP, int FQ>
static void upd_xr(int vh, int n, void *x, void *r, const void *p, const void *q, const CgState *st,
                   double *part, hipStream_t s) {
    hipLaunchKernelGGL((k_update_xr<FX, FR, FP, FQ>), site_grid(vh, n), dim3(256), 0, s, SPIN(FX, x),
                       SPIN(FR, r), SPIN(FP, p), SPIN(FQ, q), st, part);
}

void launch_update_xr(int fmt_sloppy, int vh, int n, void *x, void *r, const void *p, const void *q,
                      const CgState *st, double *part, hipStream_t s) {
    switch (fmt_sloppy) {
        case F64: upd_xr<F64, F64, F64, F64>(vh, n, x, r, p, q, st, part, s); break;
        case F32: upd_xr<F32, F32, F32, F32>(vh, n, x, r, p, q, st, part, s); break;
        // FP16S sloppy: x, r, q kept in FP32, p (the Dslash input) in FP16S
        default: upd_xr<F32, F32, H16, F32>(vh, n, x, r, p, q, st, part, s); break;
    }
}

void launch_update_r(int fmt_sloppy, int vh, int n, void *r, const void *q, const CgState *st, double *part,
                     hipStream_t s) {
    if (fmt_sloppy == F64)
        hipLaunchKernelGGL((k_update_r<F64, F64>), site_grid(vh, n), dim3(256), 0, s, SPIN(F64, r), SPIN(F64, q), st,
                           part);
    else  // FP32 and FP16S sloppy: r and q in FP32
        hipLaunchKernelGGL((k_update_r<F32, F32>), site_grid(vh, n), dim3(256), 0, s, SPIN(F32, r), SPIN(F32, q), st,
                           part);
}

void launch_update_xp(int fmt_sloppy, int vh, int n, void *x, const void *r, void *p, const CgState *st,
                      hipStream_t s) {
    switch (fmt_sloppy) {
        case F64:
            hipLaunchKernelGGL((k_update_xp<F64, F64, F64>), site_grid(vh, n), dim3(256), 0, s, SPIN(F64, x),
                               SPIN(F64, r), SPIN(F64, p), st);
            break;
        case F32:
            hipLaunchKernelGGL((k_update_xp<F32, F32, F32>), site_grid(vh, n), dim3(256), 0, s, SPIN(F32, x),
                               SPIN(F32, r), SPIN(F32, p), st);
            break;
        default:  // FP16S sloppy: x and r in FP32, p (the Dslash input) in FP16S
            hipLaunchKernelGGL((k_update_xp<F32, F32, H16>), site_grid(vh, n), dim3(256), 0, s, SPIN(F32, x),
                               SPIN(F32, r), SPIN(H16, p), st);
            break;
    }
}

void launch_update_p(int fmt_sloppy, int vh, int n, const void *r, void *p, const CgState *st, int when,
                     hipStream_t s) {
    switch (fmt_sloppy) {
        case F64:
            hipLaunchKernelGGL((k_update_p<F64, F64>), site_grid(vh, n), dim3(256), 0, s, SPIN(F64, r),
                               SPIN(F64, p), st, when);
            break;
        case F32:
            hipLaunchKernelGGL((k_update_p<F32, F32>), site_grid(vh, n), dim3(256), 0, s, SPIN(F32, r),
                               SPIN(F32, p), st, when);
            break;
        default:
            hipLaunchKernelGGL((k_update_p<F32, H16>), site_grid(vh, n), dim3(256), 0, s, SPIN(F32, r),
                               SPIN(H16, p), st, when);
            break;
    }
}

template <int FS, int FD>
static void conv(int vh, int n, const void *src, void *dst, const CgState *st, int when, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<FS, FD>), site_grid(vh, n), dim3(256), 0, s, SPIN(FS, src),
                       SPIN(FD, dst), st, when);
}

int launch_convert(int fs, int fd, int vh, int n, const void *src, void *dst, const CgState *st, int when,
                   hipStream_t s) {
#define CV(a, b) \
    if (fs == a && fd == b) { conv<a, b>(vh, n, src, dst, st, when, s); return 0; }
    CV(F64, F64) CV(F64, F32) CV(F64, H16) CV(F32, F64) CV(F32, F32) CV(F32, H16) CV(H16, F64)
    CV(H16, F32) CV(H16, H16)
#undef CV
    return -1;
}

void launch_accum_zero(int fmt_x, int vh, int n, void *xhi, void *xs, const CgState *st, int when,
                       hipStream_t s) {
    if (fmt_x == F64)
        hipLaunchKernelGGL((k_accum_zero<F64>), site_grid(vh, n), dim3(256), 0, s, SPIN(F64, xhi),
                           SPIN(F64, xs), st, when);
    else
        hipLaunchKernelGGL((k_accum_zero<F32>), site_grid(vh, n), dim3(256), 0, s, SPIN(F64, xhi),
                           SPIN(F32, xs), st, when);
}

void launch_residual(int vh, int n, const void *b, const void *ax, void *r, const CgState *st, int when,
                     double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_residual, site_grid(vh, n), dim3(256), 0, s, SPIN(F64, b), SPIN(F64, ax),
                       SPIN(F64, r), st, when, part);
}

void launch_norm2(int vh, int n, const void *v, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, site_grid(vh, n), dim3(256), 0, s, SPIN(F64, v), part);
}

void launch_zero(int fmt, int vh, int n, void *v, hipStream_t s) {
    switch (fmt) {
        case F64: hipLaunchKernelGGL(k_zero<F64>, site_grid(vh, n), dim3(256), 0, s, SPIN(F64, v)); break;
        case F32: hipLaunchKernelGGL(k_zero<F32>, site_grid(vh, n), dim3(256), 0, s, SPIN(F32, v)); break;
        default: hipLaunchKernelGGL(k_zero<H16>, site_grid(vh, n), dim3(256), 0, s, SPIN(H16, v)); break;
    }
}

void launch_reduce(int which, int n, const double *part, int nb, CgState *st, double *out, hipStream_t s) {
    switch (which) {
        case RED_ALPHA: hipLaunchKernelGGL(k_reduce_alpha, dim3(n), dim3(256), 0, s, part, nb, st); break;
        case RED_BETA: hipLaunchKernelGGL(k_reduce_beta, dim3(n), dim3(256), 0, s, part, nb, st); break;
        case RED_TRUE: hipLaunchKernelGGL(k_reduce_true, dim3(n), dim3(256), 0, s, part, nb, st); break;
        case RED_INIT: hipLaunchKernelGGL(k_reduce_init, dim3(n), dim3(256), 0, s, part, nb, st); break;
        case RED_STORE: hipLaunchKernelGGL(k_reduce_store, dim3(n), dim3(256), 0, s, part, nb, out); break;
        default: break;
    }
}

void launch_resume_flags(int n, CgState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_resume_flags, dim3(n), dim3(64), 0, s, st);
}

}  // namespace hisq
