// Flexible CG with the network preconditioner (Notay, SIAM J. Sci. Comput. 22
// (2000), FCG with one stored direction):
//   q = A p ; alpha = <p, r> / <p, q> ; x += alpha p ; r -= alpha q ;
//   z = N(r) ; beta = -<q, z> / <q, p> ; p = z + beta p
// with complex alpha and beta, since the preconditioner need not be Hermitian.
// The iteration runs in FP32.  Every ru_period iterations, and whenever the
// iterated residual reaches the target, a reliable update folds the FP32
// solution into the FP64 one and recomputes r = b - A x in FP64; the direction
// then continues (z = N(r), beta against the last p, q), as mixed-precision CG
// does after its reliable updates.  A breakdown, or a true residual that fails
// to halve over three reliable updates, hands the solve to plain FP64 CG from
// the current x.  Chunks of iterations are captured once into a hipGraph and
// replayed; scalars and the stop flag live in device memory.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "nn_internal.h"

namespace hisq {

int nn_forward(hisq_nn_s *n, const float *in, float *out, hipStream_t s);

// The CgState prefix carries flag / counters / <p, A p> (as pap), so the
// Dslash's per-RHS skip test works on this state unchanged.
struct FcgState {
    CgState cg;
    double pr_re, pr_im;  // <p, r>
    double qz_re, qz_im;  // <q, z>
    double al_re, al_im;  // alpha
    double be_re, be_im;  // beta
    double rr;            // |r|^2 of the FP32 residual
};

__device__ __forceinline__ double block_sum2(double v) {
    __shared__ double red[8];
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ double reduce_fixed(const double *p, int n, int stride) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[(size_t)i * stride];
    return block_sum2(s);
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && fabs(v) <= 1.7e308; }

// per-block partial <u, v> = sum conj(u) v as (re, im)
__global__ __launch_bounds__(256) void k_cdot(Spinor<F32> u, Spinor<F32> v, const FcgState *st, double *part) {
    if (st->cg.flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double re = 0.0, im = 0.0;
    if (h < u.vh) {
        cx<float> a[3], b[3];
        u.load(h, a);
        v.load(h, b);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            re += (double)a[c].re * b[c].re + (double)a[c].im * b[c].im;
            im += (double)a[c].re * b[c].im - (double)a[c].im * b[c].re;
        }
    }
    re = block_sum2(re);
    im = block_sum2(im);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = re;
        part[2 * blockIdx.x + 1] = im;
    }
}

// alpha = <p, r> / <p, q>;  <p, q> comes from the Dslash epilogue partials
__global__ void k_fcg_alpha(const double *pq_part, int nbq, const double *pr_part, int nbr, FcgState *st) {
    if (st->cg.flag != CG_RUNNING) return;
    const double pq = reduce_fixed(pq_part, nbq, 1);
    const double pre = reduce_fixed(pr_part, nbr, 2);
    const double pim = reduce_fixed(pr_part + 1, nbr, 2);
    if (threadIdx.x == 0) {
        st->cg.pap = pq;
        st->pr_re = pre;
        st->pr_im = pim;
        if (!(pq > 0.0) || !finite_d(pq) || !finite_d(pre) || !finite_d(pim)) {
            st->cg.flag = CG_BREAKDOWN;
        } else {
            st->al_re = pre / pq;
            st->al_im = pim / pq;
        }
    }
}

// x += alpha p ; r -= alpha q ; partial |r|^2
__global__ __launch_bounds__(256) void k_fcg_xr(Spinor<F32> x, Spinor<F32> r, Spinor<F32> p, Spinor<F32> q,
                                               const FcgState *st, double *part) {
    if (st->cg.flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (h < x.vh) {
        const float ar = (float)st->al_re, ai = (float)st->al_im;
        cx<float> xv[3], rv[3], pv[3], qv[3];
        x.load(h, xv);
        r.load(h, rv);
        p.load(h, pv);
        q.load(h, qv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += ar * pv[c].re - ai * pv[c].im;
            xv[c].im += ar * pv[c].im + ai * pv[c].re;
            rv[c].re -= ar * qv[c].re - ai * qv[c].im;
            rv[c].im -= ar * qv[c].im + ai * qv[c].re;
            rr += (double)rv[c].re * rv[c].re + (double)rv[c].im * rv[c].im;
        }
        x.store(h, xv);
        r.store(h, rv);
    }
    rr = block_sum2(rr);
    if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

// |r|^2 -> iteration count, convergence / reliable-update / cap flags
__global__ void k_fcg_check(const double *part, int nb, FcgState *st) {
    if (st->cg.flag != CG_RUNNING) return;
    const double rr = reduce_fixed(part, nb, 1);
    if (threadIdx.x == 0) {
        CgState &c = st->cg;
        st->rr = rr;
        c.iter += 1;
        c.since_ru += 1;
        if (!finite_d(rr)) c.flag = CG_BREAKDOWN;
        else if (rr <= c.stop2 || c.since_ru >= c.ru_period || c.iter >= c.max_iter) c.flag = CG_ATTENTION;
    }
}

// beta = -<q, z> / <q, p>, with <q, p> = <p, q> real (A Hermitian)
__global__ void k_fcg_beta(const double *qz_part, int nb, FcgState *st) {
    if (st->cg.flag != CG_RUNNING) return;
    const double re = reduce_fixed(qz_part, nb, 2);
    const double im = reduce_fixed(qz_part + 1, nb, 2);
    if (threadIdx.x == 0) {
        st->qz_re = re;
        st->qz_im = im;
        if (!finite_d(re) || !finite_d(im)) {
            st->cg.flag = CG_BREAKDOWN;
        } else {
            st->be_re = -re / st->cg.pap;
            st->be_im = -im / st->cg.pap;
        }
    }
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_fcg_p(Spinor<F32> z, Spinor<F32> p, const FcgState *st) {
    if (st->cg.flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= p.vh) return;
    const float br = (float)st->be_re, bi = (float)st->be_im;
    cx<float> zv[3], pv[3];
    z.load(h, zv);
    p.load(h, pv);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float pr = pv[c].re, pi = pv[c].im;
        pv[c].re = zv[c].re + br * pr - bi * pi;
        pv[c].im = zv[c].im + br * pi + bi * pr;
    }
    p.store(h, pv);
}

// p = z (first direction; p's old contents are never read)
__global__ __launch_bounds__(256) void k_copy32(Spinor<F32> z, Spinor<F32> p) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= p.vh) return;
    cx<float> zv[3];
    z.load(h, zv);
    p.store(h, zv);
}

// x64 += x32 ; x32 = 0
__global__ __launch_bounds__(256) void k_fold_x(Spinor<F64> xhi, Spinor<F32> xs) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= xhi.vh) return;
    cx<double> a[3];
    cx<float> b[3];
    xhi.load(h, a);
    xs.load(h, b);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c].re += b[c].re;
        a[c].im += b[c].im;
        b[c] = {0.f, 0.f};
    }
    xhi.store(h, a);
    xs.store(h, b);
}

FcgWorkspace::~FcgWorkspace() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
}

static int fcg_ws_get(hisq_gauge_s *g, FcgWorkspace **out) {
    if (!g->fcg_ws) g->fcg_ws.reset(new (std::nothrow) FcgWorkspace());
    if (!g->fcg_ws) {
        set_error("flexible CG: host allocation failed");
        return HISQ_ERR_OOM;
    }
    FcgWorkspace &w = *g->fcg_ws;
    const int vh = g->geom.vh;
    const size_t s64 = spinor_bytes(F64, vh), s32 = spinor_bytes(F32, vh);
    const int nb = blas_blocks(vh);
    int rc;
    for (DevBuf *bf : {&w.b64, &w.x64, &w.r64, &w.t64, &w.ax64})
        if ((rc = bf->alloc(s64))) return rc;
    for (DevBuf *bf : {&w.xs, &w.rs, &w.ps, &w.qs, &w.zs, &w.ts})
        if ((rc = bf->alloc(s32))) return rc;
    if ((rc = w.part.alloc(sizeof(double) * 2 * ((vh + 63) / 64))) || (rc = w.part2.alloc(sizeof(double) * 2 * nb)) ||
        (rc = w.state.alloc(sizeof(FcgState))) || (rc = w.diag.alloc(sizeof(double))) ||
        (rc = w.scal.alloc(sizeof(double) * 2)))
        return rc;
    *out = &w;
    return HISQ_OK;
}

// ax64 = A x64 in FP64
static int fcg_A64(hisq_gauge_s *g, FcgWorkspace &w, hipStream_t s) {
    int rc;
    if ((rc = gauge_dslash(g, 1, F64, F64, F64, 1, w.x64.p, w.t64.p, nullptr, nullptr, nullptr, nullptr, s))) return rc;
    return gauge_dslash(g, 0, F64, F64, F64, 1, w.t64.p, w.ax64.p, w.x64.p, (const double *)w.diag.p,
                        (double *)w.part.p, nullptr, s);
}

// |b - A x64|^2 into r64 (and returned), synchronous
static int fcg_true_residual(hisq_gauge_s *g, FcgWorkspace &w, double *tr, hipStream_t s) {
    const int vh = g->geom.vh, nb = blas_blocks(vh);
    int rc;
    if ((rc = fcg_A64(g, w, s))) return rc;
    launch_residual(vh, 1, w.b64.p, w.ax64.p, w.r64.p, nullptr, -1, (double *)w.part2.p, s);
    launch_reduce(RED_STORE, 1, (double *)w.part2.p, nb, nullptr, (double *)w.scal.p, s);
    HISQ_HIP_CHECK(hipMemcpyAsync(tr, w.scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    return HISQ_OK;
}

// One FCG iteration (every kernel idles once the flag leaves CG_RUNNING).
static int fcg_iteration(hisq_gauge_s *g, hisq_nn_s *net, FcgWorkspace &w, hipStream_t s) {
    const int vh = g->geom.vh, nb = blas_blocks(vh);
    FcgState *st = (FcgState *)w.state.p;
    const CgState *skip = &st->cg;
    Spinor<F32> X = spinor_view<F32>(w.xs.p, vh), R = spinor_view<F32>(w.rs.p, vh), P = spinor_view<F32>(w.ps.p, vh),
                Q = spinor_view<F32>(w.qs.p, vh), Z = spinor_view<F32>(w.zs.p, vh);
    double *part2 = (double *)w.part2.p;
    int rc;
    if ((rc = gauge_dslash(g, 1, F32, F32, F32, 1, w.ps.p, w.ts.p, nullptr, nullptr, nullptr, skip, s))) return rc;
    if ((rc = gauge_dslash(g, 0, F32, F32, F32, 1, w.ts.p, w.qs.p, w.ps.p, (const double *)w.diag.p,
                           (double *)w.part.p, skip, s)))
        return rc;
    hipLaunchKernelGGL(k_cdot, dim3(nb), dim3(256), 0, s, P, R, st, part2);
    hipLaunchKernelGGL(k_fcg_alpha, dim3(1), dim3(256), 0, s, (const double *)w.part.p,
                       nb_dslash(g, F32, F32, F32, 1, true), (const double *)part2, nb, st);
    hipLaunchKernelGGL(k_fcg_xr, dim3(nb), dim3(256), 0, s, X, R, P, Q, st, part2);
    hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(256), 0, s, (const double *)part2, nb, st);
    if ((rc = nn_forward(net, (const float *)w.rs.p, (float *)w.zs.p, s))) return rc;
    hipLaunchKernelGGL(k_cdot, dim3(nb), dim3(256), 0, s, Q, Z, st, part2);
    hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(256), 0, s, (const double *)part2, nb, st);
    hipLaunchKernelGGL(k_fcg_p, dim3(nb), dim3(256), 0, s, Z, P, st);
    return HISQ_OK;
}

static int fcg_run_chunk(hisq_gauge_s *g, hisq_nn_s *net, FcgWorkspace &w, int chunk, bool use_graph,
                         hipStream_t s) {
    int rc;
    if (!use_graph) {
        for (int i = 0; i < chunk; ++i)
            if ((rc = fcg_iteration(g, net, w, s))) return rc;
        HISQ_HIP_CHECK(hipGetLastError());
        return HISQ_OK;
    }
    // a captured graph holds the network's buffers: rebuild it for another network
    if (w.exec && (w.net_id != net->id || w.chunk != chunk)) {
        (void)hipGraphExecDestroy(w.exec);
        (void)hipGraphDestroy(w.graph);
        w.exec = nullptr;
        w.graph = nullptr;
    }
    if (!w.exec) {
        hipStream_t cs = g->capture_stream;
        HISQ_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < chunk; ++i) {
            if ((rc = fcg_iteration(g, net, w, cs))) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(cs, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                return rc;
            }
        }
        HISQ_HIP_CHECK(hipStreamEndCapture(cs, &w.graph));
        HISQ_HIP_CHECK(hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0));
        w.net_id = net->id;
        w.chunk = chunk;
    }
    HISQ_HIP_CHECK(hipGraphLaunch(w.exec, s));
    return HISQ_OK;
}

int fcg_solve(hisq_gauge_s *g, double mass, const double *b, double *x, const hisq_solver_params &prm,
              hisq_solver_stats *stats, hipStream_t s) {
    TraceRange tr_("flexible CG");
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    hisq_nn_s *net = (hisq_nn_s *)prm.precond;
    if (net->gauge != g) {
        set_error("the preconditioner network belongs to another gauge handle");
        return HISQ_ERR_INVALID;
    }
    if (!g->links[F64][0].p || !g->links[F32][0].p) {
        set_error("flexible CG needs packed FP64 and FP32 links");
        return HISQ_ERR_UNSUPPORTED;
    }
    if (!g->thin.p) {
        set_error("flexible CG: the gauge handle has no thin links (hisq_gauge_set_thin)");
        return HISQ_ERR_UNSUPPORTED;
    }
    const int vh = g->geom.vh, nb = blas_blocks(vh);
    const size_t s64 = spinor_bytes(F64, vh);
    FcgWorkspace *wp = nullptr;
    int rc = fcg_ws_get(g, &wp);
    if (rc) return rc;
    FcgWorkspace &w = *wp;
    FcgState *st = (FcgState *)w.state.p;
    const double diag = 4.0 * mass * mass;
    HISQ_HIP_CHECK(hipMemcpyAsync(w.diag.p, &diag, sizeof(double), hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(w.b64.p, b, s64, hipMemcpyDeviceToDevice, s));
    if (prm.warm_start) HISQ_HIP_CHECK(hipMemcpyAsync(w.x64.p, x, s64, hipMemcpyDeviceToDevice, s));
    else launch_zero(F64, vh, 1, w.x64.p, s);
    launch_zero(F32, vh, 1, w.xs.p, s);
    launch_norm2(vh, 1, w.b64.p, (double *)w.part2.p, s);
    launch_reduce(RED_STORE, 1, (double *)w.part2.p, nb, nullptr, (double *)w.scal.p, s);
    double b2 = 0;
    HISQ_HIP_CHECK(hipMemcpyAsync(&b2, w.scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));

    // HISQ_SOLVER_TRACE=1 prints the reliable update at the start, after every
    // 2000 iterations and at convergence to stderr
    static const bool trace = std::getenv("HISQ_SOLVER_TRACE") != nullptr;
    int next_report = 2000;
    FcgState hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.cg.stop2 = kResidualMargin * kResidualMargin * prm.tol * prm.tol * b2;  // iterated-residual trigger (tightened below)
    hs.cg.true2 = hs.cg.stop2;             // target of the true residual
    hs.cg.ru_period = std::max(1, prm.ru_period);
    hs.cg.max_iter = prm.max_iter;
    // host checks between chunks land on periodic reliable updates: the chunk
    // is the largest divisor of ru_period not above graph_chunk (10 if eager)
    const bool use_graph = prm.graph_chunk > 0;
    const int cap = use_graph ? prm.graph_chunk : 10;
    int chunk = 1;
    for (int c = std::min(cap, hs.cg.ru_period); c >= 1; --c)
        if (hs.cg.ru_period % c == 0) {
            chunk = c;
            break;
        }

    int status = HISQ_OK, stagnant = 0;
    double best_true = 1e300;
    bool fallback = false, broke = false;  // hand over to plain CG; the reason was a breakdown
    bool first = true;
    while (true) {
        // reliable update: fold x, r = b - A x in FP64, decide
        double tr = 0;
        if (!first)
            hipLaunchKernelGGL(k_fold_x, dim3(nb), dim3(256), 0, s, spinor_view<F64>(w.x64.p, vh),
                               spinor_view<F32>(w.xs.p, vh));
        if (!first && hs.cg.flag == CG_BREAKDOWN) {
            if (trace)
                std::fprintf(stderr, "[fcg] breakdown at iter %d: pq %.3e <p,r> %.3e%+.3ei <q,z> %.3e%+.3ei\n",
                             hs.cg.iter, hs.cg.pap, hs.pr_re, hs.pr_im, hs.qz_re, hs.qz_im);
            fallback = broke = true;
            break;
        }
        if ((rc = fcg_true_residual(g, w, &tr, s))) return rc;
        hs.cg.reliable += 1;
        if (trace && (first || hs.cg.iter >= next_report || tr <= hs.cg.true2)) {
            std::fprintf(stderr, "[fcg] iter %d reliable %d |r|/|b| true %.3e iterated %.3e\n", hs.cg.iter,
                         hs.cg.reliable, std::sqrt(tr / std::max(b2, 1e-300)),
                         std::sqrt(std::max(hs.rr, 0.0) / std::max(b2, 1e-300)));
            next_report = (hs.cg.iter / 2000 + 1) * 2000;
        }
        if (!std::isfinite(tr)) {
            fallback = broke = true;
            break;
        }
        if (tr <= hs.cg.true2) break;
        // the iterated residual claimed convergence but the true one has not
        // followed: aim the iterated residual lower
        if (!first && hs.rr <= hs.cg.stop2) hs.cg.stop2 *= 0.25;
        if (tr < 0.5 * best_true) {
            best_true = tr;
            stagnant = 0;
        } else if (++stagnant >= 3) {
            if (trace) std::fprintf(stderr, "[fcg] stagnation at iter %d\n", hs.cg.iter);
            fallback = true;
            break;
        }
        if (hs.cg.iter >= hs.cg.max_iter) {
            status = HISQ_NOT_CONVERGED;
            break;
        }
        // continue from the corrected residual
        if ((rc = launch_convert(F64, F32, vh, 1, w.r64.p, w.rs.p, nullptr, -1, s))) return rc;
        if ((rc = nn_forward(net, (const float *)w.rs.p, (float *)w.zs.p, s))) return rc;
        hs.cg.flag = CG_RUNNING;
        hs.cg.since_ru = 0;
        HISQ_HIP_CHECK(hipMemcpyAsync(st, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
        if (first) {
            hipLaunchKernelGGL(k_copy32, dim3(nb), dim3(256), 0, s, spinor_view<F32>(w.zs.p, vh),
                               spinor_view<F32>(w.ps.p, vh));
        } else {
            Spinor<F32> Q = spinor_view<F32>(w.qs.p, vh), Z = spinor_view<F32>(w.zs.p, vh),
                        P = spinor_view<F32>(w.ps.p, vh);
            hipLaunchKernelGGL(k_cdot, dim3(nb), dim3(256), 0, s, Q, Z, st, (double *)w.part2.p);
            hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(256), 0, s, (const double *)w.part2.p, nb, st);
            hipLaunchKernelGGL(k_fcg_p, dim3(nb), dim3(256), 0, s, Z, P, st);
        }
        first = false;
        // iterate until the device asks for the host
        do {
            if ((rc = fcg_run_chunk(g, net, w, chunk, use_graph, s))) return rc;
            HISQ_HIP_CHECK(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
            HISQ_HIP_CHECK(hipStreamSynchronize(s));
        } while (hs.cg.flag == CG_RUNNING);
    }
    const int fcg_iters = hs.cg.iter, fcg_ru = hs.cg.reliable;
    HISQ_HIP_CHECK(hipMemcpyAsync(x, w.x64.p, s64, hipMemcpyDeviceToDevice, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    hisq_solver_stats cg_st;
    std::memset(&cg_st, 0, sizeof(cg_st));
    if (fallback && prm.fallback) {
        hisq_solver_params cp = prm;
        cp.precond = nullptr;
        cp.warm_start = 1;
        cp.sloppy_prec = HISQ_PREC_FP64;
        rc = cg_solve(g, mass, 1, b, x, nullptr, cp, &cg_st, s);
        if (rc < 0) return rc;
        status = rc == HISQ_OK ? HISQ_CONVERGED_AFTER_FALLBACK : rc;
        HISQ_HIP_CHECK(hipMemcpyAsync(w.x64.p, x, s64, hipMemcpyDeviceToDevice, s));
    } else if (fallback) {
        status = broke ? HISQ_BREAKDOWN : HISQ_NOT_CONVERGED;
    }
    // final FP64 true residual of what x holds
    double tr = 0;
    if ((rc = fcg_true_residual(g, w, &tr, s))) return rc;
    const double rel = b2 > 0 ? std::sqrt(tr / b2) : std::sqrt(tr);
    if (status == HISQ_OK && !(rel <= prm.tol)) status = HISQ_NOT_CONVERGED;
    if (stats) {
        stats->status = status;
        stats->iterations = fcg_iters + cg_st.iterations;
        stats->reliable_updates = fcg_ru + cg_st.reliable_updates;
        stats->fallback_used = fallback && prm.fallback;
        stats->true_residual = rel;
        stats->wall_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        stats->dslash_bytes =
            (double)fcg_iters * (double)(dslash_algorithmic_bytes(F32, F32, F32, vh, 1, false, g->comp_mode) +
                                         dslash_algorithmic_bytes(F32, F32, F32, vh, 1, true, g->comp_mode)) +
            (double)(fcg_ru + 1) * (double)(dslash_algorithmic_bytes(F64, F64, F64, vh, 1, false, g->comp_mode) +
                                            dslash_algorithmic_bytes(F64, F64, F64, vh, 1, true, g->comp_mode)) +
            cg_st.dslash_bytes;
    }
    return status;
}

}  // namespace hisq
