// Multi-shift CG (Jegerlehner, hep-lat/9612014): one Krylov space of the base
// system A + sigma_0 (sigma_0 = smallest shift) serves every shifted system
// A + sigma_k, because the shifted residuals stay collinear with the base
// residual, r_k = zeta_k r.  Per iteration and shift, with D_k = sigma_k -
// sigma_0 and the previous base coefficients alpha', beta':
//   zeta_k'' = zeta_k zeta_k' alpha' / ( alpha beta' (zeta_k' - zeta_k)
//                                        + zeta_k' alpha' (1 + alpha D_k) )
//   alpha_k  = alpha zeta_k'' / zeta_k
//   beta_k   = beta (zeta_k'' / zeta_k)^2
//   x_k += alpha_k p_k ;  p_k = zeta_k'' r + beta_k p_k
// (zeta' = value of the previous iteration, zeta'' = of the next).  A shift
// stops once |zeta_k''| |r| <= tol |b|.  Afterwards every shift's FP64 true
// residual is checked by a batched CG warm-started from the multi-shift
// solution, which also refines any shift that has not reached the target.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "solver_internal.h"

namespace hisq {

struct MsState {
    double delta;      // sigma_k - sigma_0
    double zeta;       // zeta_k of the current iteration
    double zeta_old;   // of the previous iteration
    double zeta_new;   // of the next iteration
    double alpha, beta;
    int active;        // still iterating
    int stop_next;     // converged: leaves after this iteration's update
    int pending;       // alpha_k computed but x_k not yet updated
    int iters;         // iterations in which this shift was updated
};

struct MsGlobal {
    double alpha_old, beta_old, stop;  // stop = tol |b|
};

// Several sources (nsrc) run in lockstep: source j = blockIdx.y has its own
// base state base[j], shift states ms[j][k] and globals gl[j]; the vector
// stacks are shift-major, slot k * nsrc + j (so the sources' base vectors,
// k = 0, are one contiguous multi-RHS stack).

// after alpha: new zeta and alpha_k for every active shift
__global__ void k_ms_alpha(const CgState *__restrict__ base_, MsState *ms_, MsGlobal *gl_, int nshift) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    const CgState *base = base_ + j;
    MsGlobal *gl = gl_ + j;
    if (k == 0 || k >= nshift || base->flag != CG_RUNNING) return;
    MsState &S = ms_[(size_t)j * nshift + k];
    if (S.stop_next) S.active = 0;
    if (!S.active) return;
    const double a = base->alpha, ao = gl->alpha_old, bo = gl->beta_old;
    const double den = a * bo * (S.zeta_old - S.zeta) + S.zeta_old * ao * (1.0 + a * S.delta);
    S.zeta_new = S.zeta * S.zeta_old * ao / den;
    S.alpha = a * S.zeta_new / S.zeta;
    S.pending = 1;
}

// after beta: beta_k, roll the zetas, convergence of each shift (base flag ==
// when); one block per source
__global__ void k_ms_beta(const CgState *__restrict__ base_, MsState *ms_, MsGlobal *gl_, int nshift, int when) {
    const int j = blockIdx.y;
    const CgState *base = base_ + j;
    MsGlobal *gl = gl_ + j;
    if (base->flag != when) return;
    for (int k = threadIdx.x; k < nshift; k += blockDim.x) {
        if (k == 0) continue;
        MsState &S = ms_[(size_t)j * nshift + k];
        if (S.active) {
            const double ratio = S.zeta_new / S.zeta;
            S.beta = base->beta * ratio * ratio;
            S.zeta_old = S.zeta;
            S.zeta = S.zeta_new;
            S.iters += 1;
            if (fabs(S.zeta) * sqrt(base->rho_new) <= gl->stop) S.stop_next = 1;
        }
    }
    if (threadIdx.x == 0) {
        gl->alpha_old = base->alpha;
        gl->beta_old = base->beta;
    }
}

// x_k += alpha_k p_k ; p_k = zeta_k r + beta_k p_k   for every active shift, r read once
template <int F>
__global__ __launch_bounds__(256) void k_ms_update(Spinor<F> x, Spinor<F> p, Spinor<F> r,
                                                   const CgState *__restrict__ base_, const MsState *ms_,
                                                   int nshift, int nsrc, int when) {
    const int j = blockIdx.y;
    if (base_[j].flag != when) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= r.vh) return;
    const MsState *ms = ms_ + (size_t)j * nshift;
    typedef typename RealOf<F>::T R;
    cx<R> rv[3];
    r.rhs(j).load(h, rv);
    for (int k = 1; k < nshift; ++k) {
        const MsState &S = ms[k];
        if (!S.active) continue;
        const R a = (R)S.alpha, z = (R)S.zeta, bk = (R)S.beta;
        cx<R> xv[3], pv[3];
        const Spinor<F> X = x.rhs(k * nsrc + j), P = p.rhs(k * nsrc + j);
        X.load(h, xv);
        P.load(h, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += a * pv[c].re;
            xv[c].im += a * pv[c].im;
            pv[c].re = z * rv[c].re + bk * pv[c].re;
            pv[c].im = z * rv[c].im + bk * pv[c].im;
        }
        X.store(h, xv);
        P.store(h, pv);
    }
}

__global__ void k_ms_clear_pending(const CgState *__restrict__ base_, MsState *ms_, int nshift, int when) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (base_[j].flag != when || k >= nshift) return;
    ms_[(size_t)j * nshift + k].pending = 0;
}

// final x_k += alpha_k p_k for shifts whose last update is still pending
template <int F>
__global__ __launch_bounds__(256) void k_ms_flush(Spinor<F> x, Spinor<F> p, const MsState *ms_, int nshift,
                                                  int nsrc) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (h >= x.vh) return;
    const MsState *ms = ms_ + (size_t)j * nshift;
    typedef typename RealOf<F>::T R;
    for (int k = 1; k < nshift; ++k) {
        const MsState &S = ms[k];
        if (!S.pending) continue;
        const R a = (R)S.alpha;
        cx<R> xv[3], pv[3];
        const Spinor<F> X = x.rhs(k * nsrc + j);
        X.load(h, xv);
        p.rhs(k * nsrc + j).load(h, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += a * pv[c].re;
            xv[c].im += a * pv[c].im;
        }
        X.store(h, xv);
    }
}

// slot i of a stack of format F = source i % nsrc (FP64): the sources
// replicated into every shift's slots of a shift-major stack
template <int F>
__global__ __launch_bounds__(256) void k_replicate(Spinor<F64> src, Spinor<F> dst, int nsrc) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= src.vh) return;
    typedef typename RealOf<F>::T R;
    cx<double> v[3];
    src.rhs(blockIdx.y % nsrc).load(h, v);
    cx<R> w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = {(R)v[c].re, (R)v[c].im};
    dst.rhs(blockIdx.y).store(h, w);
}

struct MsWorkspace {
    DevBuf t, q, r, p0, pk, part, state, ms, gl, diag, bstack;
};

// Multi-shift CG for nsrc sources in lockstep, its Krylov iteration in
// precision K (FP32: the mixed form; FP64).  Links and vectors of the
// iteration (base residual and direction, every shifted direction and
// solution) are in K; the sources' base directions form one multi-RHS stack,
// so each link load of the Dslash serves every source.  The
// base solutions are accumulated in FP64 with reliable updates (x_hi +=
// x_sloppy, r = b - (A + sigma_0) x_hi in FP64, every ru_period iterations,
// after a tenfold fall of the iterated residual and at apparent convergence);
// after such an update the recurrences continue from the recomputed residual,
// with each shifted residual taken as zeta_k times it.  The shifted residuals
// are collinear with the base residual only up to the rounding of the K
// operator; in FP32 the shifted solutions stall far above the target (the smaller
// the shift, the higher: between ~1e-3 and ~1e-7 relative for shifts from
// 1e-4 to 10 in a model of this iteration); the batched mixed-precision CG
// warm-started from them finishes every (source, shift) on its own FP64 true
// residual.
//   b: nsrc FP64 sources [nsrc][spinor];  x: [nsrc][ns][spinor] in the
//   caller's shift order;  stats: [nsrc][ns] or NULL.
template <int K>
static int multishift_solve_lockstep(hisq_gauge_s *g, double mass, int m, int ns, const int *order,
                                     const double *shifts, const double *b, double *x,
                                     const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const int vh = g->geom.vh;
    if (!g->links[K][0].p) {
        set_error(K == F64 ? "multishift: the handle lacks packed FP64 links"
                           : "multishift: mixed precision needs packed FP32 links in the handle");
        return HISQ_ERR_UNSUPPORTED;
    }
    const double sig0 = shifts[order[0]];
    const size_t s64 = spinor_bytes(F64, vh), sk = spinor_bytes(K, vh);
    const int nb = blas_blocks(vh), nall = m * ns;
    const int nbmax = std::max((vh + 63) / 64, nb);
    DevBuf rk, tk, qk, pk, xk, x64, t64, ax64, r64, part, state, msb, glb, diag, scal, bstack;
    int rc;
    if ((rc = rk.alloc(sk * m)) || (rc = tk.alloc(sk * m)) || (rc = qk.alloc(sk * m)) ||
        (rc = pk.alloc(sk * nall)) || (rc = xk.alloc(sk * nall)) || (rc = x64.alloc(s64 * nall)) ||
        (rc = t64.alloc(s64 * m)) || (rc = ax64.alloc(s64 * m)) || (rc = r64.alloc(s64 * m)) ||
        (rc = part.alloc(sizeof(double) * (size_t)m * nbmax)) || (rc = state.alloc(sizeof(CgState) * m)) ||
        (rc = msb.alloc(sizeof(MsState) * nall)) || (rc = glb.alloc(sizeof(MsGlobal) * m)) ||
        (rc = diag.alloc(sizeof(double) * m)) || (rc = scal.alloc(sizeof(double) * m)) ||
        (rc = bstack.alloc(s64 * nall)))
        return rc;
    CgState *base = (CgState *)state.p;
    MsState *ms = (MsState *)msb.p;
    MsGlobal *gl = (MsGlobal *)glb.p;
    double *pt = (double *)part.p;
    // shift-major stacks: slot k * m + j; the base (k = 0) slots of the
    // direction, sloppy and FP64 solution stacks are the sources' base stacks
    const Spinor<K> X = spinor_view<K>(xk.p, vh), P = spinor_view<K>(pk.p, vh);
    const Spinor<K> Rv = spinor_view<K>(rk.p, vh);
    void *p0 = pk.p, *xhi = x64.p;

    const std::vector<double> diag0(m, 4.0 * mass * mass + sig0);
    HISQ_HIP_CHECK(hipMemcpyAsync(diag.p, diag0.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    launch_norm2(vh, m, b, pt, s);
    launch_reduce(RED_STORE, m, pt, nb, nullptr, (double *)scal.p, s);
    std::vector<double> b2(m);
    HISQ_HIP_CHECK(hipMemcpyAsync(b2.data(), scal.p, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));

    std::vector<CgState> hb(m);
    std::vector<MsState> hm(nall);
    std::vector<MsGlobal> hg(m);
    for (int j = 0; j < m; ++j) {
        CgState &c = hb[j];
        std::memset(&c, 0, sizeof(c));
        c.stop2 = kResidualMargin * kResidualMargin * prm.tol * prm.tol * b2[j];
        c.true2 = c.stop2;
        c.ru_period = std::max(1, prm.ru_period);
        c.ru_delta2 = prm.ru_delta * prm.ru_delta;
        c.max_iter = prm.max_iter;
        c.flag = CG_ATTENTION;
        for (int k = 0; k < ns; ++k) {
            MsState &S = hm[(size_t)j * ns + k];
            std::memset(&S, 0, sizeof(MsState));
            S.delta = shifts[order[k]] - sig0;
            S.zeta = S.zeta_old = S.zeta_new = 1.0;
            S.active = 1;
        }
        hg[j] = MsGlobal{1.0, 0.0, prm.tol * std::sqrt(b2[j])};
    }
    HISQ_HIP_CHECK(hipMemcpyAsync(base, hb.data(), sizeof(CgState) * m, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(ms, hm.data(), sizeof(MsState) * nall, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(gl, hg.data(), sizeof(MsGlobal) * m, hipMemcpyHostToDevice, s));

    // r = b, p = p_k = b, x_k = 0, x_hi = 0
    launch_convert(F64, K, vh, m, b, rk.p, nullptr, -1, s);
    launch_norm2(vh, m, b, pt, s);
    launch_reduce(RED_INIT, m, pt, nb, base, nullptr, s);
    launch_zero(K, vh, nall, xk.p, s);
    launch_zero(F64, vh, m, xhi, s);
    const dim3 rep_grid((vh + 255) / 256, nall);
    hipLaunchKernelGGL(k_replicate<K>, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh), P, m);
    HISQ_HIP_CHECK(hipGetLastError());

    const int tb = 64;
    const dim3 shift_grid((ns + tb - 1) / tb, m), site_grid((vh + 255) / 256, m), beta_grid(1, m);
    const dim3 beta_block(std::max(64, std::min(256, ((ns + 63) / 64) * 64)));
    auto iteration = [&](hipStream_t st) -> int {
        int r2;
        if ((r2 = gauge_dslash(g, 1, K, K, K, m, p0, tk.p, nullptr, nullptr, nullptr, base, st))) return r2;
        if ((r2 = gauge_dslash(g, 0, K, K, K, m, tk.p, qk.p, p0, (const double *)diag.p, pt, base, st)))
            return r2;
        launch_reduce(RED_ALPHA, m, pt, nb_dslash(g, K, K, K, m, true), base, nullptr, st);
        hipLaunchKernelGGL(k_ms_alpha, shift_grid, dim3(tb), 0, st, base, ms, gl, ns);
        launch_update_xr(K, vh, m, xk.p, rk.p, p0, qk.p, base, pt, st);
        launch_reduce(RED_BETA, m, pt, nb, base, nullptr, st);
        hipLaunchKernelGGL(k_ms_beta, beta_grid, beta_block, 0, st, base, ms, gl, ns, (int)CG_RUNNING);
        hipLaunchKernelGGL(k_ms_update<K>, site_grid, dim3(256), 0, st, X, P, Rv, base, ms, ns, m,
                           (int)CG_RUNNING);
        hipLaunchKernelGGL(k_ms_clear_pending, shift_grid, dim3(tb), 0, st, base, ms, ns, (int)CG_RUNNING);
        launch_update_p(K, vh, m, rk.p, p0, base, CG_RUNNING, st);
        return (int)(hipGetLastError() == hipSuccess ? HISQ_OK : HISQ_ERR_HIP);
    };
    // FP64 reliable update of the base systems flagged CG_ATTENTION
    auto reliable = [&]() -> int {
        int r2;
        launch_accum_zero(K, vh, m, xhi, xk.p, base, CG_ATTENTION, s);
        if ((r2 = gauge_dslash(g, 1, F64, F64, F64, m, xhi, t64.p, nullptr, nullptr, nullptr, nullptr, s))) return r2;
        if ((r2 = gauge_dslash(g, 0, F64, F64, F64, m, t64.p, ax64.p, xhi, (const double *)diag.p, pt, nullptr, s)))
            return r2;
        launch_residual(vh, m, b, ax64.p, r64.p, base, CG_ATTENTION, pt, s);
        launch_reduce(RED_TRUE, m, pt, nb, base, nullptr, s);
        launch_convert(F64, K, vh, m, r64.p, rk.p, base, CG_RESUME, s);
        // the shifts' beta and direction updates of this iteration, from the new residual
        hipLaunchKernelGGL(k_ms_beta, beta_grid, beta_block, 0, s, base, ms, gl, ns, (int)CG_RESUME);
        hipLaunchKernelGGL(k_ms_update<K>, site_grid, dim3(256), 0, s, X, P, Rv, base, ms, ns, m,
                           (int)CG_RESUME);
        hipLaunchKernelGGL(k_ms_clear_pending, shift_grid, dim3(tb), 0, s, base, ms, ns, (int)CG_RESUME);
        launch_update_p(K, vh, m, rk.p, p0, base, CG_RESUME, s);
        launch_resume_flags(m, base, s);
        return (int)(hipGetLastError() == hipSuccess ? HISQ_OK : HISQ_ERR_HIP);
    };

    const int chunk = std::max(1, prm.graph_chunk > 0 ? prm.graph_chunk : 8);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const bool use_graph = prm.graph_chunk > 0;
    rc = HISQ_OK;
    if (use_graph) {
        hipStream_t cs = g->capture_stream;
        HISQ_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < chunk && rc == HISQ_OK; ++i) rc = iteration(cs);
        hipError_t e = hipStreamEndCapture(cs, &graph);
        if (rc == HISQ_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (!rc) set_error(std::string("multishift graph: ") + hipGetErrorString(e));
            return rc ? rc : HISQ_ERR_HIP;
        }
    }
    const long max_chunks = 2L * prm.max_iter + 16;  // chunk replays and reliable updates
    for (long c = 0; c < max_chunks && rc == HISQ_OK; ++c) {
        HISQ_HIP_CHECK(hipMemcpyAsync(hb.data(), base, sizeof(CgState) * m, hipMemcpyDeviceToHost, s));
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        bool attention = false, running = false;
        for (const CgState &cj : hb) {
            attention |= cj.flag == CG_ATTENTION;
            running |= cj.flag == CG_RUNNING;
        }
        if (attention) {
            rc = reliable();
            continue;
        }
        if (!running) break;
        if (use_graph) {
            if (hipGraphLaunch(exec, s) != hipSuccess) rc = HISQ_ERR_HIP;
        } else {
            for (int i = 0; i < chunk && rc == HISQ_OK; ++i) rc = iteration(s);
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    HISQ_HIP_CHECK(hipMemcpyAsync(hb.data(), base, sizeof(CgState) * m, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    // a breakdown or a stop at the cap leaves a base's sloppy part unfolded
    for (int f : {(int)CG_BREAKDOWN, (int)CG_MAXITER}) launch_accum_zero(K, vh, m, xhi, xk.p, base, f, s);
    hipLaunchKernelGGL(k_ms_flush<K>, site_grid, dim3(256), 0, s, X, P, ms, ns, m);
    HISQ_HIP_CHECK(hipMemcpyAsync(hm.data(), ms, sizeof(MsState) * nall, hipMemcpyDeviceToHost, s));
    if (ns > 1)
        launch_convert(K, F64, vh, nall - m, (char *)xk.p + sk * m, (char *)x64.p + s64 * m, nullptr, -1, s);

    // every (source, shift) finished on its FP64 true residual by the batched mixed CG
    static const bool trace = std::getenv("HISQ_SOLVER_TRACE") != nullptr;
    if (trace) {
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        int it = 0, ru = 0;
        for (const CgState &cj : hb) {
            it = std::max(it, cj.iter);
            ru += cj.reliable;
        }
        std::fprintf(stderr, "[multishift] %s: %d source(s) x %d shifts, %d base iterations, %d reliable updates, %.3f s\n",
                     K == F64 ? "FP64 lockstep" : "mixed", m, ns, it, ru, std::chrono::duration<double>(clk::now() - t0).count());
    }
    hipLaunchKernelGGL(k_replicate<F64>, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh),
                       spinor_view<F64>(bstack.p, vh), m);
    HISQ_HIP_CHECK(hipGetLastError());
    std::vector<double> sig(nall);
    for (int k = 0; k < ns; ++k)
        for (int j = 0; j < m; ++j) sig[(size_t)k * m + j] = shifts[order[k]];
    hisq_solver_params rp = prm;
    rp.warm_start = 1;
    std::vector<hisq_solver_stats> rs(nall);
    int worst = cg_solve(g, mass, nall, (const double *)bstack.p, (double *)x64.p, sig.data(), rp, rs.data(), s);
    if (worst < 0) return worst;
    for (int k = 0; k < ns; ++k)
        for (int j = 0; j < m; ++j)
            HISQ_HIP_CHECK(hipMemcpyAsync((char *)x + s64 * ((size_t)j * ns + order[k]),
                                          (char *)x64.p + s64 * ((size_t)k * m + j), s64, hipMemcpyDeviceToDevice, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    const double total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (trace) {
        int most = 0;
        for (const hisq_solver_stats &r : rs) most = std::max(most, r.iterations);
        std::fprintf(stderr, "[multishift] refinement: at most %d iterations, total %.3f s\n", most, total_ms / 1e3);
    }
    if (stats) {
        const double per_iter = (double)(dslash_algorithmic_bytes(K, K, K, vh, m, false, g->comp_mode) +
                                         dslash_algorithmic_bytes(K, K, K, vh, m, true, g->comp_mode));
        const double per_ru = (double)(dslash_algorithmic_bytes(F64, F64, F64, vh, 1, false, g->comp_mode) +
                                       dslash_algorithmic_bytes(F64, F64, F64, vh, 1, true, g->comp_mode));
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < ns; ++k) {
                const hisq_solver_stats &r = rs[(size_t)k * m + j];
                hisq_solver_stats o = r;
                o.iterations = (k == 0 ? hb[j].iter : hm[(size_t)j * ns + k].iters) + r.iterations;
                o.wall_ms = total_ms;
                o.reliable_updates = (k == 0 ? hb[j].reliable : 0) + r.reliable_updates;
                o.dslash_bytes =
                    ((double)hb[j].iter * per_iter / m + (double)hb[j].reliable * per_ru) / ns + r.dslash_bytes;
                stats[(size_t)j * ns + order[k]] = o;
            }
    }
    return worst;
}

int multishift_solve(hisq_gauge_s *g, double mass, int ns, const double *shifts, const double *b, double *x,
                     const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const Geom &G = g->geom;
    const int vh = G.vh;
    if (!g->links[F64][0].p) {
        set_error("multishift: the handle lacks packed FP64 links");
        return HISQ_ERR_UNSUPPORTED;
    }
    // order: base = smallest shift placed in slot 0 of the internal ordering
    std::vector<int> order(ns);
    for (int k = 0; k < ns; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return shifts[a] < shifts[c]; });
    if (prm.sloppy_prec != HISQ_PREC_FP64)
        return multishift_solve_lockstep<F32>(g, mass, 1, ns, order.data(), shifts, b, x, prm, stats, s);
    const double sig0 = shifts[order[0]];

    const size_t s64 = spinor_bytes(F64, vh);
    MsWorkspace w;
    int rc;
    const int nb = blas_blocks(vh);
    if ((rc = w.t.alloc(s64)) || (rc = w.q.alloc(s64)) || (rc = w.r.alloc(s64)) || (rc = w.pk.alloc(s64 * ns)) ||
        (rc = w.part.alloc(sizeof(double) * ((vh + 63) / 64))) || (rc = w.state.alloc(sizeof(CgState))) ||
        (rc = w.ms.alloc(sizeof(MsState) * ns)) || (rc = w.gl.alloc(sizeof(MsGlobal))) ||
        (rc = w.diag.alloc(sizeof(double))) || (rc = w.bstack.alloc(s64 * ns)))
        return rc;
    // internal x stack in sorted order: reuse bstack later; solutions go to a temp stack
    DevBuf xs;
    if ((rc = xs.alloc(s64 * ns))) return rc;
    Spinor<F64> X = spinor_view<F64>(xs.p, vh), P = spinor_view<F64>(w.pk.p, vh);
    Spinor<F64> Rv = spinor_view<F64>(w.r.p, vh);
    CgState *base = (CgState *)w.state.p;
    MsState *ms = (MsState *)w.ms.p;
    MsGlobal *gl = (MsGlobal *)w.gl.p;

    const double diag0 = 4.0 * mass * mass + sig0;
    HISQ_HIP_CHECK(hipMemcpyAsync(w.diag.p, &diag0, sizeof(double), hipMemcpyHostToDevice, s));
    launch_norm2(vh, 1, b, (double *)w.part.p, s);
    DevBuf scal;
    if ((rc = scal.alloc(sizeof(double)))) return rc;
    launch_reduce(RED_STORE, 1, (double *)w.part.p, nb, nullptr, (double *)scal.p, s);
    double b2 = 0;
    HISQ_HIP_CHECK(hipMemcpyAsync(&b2, scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));

    CgState hb;
    std::memset(&hb, 0, sizeof(hb));
    hb.stop2 = kResidualMargin * kResidualMargin * prm.tol * prm.tol * b2;
    hb.true2 = hb.stop2;
    hb.max_iter = prm.max_iter;
    hb.flag = CG_ATTENTION;
    std::vector<MsState> hm(ns);
    for (int k = 0; k < ns; ++k) {
        std::memset(&hm[k], 0, sizeof(MsState));
        hm[k].delta = shifts[order[k]] - sig0;
        hm[k].zeta = hm[k].zeta_old = hm[k].zeta_new = 1.0;
        hm[k].active = 1;
    }
    MsGlobal hg{1.0, 0.0, prm.tol * std::sqrt(b2)};
    HISQ_HIP_CHECK(hipMemcpyAsync(base, &hb, sizeof(hb), hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(ms, hm.data(), sizeof(MsState) * ns, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(gl, &hg, sizeof(hg), hipMemcpyHostToDevice, s));

    // r = b, p = p_k = b, x_k = 0
    HISQ_HIP_CHECK(hipMemcpyAsync(w.r.p, b, s64, hipMemcpyDeviceToDevice, s));
    launch_norm2(vh, 1, w.r.p, (double *)w.part.p, s);
    launch_reduce(RED_INIT, 1, (double *)w.part.p, nb, base, nullptr, s);
    launch_zero(F64, vh, ns, xs.p, s);
    const dim3 rep_grid((vh + 255) / 256, ns);
    hipLaunchKernelGGL(k_replicate<F64>, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh), P, 1);
    HISQ_HIP_CHECK(hipGetLastError());

    const int chunk = std::max(1, prm.graph_chunk > 0 ? prm.graph_chunk : 8);
    const int nb_d0 = nb_dslash(g, F64, F64, F64, 1, true);
    auto iteration = [&](hipStream_t st) -> int {
        int r2;
        void *p0 = w.pk.p;  // base direction lives in slot 0 of the p stack
        if ((r2 = gauge_dslash(g, 1, F64, F64, F64, 1, p0, w.t.p, nullptr, nullptr, nullptr, base, st))) return r2;
        if ((r2 = gauge_dslash(g, 0, F64, F64, F64, 1, w.t.p, w.q.p, p0, (const double *)w.diag.p,
                               (double *)w.part.p, base, st)))
            return r2;
        launch_reduce(RED_ALPHA, 1, (double *)w.part.p, nb_d0, base, nullptr, st);
        const int tb = 64, gb = (ns + tb - 1) / tb;
        hipLaunchKernelGGL(k_ms_alpha, dim3(gb), dim3(tb), 0, st, base, ms, gl, ns);
        launch_update_xr(F64, vh, 1, xs.p, w.r.p, p0, w.q.p, base, (double *)w.part.p, st);
        launch_reduce(RED_BETA, 1, (double *)w.part.p, nb, base, nullptr, st);
        hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(std::max(64, ((ns + 63) / 64) * 64)), 0, st, base, ms,
                           gl, ns, (int)CG_RUNNING);
        hipLaunchKernelGGL(k_ms_update<F64>, dim3((vh + 255) / 256), dim3(256), 0, st, X, P, Rv, base, ms, ns, 1,
                           (int)CG_RUNNING);
        hipLaunchKernelGGL(k_ms_clear_pending, dim3(gb), dim3(tb), 0, st, base, ms, ns, (int)CG_RUNNING);
        launch_update_p(F64, vh, 1, w.r.p, p0, base, CG_RUNNING, st);
        return (int)(hipGetLastError() == hipSuccess ? HISQ_OK : HISQ_ERR_HIP);
    };

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const bool use_graph = prm.graph_chunk > 0;
    if (use_graph) {
        hipStream_t cs = g->capture_stream;
        HISQ_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < chunk && rc == HISQ_OK; ++i) rc = iteration(cs);
        hipError_t e = hipStreamEndCapture(cs, &graph);
        if (rc == HISQ_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (!rc) set_error(std::string("multishift graph: ") + hipGetErrorString(e));
            return rc ? rc : HISQ_ERR_HIP;
        }
    }
    int iters_total = 0;
    for (long c = 0; c < (long)prm.max_iter / chunk + 2; ++c) {
        HISQ_HIP_CHECK(hipMemcpyAsync(&hb, base, sizeof(hb), hipMemcpyDeviceToHost, s));
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        if (hb.flag != CG_RUNNING) break;
        if (use_graph) {
            HISQ_HIP_CHECK(hipGraphLaunch(exec, s));
        } else {
            for (int i = 0; i < chunk; ++i)
                if ((rc = iteration(s))) return rc;
        }
    }
    iters_total = hb.iter;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    hipLaunchKernelGGL(k_ms_flush<F64>, dim3((vh + 255) / 256), dim3(256), 0, s, X, P, ms, ns, 1);
    HISQ_HIP_CHECK(hipMemcpyAsync(hm.data(), ms, sizeof(MsState) * ns, hipMemcpyDeviceToHost, s));

    // FP64 verification and refinement of every shift: batched CG warm-started
    // from the multi-shift solutions (converged shifts leave at once).
    Spinor<F64> Bs = spinor_view<F64>(w.bstack.p, vh);
    hipLaunchKernelGGL(k_replicate<F64>, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh), Bs, 1);
    std::vector<double> sig(ns);
    for (int k = 0; k < ns; ++k) sig[k] = shifts[order[k]];
    hisq_solver_params rp = prm;
    rp.sloppy_prec = HISQ_PREC_FP64;
    rp.warm_start = 1;
    std::vector<hisq_solver_stats> rs(ns);
    int worst = cg_solve(g, mass, ns, (const double *)w.bstack.p, (double *)xs.p, sig.data(), rp, rs.data(), s);
    if (worst < 0) return worst;
    // scatter back to the caller's order
    for (int k = 0; k < ns; ++k)
        HISQ_HIP_CHECK(hipMemcpyAsync((char *)x + s64 * order[k], (char *)xs.p + s64 * k, s64,
                                      hipMemcpyDeviceToDevice, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    const double total_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    if (stats) {
        for (int k = 0; k < ns; ++k) {
            hisq_solver_stats o = rs[k];
            o.iterations = (k == 0 ? iters_total : hm[k].iters) + rs[k].iterations;
            o.wall_ms = total_ms;
            o.reliable_updates = rs[k].reliable_updates;
            o.dslash_bytes = (double)iters_total * (double)(dslash_algorithmic_bytes(F64, F64, F64, vh, 1, false, g->comp_mode) +
                                                            dslash_algorithmic_bytes(F64, F64, F64, vh, 1, true, g->comp_mode)) /
                                 ns +
                             rs[k].dslash_bytes;
            stats[order[k]] = o;
        }
    }
    return worst;
}

// nsrc sources, each with every shift, run in lockstep (one source: the
// single-source solver).  With FP64 sloppy precision the Krylov vectors are
// FP64 as well; the reliable updates then only re-anchor the iterated residual
// on the true one every ru_period iterations.
int multishift_solve_batched(hisq_gauge_s *g, double mass, int nsrc, int ns, const double *shifts, const double *b,
                             double *x, const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s) {
    if (nsrc == 1) return multishift_solve(g, mass, ns, shifts, b, x, prm, stats, s);
    std::vector<int> order(ns);
    for (int k = 0; k < ns; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return shifts[a] < shifts[c]; });
    if (prm.sloppy_prec != HISQ_PREC_FP64)
        return multishift_solve_lockstep<F32>(g, mass, nsrc, ns, order.data(), shifts, b, x, prm, stats, s);
    return multishift_solve_lockstep<F64>(g, mass, nsrc, ns, order.data(), shifts, b, x, prm, stats, s);
}

}  // namespace hisq
