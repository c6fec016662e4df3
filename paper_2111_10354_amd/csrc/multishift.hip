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

// after alpha: new zeta and alpha_k for every active shift
__global__ void k_ms_alpha(const CgState *__restrict__ base, MsState *ms, MsGlobal *gl, int nshift) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 || k >= nshift || base->flag != CG_RUNNING) return;
    MsState &S = ms[k];
    if (S.stop_next) S.active = 0;
    if (!S.active) return;
    const double a = base->alpha, ao = gl->alpha_old, bo = gl->beta_old;
    const double den = a * bo * (S.zeta_old - S.zeta) + S.zeta_old * ao * (1.0 + a * S.delta);
    S.zeta_new = S.zeta * S.zeta_old * ao / den;
    S.alpha = a * S.zeta_new / S.zeta;
    S.pending = 1;
}

// after beta: beta_k, roll the zetas, convergence of each shift
__global__ void k_ms_beta(const CgState *__restrict__ base, MsState *ms, MsGlobal *gl, int nshift) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (base->flag != CG_RUNNING) return;
    if (k < nshift && k > 0) {
        MsState &S = ms[k];
        if (S.active) {
            const double ratio = S.zeta_new / S.zeta;
            S.beta = base->beta * ratio * ratio;
            S.zeta_old = S.zeta;
            S.zeta = S.zeta_new;
            S.iters += 1;
            if (fabs(S.zeta) * sqrt(base->rho_new) <= gl->stop) S.stop_next = 1;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        gl->alpha_old = base->alpha;
        gl->beta_old = base->beta;
    }
}

// x_k += alpha_k p_k ; p_k = zeta_k r + beta_k p_k   for every active shift, r read once
__global__ __launch_bounds__(256) void k_ms_update(Spinor<F64> x, Spinor<F64> p, Spinor<F64> r,
                                                   const CgState *__restrict__ base, MsState *ms,
                                                   int nshift) {
    if (base->flag != CG_RUNNING) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= r.vh) return;
    cx<double> rv[3];
    r.load(h, rv);
    for (int k = 1; k < nshift; ++k) {
        const MsState &S = ms[k];
        if (!S.active) continue;
        cx<double> xv[3], pv[3];
        const Spinor<F64> X = x.rhs(k), P = p.rhs(k);
        X.load(h, xv);
        P.load(h, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += S.alpha * pv[c].re;
            xv[c].im += S.alpha * pv[c].im;
            pv[c].re = S.zeta * rv[c].re + S.beta * pv[c].re;
            pv[c].im = S.zeta * rv[c].im + S.beta * pv[c].im;
        }
        X.store(h, xv);
        P.store(h, pv);
    }
}

__global__ void k_ms_clear_pending(const CgState *__restrict__ base, MsState *ms, int nshift) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (base->flag != CG_RUNNING || k >= nshift) return;
    ms[k].pending = 0;
}

// final x_k += alpha_k p_k for shifts whose last update is still pending
__global__ __launch_bounds__(256) void k_ms_flush(Spinor<F64> x, Spinor<F64> p, const MsState *ms,
                                                  int nshift) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= x.vh) return;
    for (int k = 1; k < nshift; ++k) {
        const MsState &S = ms[k];
        if (!S.pending) continue;
        cx<double> xv[3], pv[3];
        const Spinor<F64> X = x.rhs(k);
        X.load(h, xv);
        p.rhs(k).load(h, pv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c].re += S.alpha * pv[c].re;
            xv[c].im += S.alpha * pv[c].im;
        }
        X.store(h, xv);
    }
}

// b replicated into every slot of a stack
__global__ __launch_bounds__(256) void k_replicate(Spinor<F64> src, Spinor<F64> dst) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= src.vh) return;
    cx<double> v[3];
    src.load(h, v);
    dst.rhs(blockIdx.y).store(h, v);
}

struct MsWorkspace {
    DevBuf t, q, r, p0, pk, part, state, ms, gl, diag, bstack;
};

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
    hb.stop2 = prm.tol * prm.tol * b2;
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
    hipLaunchKernelGGL(k_replicate, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh), P);
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
                           gl, ns);
        hipLaunchKernelGGL(k_ms_update, dim3((vh + 255) / 256), dim3(256), 0, st, X, P, Rv, base, ms, ns);
        hipLaunchKernelGGL(k_ms_clear_pending, dim3(gb), dim3(tb), 0, st, base, ms, ns);
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
    hipLaunchKernelGGL(k_ms_flush, dim3((vh + 255) / 256), dim3(256), 0, s, X, P, ms, ns);
    HISQ_HIP_CHECK(hipMemcpyAsync(hm.data(), ms, sizeof(MsState) * ns, hipMemcpyDeviceToHost, s));

    // FP64 verification and refinement of every shift: batched CG warm-started
    // from the multi-shift solutions (converged shifts leave at once).
    Spinor<F64> Bs = spinor_view<F64>(w.bstack.p, vh);
    hipLaunchKernelGGL(k_replicate, rep_grid, dim3(256), 0, s, spinor_view<F64>((void *)b, vh), Bs);
    std::vector<double> sig(ns);
    for (int k = 0; k < ns; ++k) sig[k] = shifts[order[k]];
    hisq_solver_params rp = prm;
    rp.sloppy_prec = HISQ_PREC_FP64;
    rp.warm_start = 1;
    std::vector<hisq_solver_stats> rs(ns);
    const double ms_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
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
            o.dslash_bytes = (double)iters_total * (double)(dslash_algorithmic_bytes(F64, F64, F64, vh, 1, false, g->compressed) +
                                                            dslash_algorithmic_bytes(F64, F64, F64, vh, 1, true, g->compressed)) /
                                 ns +
                             rs[k].dslash_bytes;
            stats[order[k]] = o;
        }
    }
    (void)ms_ms;
    return worst;
}

}  // namespace hisq
