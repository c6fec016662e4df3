// CG drivers: plain FP64 CG and mixed-precision CG with FP64 reliable updates,
// for one or many right-hand sides in lockstep.
//
// One iteration on the device (per running RHS i):
//   t   = D_oe p                      (Dslash, sloppy precision)
//   q   = diag_i p - D_eo t           (Dslash epilogue) and partial Re<p, q>
//   alpha = rho / Re<p, q>            (single-block reduction, device scalars)
//   r  -= alpha q                     and partial |r|^2
//   rho' = |r|^2 ; flag if |r| <= tol|b|, a reliable update is due or the cap
//   x  += alpha p ; p = r + (rho'/rho) p   (one pass; p only if still running)
// A chunk of such iterations is captured once into a hipGraph and replayed;
// flagged RHS turn every later kernel of the chunk into a no-op.  Between
// chunks the host looks at the per-RHS flags and, for flagged RHS, performs
// the reliable update in FP64: x_hi += x_sloppy, r = b - A x_hi, and either
// stops (true residual below target) or resumes with the recomputed residual
// (Sleijpen and van der Vorst's reliable updates, as used for mixed-precision
// lattice solvers by Clark et al. 2010).

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "solver_internal.h"

namespace hisq {

int DevBuf::alloc(size_t n) {
    if (p && bytes >= n) return HISQ_OK;
    if (p) {
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    if (n == 0) return HISQ_OK;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        set_error(std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? HISQ_ERR_OOM : HISQ_ERR_HIP;
    }
    bytes = n;
    return HISQ_OK;
}

static size_t real_bytes(int f) { return f == F64 ? 8 : f == F32 ? 4 : 2; }

size_t dslash_algorithmic_bytes(int fl, int fi, int fo, int64_t vh, int nrhs, bool epi, int comp) {
    if (fl == F64) comp = COMP_NONE;
    const size_t links = comp == COMP_SIGN    ? (8 * 18 + 8 * 12) * real_bytes(fl) + 4
                         : comp == COMP_KAPPA ? (8 * 18 + 8 * 12 + 8 * 2) * real_bytes(fl)
                                              : 16 * 18 * real_bytes(fl);
    const size_t per_rhs = spinor_bytes(fi, 1) + spinor_bytes(fo, 1) + (epi ? spinor_bytes(fi, 1) : 0);
    return (size_t)vh * (links + (size_t)nrhs * per_rhs);
}

DslashShape pick_shape(hisq_gauge_s *g, int fl, int fi, int fo, int nrhs, bool epi) {
    auto it = g->shapes.find(std::make_tuple(fl, fi, fo, nrhs, (int)epi));
    if (it != g->shapes.end()) return it->second;
    DslashShape s;
    const int maxt = (fl == F64) ? 4 : 8;
    s.tile = 1;
    while (s.tile * 2 <= std::min(nrhs, maxt)) s.tile *= 2;
    // measured on the 96^3 x 24 FP32 Dslash: 128-thread blocks are best for one RHS
    s.block = s.tile == 1 ? 128 : 256;
    return s;
}

int gauge_dslash(hisq_gauge_s *g, int out_parity, int fl, int fi, int fo, int nrhs, const void *in,
                 void *out, const void *y, const double *diag_dev, double *partials, const CgState *skip,
                 hipStream_t s) {
    const void *links = g->links[fl][out_parity].p;
    if (!links) {
        set_error("links of this precision were not packed (prec_mask)");
        return HISQ_ERR_UNSUPPORTED;
    }
    const DslashShape sh = pick_shape(g, fl, fi, fo, nrhs, diag_dev != nullptr);
    DslashLaunch a{};
    a.links = links;
    a.in = in;
    a.out = out;
    a.y = y;
    a.diag = diag_dev;
    a.partials = partials;
    a.skip = skip;
    a.nrhs = nrhs;
    a.parity = out_parity;
    a.fmt_links = fl;
    a.fmt_in = fi;
    a.fmt_out = fo;
    a.tile = sh.tile;
    a.block = sh.block;
    a.order = sh.order;
    a.compressed = links_compressed(g, fl);
    return launch_dslash(g->geom, a, s);
}

// ------------------------------------------------------------------ workspace
static int ws_alloc(CgWorkspace &w, const Geom &g, int n, int fmt) {
    const size_t s64 = spinor_bytes(F64, g.vh) * n;
    int rc;
    for (DevBuf *b : {&w.b64, &w.x64, &w.r64, &w.t64, &w.ax64})
        if ((rc = b->alloc(s64))) return rc;
    if (fmt == F64) {
        if ((rc = w.p64.alloc(s64)) || (rc = w.q64.alloc(s64))) return rc;
    } else {
        const size_t s32 = spinor_bytes(F32, g.vh) * n, sp = spinor_bytes(fmt, g.vh) * n;
        if ((rc = w.xs.alloc(s32)) || (rc = w.rs.alloc(s32)) || (rc = w.qs.alloc(s32)) ||
            (rc = w.ps.alloc(sp)) || (rc = w.ts.alloc(sp)))
            return rc;
    }
    const int nbmax = (g.vh + 63) / 64;  // enough for any block size >= 64
    if ((rc = w.part.alloc(sizeof(double) * (size_t)n * nbmax))) return rc;
    if ((rc = w.state.alloc(sizeof(CgState) * n))) return rc;
    if ((rc = w.diag.alloc(sizeof(double) * n))) return rc;
    if ((rc = w.scal.alloc(sizeof(double) * n))) return rc;
    w.n = n;
    w.cap = n;
    w.fmt = fmt;
    return HISQ_OK;
}

int nb_dslash(hisq_gauge_s *g, int fl, int fi, int fo, int n, bool epi) {
    const DslashShape sh = pick_shape(g, fl, fi, fo, n, epi);
    return dslash_grid_blocks(g->geom, sh.block, sh.order);
}

// One CG iteration for every running RHS of the workspace.
static int cg_iteration(hisq_gauge_s *g, CgWorkspace &w, hipStream_t s) {
    const int S = w.fmt, LF = w.lfmt, n = w.n, vh = g->geom.vh;
    const int fq = (S == H16) ? F32 : S;
    int rc;
    if ((rc = gauge_dslash(g, 1, LF, S, S, n, w.P(), w.T(), nullptr, nullptr, nullptr, w.st(), s))) return rc;
    if ((rc = gauge_dslash(g, 0, LF, S, fq, n, w.T(), w.Q(), w.P(), (const double *)w.diag.p,
                           (double *)w.part.p, w.st(), s)))
        return rc;
    launch_reduce(RED_ALPHA, n, (double *)w.part.p, nb_dslash(g, LF, S, fq, n, true), w.st(), nullptr, s);
    launch_update_r(S, vh, n, w.R(), w.Q(), w.st(), (double *)w.part.p, s);
    launch_reduce(RED_BETA, n, (double *)w.part.p, blas_blocks(vh), w.st(), nullptr, s);
    // x += alpha p with the direction of this iteration, in the pass that
    // replaces p (each of x, p, r read once)
    launch_update_xp(S, vh, n, w.X(), w.R(), w.P(), w.st(), s);
    return HISQ_OK;
}

// ax64 = (A + sigma) x64 for every RHS, in FP64.
static int apply_A64(hisq_gauge_s *g, CgWorkspace &w, const void *x, void *ax, hipStream_t s) {
    int rc;
    if ((rc = gauge_dslash(g, 1, F64, F64, F64, w.n, x, w.t64.p, nullptr, nullptr, nullptr, nullptr, s)))
        return rc;
    return gauge_dslash(g, 0, F64, F64, F64, w.n, w.t64.p, ax, x, (const double *)w.diag.p,
                        (double *)w.part.p, nullptr, s);
}

// Reliable update for RHS flagged CG_ATTENTION.
static int cg_reliable(hisq_gauge_s *g, CgWorkspace &w, hipStream_t s) {
    TraceRange tr_("cg reliable update");
    const int S = w.fmt, n = w.n, vh = g->geom.vh;
    int rc;
    if (S != F64) launch_accum_zero(F32, vh, n, w.x64.p, w.xs.p, w.st(), CG_ATTENTION, s);
    if ((rc = apply_A64(g, w, w.x64.p, w.ax64.p, s))) return rc;
    launch_residual(vh, n, w.b64.p, w.ax64.p, w.r64.p, w.st(), CG_ATTENTION, (double *)w.part.p, s);
    launch_reduce(RED_TRUE, n, (double *)w.part.p, blas_blocks(vh), w.st(), nullptr, s);
    if (S != F64) launch_convert(F64, F32, vh, n, w.r64.p, w.rs.p, w.st(), CG_RESUME, s);
    launch_update_p(S, vh, n, w.R(), w.P(), w.st(), CG_RESUME, s);
    launch_resume_flags(n, w.st(), s);
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

static int run_chunk(hisq_gauge_s *g, CgWorkspace &w, int chunk, bool use_graph, hipStream_t s) {
    int rc;
    if (!use_graph) {
        for (int i = 0; i < chunk; ++i)
            if ((rc = cg_iteration(g, w, s))) return rc;
        HISQ_HIP_CHECK(hipGetLastError());
        return HISQ_OK;
    }
    auto &gr = w.graphs[w.n];
    if (!gr.second) {
        hipStream_t cs = g->capture_stream;
        HISQ_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < chunk; ++i) {
            if ((rc = cg_iteration(g, w, cs))) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(cs, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                return rc;
            }
        }
        HISQ_HIP_CHECK(hipStreamEndCapture(cs, &gr.first));
        HISQ_HIP_CHECK(hipGraphInstantiate(&gr.second, gr.first, nullptr, nullptr, 0));
        w.chunk = chunk;
    }
    HISQ_HIP_CHECK(hipGraphLaunch(gr.second, s));
    return HISQ_OK;
}

// Compaction of a batched solve: once few enough RHS are still running, the
// finished ones leave the batch (their solutions go to the
// caller's x) and the running ones move to the lowest slots, so that the
// multi-RHS Dslash and the vector kernels stop paying for finished RHS (a
// Dslash workgroup runs as long as any RHS of its tile group is running).
// slot_of[j] is the caller's index of slot j; hs holds the slots' states.
static int cg_compact(hisq_gauge_s *g, CgWorkspace &w, std::vector<int> &slot_of, const std::vector<CgState> &hs,
                      std::vector<CgState> &fin, const std::vector<double> &diag, double *x, hipStream_t s) {
    const int vh = g->geom.vh, S = w.fmt;
    const size_t s64 = spinor_bytes(F64, vh), s32 = spinor_bytes(F32, vh), sp = spinor_bytes(S, vh);
    // a breakdown in mixed precision leaves a sloppy partial solution
    if (S != F64) launch_accum_zero(F32, vh, w.n, w.x64.p, w.xs.p, w.st(), CG_BREAKDOWN, s);
    auto cp = [&](DevBuf &b, size_t bytes, int to, int from) -> hipError_t {
        return hipMemcpyAsync((char *)b.p + bytes * to, (char *)b.p + bytes * from, bytes, hipMemcpyDeviceToDevice,
                              s);
    };
    std::vector<int> moved;
    std::vector<double> dnew;
    for (int j = 0; j < w.n; ++j) {
        if (hs[j].flag != CG_RUNNING) {
            HISQ_HIP_CHECK(hipMemcpyAsync((char *)x + s64 * slot_of[j], (char *)w.x64.p + s64 * j, s64,
                                          hipMemcpyDeviceToDevice, s));
            fin[slot_of[j]] = hs[j];
            continue;
        }
        const int i = (int)moved.size();
        if (i != j) {
            HISQ_HIP_CHECK(cp(w.b64, s64, i, j));
            HISQ_HIP_CHECK(cp(w.x64, s64, i, j));
            if (S == F64) {
                HISQ_HIP_CHECK(cp(w.r64, s64, i, j));
                HISQ_HIP_CHECK(cp(w.p64, s64, i, j));
            } else {
                HISQ_HIP_CHECK(cp(w.xs, s32, i, j));
                HISQ_HIP_CHECK(cp(w.rs, s32, i, j));
                HISQ_HIP_CHECK(cp(w.ps, sp, i, j));
            }
            HISQ_HIP_CHECK(cp(w.state, sizeof(CgState), i, j));
        }
        moved.push_back(slot_of[j]);
        dnew.push_back(diag[slot_of[j]]);
    }
    HISQ_HIP_CHECK(hipMemcpyAsync(w.diag.p, dnew.data(), sizeof(double) * dnew.size(), hipMemcpyHostToDevice, s));
    // dnew is read by the copy engine before the next synchronisation
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    slot_of = moved;
    w.n = (int)moved.size();
    return HISQ_OK;
}

static CgWorkspace *get_ws(hisq_gauge_s *g, int n, int fmt, int lfmt, int chunk, int *rc) {
    auto key = std::make_tuple(n, fmt | lfmt << 4, chunk);
    auto it = g->cg_ws.find(key);
    if (it != g->cg_ws.end()) {
        *rc = HISQ_OK;
        return it->second.get();
    }
    std::unique_ptr<CgWorkspace> w(new (std::nothrow) CgWorkspace());
    if (!w) {
        set_error("cg: host allocation failed");
        *rc = HISQ_ERR_OOM;
        return nullptr;
    }
    *rc = ws_alloc(*w, g->geom, n, fmt);
    if (*rc) return nullptr;
    w->lfmt = lfmt;
    CgWorkspace *p = w.get();
    g->cg_ws[key] = std::move(w);
    return p;
}

int cg_solve(hisq_gauge_s *g, double mass, int n, const double *b, double *x, const double *sigma,
             const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const Geom &G = g->geom;
    const int vh = G.vh;
    const int S = sloppy_vec_fmt(prm.sloppy_prec), LF = sloppy_link_fmt(prm.sloppy_prec);
    if (!g->links[F64][0].p || !g->links[LF][0].p) {
        set_error("cg: the handle lacks packed FP64 links or links of the sloppy precision");
        return HISQ_ERR_UNSUPPORTED;
    }
    const int chunk = std::max(1, prm.graph_chunk > 0 ? prm.graph_chunk : 8);
    const bool use_graph = prm.graph_chunk > 0;
    int rc;
    CgWorkspace *wp = get_ws(g, n, S, LF, use_graph ? chunk : 0, &rc);
    if (!wp) return rc;
    CgWorkspace &w = *wp;
    // compaction shrinks w.n during the solve; every exit restores it
    struct RestoreN {
        CgWorkspace &w;
        ~RestoreN() { w.n = w.cap; }
    } restore_n{w};
    w.n = w.cap;
    const size_t s64 = spinor_bytes(F64, vh) * n;
    const size_t sb = spinor_bytes(F64, vh);

    // coefficients and |b|
    std::vector<double> diag(n);
    for (int i = 0; i < n; ++i) diag[i] = 4.0 * mass * mass + (sigma ? sigma[i] : 0.0);
    HISQ_HIP_CHECK(hipMemcpyAsync(w.diag.p, diag.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(w.b64.p, b, s64, hipMemcpyDeviceToDevice, s));
    launch_norm2(vh, n, w.b64.p, (double *)w.part.p, s);
    launch_reduce(RED_STORE, n, (double *)w.part.p, blas_blocks(vh), nullptr, (double *)w.scal.p, s);
    std::vector<double> b2(n);
    HISQ_HIP_CHECK(hipMemcpyAsync(b2.data(), w.scal.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));

    std::vector<CgState> hs(n);
    for (int i = 0; i < n; ++i) {
        CgState &c = hs[i];
        std::memset(&c, 0, sizeof(c));
        c.stop2 = kResidualMargin * kResidualMargin * prm.tol * prm.tol * b2[i];
        c.true2 = c.stop2;
        c.ru_period = (S == F64) ? 0 : std::max(1, prm.ru_period);
        c.ru_delta2 = (S == F64) ? 0.0 : prm.ru_delta * prm.ru_delta;
        c.max_iter = prm.max_iter;
        c.flag = CG_ATTENTION;
    }
    HISQ_HIP_CHECK(hipMemcpyAsync(w.state.p, hs.data(), sizeof(CgState) * n, hipMemcpyHostToDevice, s));

    // r = b - A x0
    if (prm.warm_start) {
        HISQ_HIP_CHECK(hipMemcpyAsync(w.x64.p, x, s64, hipMemcpyDeviceToDevice, s));
        if ((rc = apply_A64(g, w, w.x64.p, w.ax64.p, s))) return rc;
        launch_residual(vh, n, w.b64.p, w.ax64.p, w.r64.p, w.st(), -1, (double *)w.part.p, s);
    } else {
        launch_zero(F64, vh, n, w.x64.p, s);
        HISQ_HIP_CHECK(hipMemcpyAsync(w.r64.p, w.b64.p, s64, hipMemcpyDeviceToDevice, s));
        launch_norm2(vh, n, w.r64.p, (double *)w.part.p, s);
    }
    launch_reduce(RED_INIT, n, (double *)w.part.p, blas_blocks(vh), w.st(), nullptr, s);
    if (S == F64) {
        HISQ_HIP_CHECK(hipMemcpyAsync(w.p64.p, w.r64.p, s64, hipMemcpyDeviceToDevice, s));
    } else {
        launch_zero(F32, vh, n, w.xs.p, s);
        launch_convert(F64, F32, vh, n, w.r64.p, w.rs.p, nullptr, -1, s);
        launch_convert(F64, S, vh, n, w.r64.p, w.ps.p, nullptr, -1, s);
    }
    HISQ_HIP_CHECK(hipGetLastError());

    // iterate
    // HISQ_SOLVER_TRACE=1 prints the progress every 2000 iterations to stderr
    static const bool trace = std::getenv("HISQ_SOLVER_TRACE") != nullptr;
    int next_report = 2000;
    // every pass either replays a chunk (at least one iteration of each running
    // RHS) or performs the reliable updates that the last chunk flagged
    const long max_chunks = 2L * prm.max_iter + 16;
    std::vector<int> slot_of(n);  // caller's index of each slot
    for (int i = 0; i < n; ++i) slot_of[i] = i;
    std::vector<CgState> fin(n);  // final states, by the caller's index
    for (long c = 0; c < max_chunks; ++c) {
        const int m = w.n;
        HISQ_HIP_CHECK(hipMemcpyAsync(hs.data(), w.state.p, sizeof(CgState) * m, hipMemcpyDeviceToHost, s));
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        if (trace) {
            int it = 0;
            double worst = 0.0;
            for (int i = 0; i < m; ++i) {
                it = std::max(it, hs[i].iter);
                if (hs[i].flag != CG_DONE)
                    worst = std::max(worst, std::sqrt(std::max(hs[i].rho, 0.0) / b2[slot_of[i]]));
            }
            if (it >= next_report) {
                std::fprintf(stderr, "[cg] iter %d, %d of %d RHS in the batch, worst iterated |r|/|b| %.3e\n", it,
                             m, n, worst);
                next_report = (it / 2000 + 1) * 2000;
            }
        }
        bool attention = false;
        int running = 0;
        for (int i = 0; i < m; ++i) {
            attention |= hs[i].flag == CG_ATTENTION;
            running += hs[i].flag == CG_RUNNING;
        }
        if (attention) {
            if ((rc = cg_reliable(g, w, s))) return rc;
            continue;  // re-read the flags
        }
        if (!running) break;
        // compact once the running RHS fit the next power of two below the
        // batch (RHS tiles are powers of two)
        int pow2 = 1;
        while (2 * pow2 < m) pow2 *= 2;
        if (running <= pow2 && running < m && (rc = cg_compact(g, w, slot_of, hs, fin, diag, x, s))) return rc;
        if ((rc = run_chunk(g, w, chunk, use_graph, s))) return rc;
    }

    // a breakdown in mixed precision leaves a sloppy partial solution
    if (S != F64) launch_accum_zero(F32, vh, w.n, w.x64.p, w.xs.p, w.st(), CG_BREAKDOWN, s);
    {
        const int m = w.n;
        HISQ_HIP_CHECK(hipMemcpyAsync(hs.data(), w.state.p, sizeof(CgState) * m, hipMemcpyDeviceToHost, s));
        for (int j = 0; j < m; ++j)
            HISQ_HIP_CHECK(hipMemcpyAsync((char *)x + sb * slot_of[j], (char *)w.x64.p + sb * j, sb,
                                          hipMemcpyDeviceToDevice, s));
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        for (int j = 0; j < m; ++j) fin[slot_of[j]] = hs[j];
    }
    if (w.n != n) {
        // back to the whole batch in the caller's order for the final residual
        w.n = n;
        HISQ_HIP_CHECK(hipMemcpyAsync(w.b64.p, b, s64, hipMemcpyDeviceToDevice, s));
        HISQ_HIP_CHECK(hipMemcpyAsync(w.x64.p, x, s64, hipMemcpyDeviceToDevice, s));
        HISQ_HIP_CHECK(hipMemcpyAsync(w.diag.p, diag.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    }

    // final FP64 true residual
    if ((rc = apply_A64(g, w, w.x64.p, w.ax64.p, s))) return rc;
    launch_residual(vh, n, w.b64.p, w.ax64.p, w.r64.p, nullptr, -1, (double *)w.part.p, s);
    launch_reduce(RED_STORE, n, (double *)w.part.p, blas_blocks(vh), nullptr, (double *)w.scal.p, s);
    std::vector<double> rr(n);
    HISQ_HIP_CHECK(hipMemcpyAsync(rr.data(), w.scal.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    hs = fin;

    const double ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    int worst = HISQ_OK;
    for (int i = 0; i < n; ++i) {
        const CgState &c = hs[i];
        int status = HISQ_OK;
        const double tr = b2[i] > 0 ? std::sqrt(rr[i] / b2[i]) : std::sqrt(rr[i]);
        if (c.flag == CG_BREAKDOWN) status = HISQ_BREAKDOWN;
        else if (c.flag != CG_DONE || !(tr <= prm.tol)) status = HISQ_NOT_CONVERGED;
        worst = std::max(worst, status);
        if (stats) {
            hisq_solver_stats &o = stats[i];
            o.status = status;
            o.iterations = c.iter;
            o.reliable_updates = c.reliable;
            o.fallback_used = 0;
            o.true_residual = tr;
            o.wall_ms = ms;
            o.dslash_bytes = (double)c.iter *
                                 (double)(dslash_algorithmic_bytes(LF, S, S, vh, 1, false, g->comp_mode) +
                                          dslash_algorithmic_bytes(LF, S, S == H16 ? F32 : S, vh, 1, true, g->comp_mode)) +
                             (double)(c.reliable + 1) *
                                 (double)(dslash_algorithmic_bytes(F64, F64, F64, vh, 1, false, g->comp_mode) +
                                          dslash_algorithmic_bytes(F64, F64, F64, vh, 1, true, g->comp_mode));
        }
    }
    return worst;
}

int status_severity(int st) {
    switch (st) {
        case HISQ_OK: return 0;
        case HISQ_CONVERGED_AFTER_FALLBACK: return 1;
        case HISQ_NOT_CONVERGED: return 2;
        default: return 3;
    }
}

int cg_solve_fallback(hisq_gauge_s *g, double mass, int n, const double *b, double *x,
                      const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s) {
    std::vector<hisq_solver_stats> own(n);
    hisq_solver_stats *st = stats ? stats : own.data();
    int rc = cg_solve(g, mass, n, b, x, nullptr, prm, st, s);
    if (rc <= 0 || prm.sloppy_prec == HISQ_PREC_FP64 || !prm.fallback) return rc;
    // a mixed-precision breakdown, or a stop short of the iteration cap, is
    // finished by plain FP64 CG from the current solution
    const size_t sb = spinor_bytes(F64, g->geom.vh);
    hisq_solver_params cp = prm;
    cp.sloppy_prec = HISQ_PREC_FP64;
    cp.warm_start = 1;
    int worst = HISQ_OK;
    for (int i = 0; i < n; ++i) {
        hisq_solver_stats &o = st[i];
        const bool redo = o.status == HISQ_BREAKDOWN || (o.status == HISQ_NOT_CONVERGED && o.iterations < prm.max_iter);
        if (redo) {
            hisq_solver_stats f;
            std::memset(&f, 0, sizeof(f));
            rc = cg_solve(g, mass, 1, (const double *)((const char *)b + sb * i), (double *)((char *)x + sb * i),
                          nullptr, cp, &f, s);
            if (rc < 0) return rc;
            o.status = f.status == HISQ_OK ? HISQ_CONVERGED_AFTER_FALLBACK : f.status;
            o.iterations += f.iterations;
            o.reliable_updates += f.reliable_updates;
            o.fallback_used = 1;
            o.true_residual = f.true_residual;
            o.wall_ms += f.wall_ms;
            o.dslash_bytes += f.dslash_bytes;
        }
        if (status_severity(o.status) > status_severity(worst)) worst = o.status;
    }
    return worst;
}

}  // namespace hisq
