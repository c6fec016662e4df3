// Host-side structures of the solver runtime: the gauge handle, per-RHS CG
// state kept in device memory, workspaces and cached graphs.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "hisq_internal.h"

namespace hisq {

// Life cycle of one right-hand side inside the device-side iteration.
enum CgFlag {
    CG_RUNNING = 0,    // iterating
    CG_ATTENTION = 1,  // reliable update / convergence check / cap reached: host acts
    CG_DONE = 2,       // true residual below the target
    CG_BREAKDOWN = 3,  // non-finite value or non-positive curvature
    CG_MAXITER = 4,    // iteration cap reached without convergence
    CG_RESUME = 5      // transient: residual replaced, p update pending
};

struct CgState {
    double rho;      // <r, r> of the current residual
    double rho_new;  // <r, r> after the last update
    double pap;      // Re <p, A p>
    double alpha, beta;
    double stop2;    // iterated-residual trigger for the true-residual check, starts at (tol |b|)^2
    double true2;    // target of the FP64 true residual, (tol |b|)^2
    double true_rr;  // last |b - A x|^2 computed in FP64
    double ru_rho;   // |r|^2 right after the last reliable update (or the start)
    double ru_delta2;  // reliable update once rho_new <= ru_delta2 * ru_rho (0: off)
    int iter;        // completed iterations
    int xpend;       // x += alpha p of this iteration still to be applied
    int since_ru;    // iterations since the last reliable update
    int ru_period;   // 0: no periodic reliable update
    int max_iter;
    int flag;
    int reliable;    // reliable updates done
};

enum { RED_ALPHA, RED_BETA, RED_TRUE, RED_INIT, RED_STORE };

// The solvers stop when their own FP64 true residual |b - A x| is at most
// kResidualMargin * tol |b|.  Another FP64 evaluation of the same residual
// (other summation order, e.g. a reference implementation) differs by rounding
// of order eps |A| |x|, which grows with the condition number; on the
// benchmark lattices the two evaluations differ by up to ~5e-13 |b| at
// m = 0.002.  A 10 % margin keeps every solution at or below tol for any such
// evaluation, at the cost of ~1 % more iterations.
constexpr double kResidualMargin = 0.9;

int blas_blocks(int vh);
void launch_update_xr(int fmt_sloppy, int vh, int n, void *x, void *r, const void *p, const void *q,
                      const CgState *st, double *part, hipStream_t s);
void launch_update_p(int fmt_sloppy, int vh, int n, const void *r, void *p, const CgState *st, int when,
                     hipStream_t s);
// The two vector passes of one batched CG iteration:
//   r -= alpha q with partial |r|^2                       (running RHS)
//   x += alpha p (iteration's alpha pending); p = r + beta p (still running)
void launch_update_r(int fmt_sloppy, int vh, int n, void *r, const void *q, const CgState *st, double *part,
                     hipStream_t s);
void launch_update_xp(int fmt_sloppy, int vh, int n, void *x, const void *r, void *p, const CgState *st,
                      hipStream_t s);
int launch_convert(int fs, int fd, int vh, int n, const void *src, void *dst, const CgState *st, int when,
                   hipStream_t s);
void launch_accum_zero(int fmt_x, int vh, int n, void *xhi, void *xs, const CgState *st, int when,
                       hipStream_t s);
void launch_residual(int vh, int n, const void *b, const void *ax, void *r, const CgState *st, int when,
                     double *part, hipStream_t s);
void launch_norm2(int vh, int n, const void *v, double *part, hipStream_t s);
void launch_zero(int fmt, int vh, int n, void *v, hipStream_t s);
void launch_reduce(int which, int n, const double *part, int nb, CgState *st, double *out, hipStream_t s);
void launch_resume_flags(int n, CgState *st, hipStream_t s);

// Device allocation owned by the handle.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t n);
};

// Tuned launch shape of the Dslash for one (precision pair, nrhs).
struct DslashShape {
    int tile = 1;
    int block = 256;
    int order = 0;
};

// Buffers, device state and the captured iteration graph of one solver shape.
struct CgWorkspace {
    int n = 0, fmt = F64, chunk = 0;
    int cap = 0;     // RHS the buffers hold; n < cap while finished RHS are compacted out
    int lfmt = F64;  // links of the sloppy Dslash
    DevBuf b64, x64, r64, t64, ax64, p64, q64;
    DevBuf xs, rs, ps, ts, qs;
    DevBuf part, state, diag, scal;
    // captured chunk of iterations per active RHS count
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    ~CgWorkspace() {
        for (auto &kv : graphs) {
            if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
            if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
        }
    }
    // sloppy views (aliases of the FP64 buffers in plain mode)
    void *X() { return fmt == F64 ? x64.p : xs.p; }
    void *R() { return fmt == F64 ? r64.p : rs.p; }
    void *P() { return fmt == F64 ? p64.p : ps.p; }
    void *T() { return fmt == F64 ? t64.p : ts.p; }
    void *Q() { return fmt == F64 ? q64.p : qs.p; }
    CgState *st() { return (CgState *)state.p; }
};

// Buffers, device state and the captured iteration graph of flexible CG.
struct FcgWorkspace {
    DevBuf b64, x64, r64, t64, ax64;
    DevBuf xs, rs, ps, qs, zs, ts;
    DevBuf part, part2, state, diag, scal;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long net_id = 0;  // network the graph was captured with
    int chunk = 0;
    FcgWorkspace() = default;
    FcgWorkspace(const FcgWorkspace &) = delete;
    FcgWorkspace &operator=(const FcgWorkspace &) = delete;
    ~FcgWorkspace();
};

}  // namespace hisq

struct hisq_gauge_s {
    int dims[4];
    hisq::Geom geom;
    int device = 0;
    hisq::DevBuf links[3][2];  // [format][output parity]
    int comp_mode = 0;         // CompMode of the FP32 / FP16 long links (two rows + sign bit or kappa)
    hisq::DevBuf diag_buf;     // epilogue coefficients for hisq_dslash_multi_rhs
    hipEvent_t diag_event = nullptr;  // recorded after the last kernel that read diag_buf
    hisq::DevBuf thin;         // thin links (FP16) for the preconditioner network
    hipStream_t capture_stream = nullptr;
    std::mutex mu;
    // autotuned shapes keyed by (links fmt, in fmt, out fmt, nrhs, epilogue)
    std::map<std::tuple<int, int, int, int, int>, hisq::DslashShape> shapes;
    std::map<std::tuple<int, int, int>, std::unique_ptr<hisq::CgWorkspace>> cg_ws;  // (n, fmt | links << 4, chunk)
    std::unique_ptr<hisq::FcgWorkspace> fcg_ws;
    ~hisq_gauge_s();
};

namespace hisq {

// Link and vector formats of a solver sloppy mode (HISQ_PREC_FP16L: FP16
// links applied to FP32 vectors; otherwise both in the named precision).
inline int sloppy_link_fmt(int sloppy) { return sloppy == HISQ_PREC_FP16L ? H16 : sloppy; }
inline int sloppy_vec_fmt(int sloppy) { return sloppy == HISQ_PREC_FP16L ? F32 : sloppy; }

// The FP64 copy always keeps every link whole: it carries the true residual
// and the reliable updates, where a 1e-15 row-rebuild error times the
// condition number (up to ~1e6 at the lightest masses) would reach the 1e-10
// target.  The sloppy FP32 / FP16 copies are compressed when possible.
inline int links_compressed(const hisq_gauge_s *g, int fmt) { return fmt == F64 ? COMP_NONE : g->comp_mode; }

DslashShape pick_shape(hisq_gauge_s *g, int fl, int fi, int fo, int nrhs, bool epi);

// Argument checks shared by the multi-RHS Dslash entry points (HISQ_OK or an
// error code with the message set).
int check_multi_rhs(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in, void *out,
                    const double *diag, const void *y);

// Dslash on the handle's packed links.
int gauge_dslash(hisq_gauge_s *g, int out_parity, int fmt_links, int fmt_in, int fmt_out, int nrhs,
                 const void *in, void *out, const void *y, const double *diag_dev, double *partials,
                 const CgState *skip, hipStream_t s);

int nb_dslash(hisq_gauge_s *g, int fl, int fi, int fo, int n, bool epi);

// Time the candidate launch shapes (or read them from `cache`) and install the best.
int tune_dslash(hisq_gauge_s *g, int fl, int fi, int fo, int nrhs, bool epi, const char *cache, hipStream_t s,
                DslashShape *chosen, double *chosen_ms);
// Algorithmic bytes of one Dslash launch (links read once, spinors once per RHS);
// comp: CompMode of the long links (two rows + a sign word per site, or two
// rows + a complex factor per link).
size_t dslash_algorithmic_bytes(int fmt_links, int fmt_in, int fmt_out, int64_t vh, int nrhs, bool epi, int comp);

int cg_solve(hisq_gauge_s *g, double mass, int nrhs, const double *b, double *x, const double *sigma,
             const hisq_solver_params &p, hisq_solver_stats *st, hipStream_t s);

// Severity order of soft outcomes: OK < converged after fallback < not converged < breakdown.
int status_severity(int status);

// cg_solve, then plain FP64 CG from the current x for every RHS whose
// mixed-precision solve broke down or stopped short of the iteration cap.
int cg_solve_fallback(hisq_gauge_s *g, double mass, int n, const double *b, double *x,
                      const hisq_solver_params &prm, hisq_solver_stats *stats, hipStream_t s);

// Flexible CG for one right-hand side with z = N(r) (prm.precond set).
int fcg_solve(hisq_gauge_s *g, double mass, const double *b, double *x, const hisq_solver_params &prm,
              hisq_solver_stats *stats, hipStream_t s);

int multishift_solve(hisq_gauge_s *g, double mass, int nshift, const double *shifts, const double *b,
                     double *x, const hisq_solver_params &p, hisq_solver_stats *st, hipStream_t s);
// nsrc sources b [nsrc][spinor], x [nsrc][nshift][spinor], st [nsrc][nshift]
int multishift_solve_batched(hisq_gauge_s *g, double mass, int nsrc, int nshift, const double *shifts,
                             const double *b, double *x, const hisq_solver_params &p, hisq_solver_stats *st,
                             hipStream_t s);

// Zolotarev's minimax relative approximation of x^(-1/2) on [lmin, lmax] in
// partial fractions alpha0 + sum_k alpha[k] / (x + shift[k]); delta = its
// maximal relative error.  Host only.
int zolotarev_inv_sqrt(double lmin, double lmax, int n, double *alpha0, double *alpha, double *shift,
                       double *delta);
int remez_power(double power, double lmin, double lmax, int n, double *alpha0, double *alpha, double *shift,
                double *delta);
// out = alpha0 b + sum_k alpha[k] (A + shift[k])^(-1) b by one multi-shift CG.
int rational_apply(hisq_gauge_s *g, double mass, int nsrc, double alpha0, int n, const double *alpha,
                   const double *shift, const double *b, double *out, const hisq_solver_params &prm,
                   hisq_solver_stats *st, hipStream_t s);
// HISQ smearing of canonical thin links into folded fat and Naik links (FP64).
int smear_links(const int dims[4], const double *thin, double *fat, double *lng, unsigned flags, hipStream_t s);

// lmin = 4 m^2 (a bound); lmax = Rayleigh quotient after `iters` power iterations.
int spectral_bounds(hisq_gauge_s *g, double mass, int iters, double *lmin, double *lmax, hipStream_t s);

}  // namespace hisq
