/*
 * hisq.h - C ABI of the MI355X (gfx950) HISQ even/odd Dslash and solver library.
 *
 * The library applies the HISQ staggered operator (fat one-link plus Naik
 * three-link SU(3) stencil; the paper's D-slash, Sec. 3, whose application it
 * names the most performance-critical kernel of its CG, the solver that takes
 * about 60% of the RHMC time) and solves the even/odd-preconditioned normal
 * equations (D^+ D + 4 m^2) x = b with the CG variants the paper lists in
 * Sec. 2: multi-RHS, multi-shift and mixed precision.
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice: extents dims[4] = {Lx, Ly, Lz, Lt}, each even and >= 4, volume
 *   V = Lx*Ly*Lz*Lt < 2^31, Vh = V/2.  Site x = (x0,x1,x2,x3), direction mu =
 *   0..3 <-> x,y,z,t, parity (x0+x1+x2+x3) & 1 (0 = even).
 * Checkerboard index of a site: h = lex >> 1 with lex = x0 + Lx*(x1 + Ly*(x2 +
 *   Lz*x3)).  h runs over [0, Vh) for either parity.
 * Operator (phases and boundary signs already folded into the links):
 *   (D chi)(x) = sum_mu [ F_mu(x) chi(x+mu) - F_mu(x-mu)^+ chi(x-mu)
 *                       + L_mu(x) chi(x+3mu) - L_mu(x-3mu)^+ chi(x-3mu) ]
 *   D maps one parity to the other.  Normal operator on even sites:
 *   A = 4 m^2 - D_eo D_oe  ( = (D^+ D + 4 m^2) restricted to even sites, HPD).
 *
 * Spinor (colour-vector) buffers, one parity, sites in checkerboard order h:
 *   HISQ_PREC_FP64  : complex double [3][Vh], colour-major planes   48*Vh bytes
 *                     (colour c of site h at complex index c*Vh + h)
 *   HISQ_PREC_FP32  : plane A float[Vh][4] = (re0, im0, re1, im1), then
 *                     plane B float[Vh][2] = (re2, im2)            24*Vh bytes
 *   HISQ_PREC_FP16S : one 16-byte record per site: half[6] = (re0, im0, re1,
 *                     im1, re2, im2) then float scale; value = scale * half,
 *                     scale = max |re|,|im| over the site's 6 reals,
 *                     halves rounded to nearest even               16*Vh bytes
 *   nrhs buffers are stacked back to back: [nrhs][one buffer].
 *   hisq_spinor_bytes() returns the size of one buffer.  Every spinor pointer
 *   must be 16-byte aligned.
 *
 * Memory and streams: every data pointer is a DEVICE pointer on the current
 * HIP device unless stated otherwise.  The caller owns its buffers; the library
 * never frees them and keeps no reference after a call returns.  A gauge handle
 * owns the library's own packed link copies and solver workspaces.  `stream`
 * is a hipStream_t (NULL = the default stream).  Dslash calls are asynchronous
 * on that stream; solvers order themselves after prior work on it and return
 * when x is written (synchronous).
 *
 * Errors: 0 = OK.  Negative = hard error (nothing usable was written):
 *   -1 invalid argument, -2 HIP runtime error, -3 out of device memory,
 *   -4 unsupported.  Positive = soft solver outcome, x and stats valid:
 *   1 not converged within max_iter, 2 breakdown (non-finite or non-positive
 *   curvature), 3 converged only after falling back to plain FP64 CG.
 *   hisq_last_error() returns a message for the calling thread's last failure.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HISQ_OK 0
#define HISQ_ERR_INVALID -1
#define HISQ_ERR_HIP -2
#define HISQ_ERR_OOM -3
#define HISQ_ERR_UNSUPPORTED -4
#define HISQ_NOT_CONVERGED 1
#define HISQ_BREAKDOWN 2
#define HISQ_CONVERGED_AFTER_FALLBACK 3

#define HISQ_PREC_FP64 0
#define HISQ_PREC_FP32 1
#define HISQ_PREC_FP16S 2
/* Solver sloppy precision only (hisq_solver_params.sloppy_prec, hisq_autotune,
 * hisq_dslash_shape): the FP16 links of the FP16S copy applied to FP32
 * vectors.  Needs the FP16S links packed. */
#define HISQ_PREC_FP16L 3

/* Bit masks for hisq_gauge_create's prec_mask. */
#define HISQ_PREC_MASK(p) (1u << (p))
#define HISQ_PREC_MASK_ALL 7u
/* Store every link whole, even when the long links could be compressed. */
#define HISQ_LINKS_FULL (1u << 8)

typedef struct hisq_gauge_s *hisq_gauge_t;
typedef struct hisq_nn_s *hisq_nn_t;

/* Library version (major*10000 + minor*100 + patch); equals HISQ_VERSION of
 * the header the library was built with.  0.2.0: hisq_solver_params gained
 * ru_delta (callers built against 0.1 pass a shorter struct).  0.3.0:
 * hisq_multishift_cg_batched and hisq_rational_apply_batched. */
#define HISQ_VERSION 300
int hisq_version(void);

/* Message describing the calling thread's most recent error ("" if none). */
const char *hisq_last_error(void);

/* Bytes of one spinor buffer of precision `prec` on a lattice with Vh
 * half-lattice sites, in the layout described above; 0 for a bad prec. */
size_t hisq_spinor_bytes(int prec, int64_t vh);

/*
 * Create a gauge handle: validate dims and pack the fat and Naik links into
 * the library's per-output-site layout for every precision in prec_mask.
 *   dims     host int[4], extents as above
 *   fat, lng device, complex double [V][4][3][3] (row a, column b of
 *            U_mu(x) at ((lex*4 + mu)*3 + a)*3 + b), phases and boundary
 *            signs folded in.  Only read during the call.
 *   prec_mask which packed copies to build (HISQ_PREC_MASK bits), plus
 *            optionally HISQ_LINKS_FULL.  FP16 links need every entry below
 *            2^14 in magnitude.
 * Gauge-field compression (the paper's D-slash, Sec. 3: store part of each
 * link, recompute the rest from its SU(3) or U(3) structure): unless
 * HISQ_LINKS_FULL is set, the FP32 and FP16 copies store only the first two
 * rows of each long link and the kernels rebuild the third as
 * kappa * conj(row0 x row1), which holds for any multiple M = s U of a
 * unitary U with kappa = det(M) / s^4.  When every long link is unitary with
 * determinant +1 or -1 (deviation at most 1e-12 in FP64: SU(3) products with
 * the signs folded in) kappa is a sign bit per link (mode 1); otherwise, when
 * every long link is a positive multiple of a unitary matrix (relative
 * deviation at most 1e-12: the U(3)-projected HISQ Naik links), kappa is
 * stored as a complex number per link (mode 2).  The fat links, and every
 * link of the FP64 copy (which carries the true residual), stay whole.
 * hisq_gauge_links_compressed() reports the choice.
 * On success *out receives the handle.  Errors: -1 bad dims / null pointers /
 * empty mask, -3 out of memory, -2 HIP failure.
 */
int hisq_gauge_create(hisq_gauge_t *out, const int dims[4], const double *fat, const double *lng,
                      unsigned prec_mask, void *stream);

/*
 * HISQ link smearing: the fat and Naik links of the HISQ action (Follana et
 * al., Phys. Rev. D 75 (2007) 054502; the action of the paper's HotQCD
 * ensembles, Sec. 1) from the thin gauge links, in FP64:
 *   V = fat7[U]      one-link 1/8, 3-staple 1/16, 5-staple 1/64, 7-staple
 *                    1/384 (every ordering of the transverse directions)
 *   W = V (V^+ V)^(-1/2)                           (projection onto U(3))
 *   X = fat7[W] with one-link 1 and the Lepage (two-step staple) term -1/8
 *   L_mu(x) = -1/24 W_mu(x) W_mu(x+mu) W_mu(x+2mu)
 * with the staggered phases and boundary signs folded in, so fat = X and
 * lng = L go straight to hisq_gauge_create.  Unit links give 9/8 and -1/24.
 * The Naik links are multiples of U(3) matrices: hisq_gauge_create stores
 * them compressed (two rows and a complex factor, see there).
 *   dims      host int[4], as for hisq_gauge_create
 *   thin      device, complex double [V][4][3][3] gauge links without phases
 *             (periodic gauge field), canonical layout; only read
 *   fat, lng  device outputs in the same layout; none of the three may overlap
 *   flags     HISQ_SMEAR_ANTIPERIODIC_T: fold the antiperiodic time boundary
 *             sign (-1 on t links with t + 1 >= Lt, Naik links t + 3 >= Lt)
 * Allocates a workspace of 6 link fields of one direction (864 V bytes) for
 * the call.  Synchronous.  Errors: -1 bad dims, pointers, flags or overlap,
 * -3 out of memory, -2 HIP failure.
 */
#define HISQ_SMEAR_ANTIPERIODIC_T 1u
int hisq_smear_links(const int dims[4], const double *thin, double *fat, double *lng, unsigned flags,
                     void *stream);

/* Compression of the handle's FP32 / FP16 long links: 0 whole, 1 two rows and
 * a determinant sign bit, 2 two rows and a complex factor; -1 for NULL. */
int hisq_gauge_links_compressed(hisq_gauge_t g);

/* Release the handle and everything it owns (NULL is accepted). */
int hisq_gauge_destroy(hisq_gauge_t g);

/* Bytes of device memory owned by the handle (packed links plus workspaces). */
int hisq_gauge_device_bytes(hisq_gauge_t g, size_t *bytes);

/*
 * Single-parity Dslash (the paper's D-slash application, Sec. 3):
 *   out = D_{pi, 1-pi} in, pi = out_parity (0 even, 1 odd).
 *   in   spinor of parity 1-pi, out spinor of parity pi, both of `prec`
 *        (FP16S in and out; arithmetic in FP32 for FP32/FP16S, FP64 for FP64).
 *   in and out must not overlap.  Asynchronous on `stream`.
 * Errors: -1 bad parity/prec/pointers, -4 precision not packed in the handle.
 */
int hisq_dslash_eo(hisq_gauge_t g, int out_parity, int prec, const void *in, void *out,
                   void *stream);

/*
 * Multi-RHS Dslash (the paper's multi-RHS D-slash, Sec. 3: each link load is
 * applied to several right-hand sides):
 *   out_i = D in_i                          (diag == NULL)
 *   out_i = diag[i] * y_i - D in_i          (diag != NULL; diag is a HOST
 *                                            double[nrhs], y device spinors)
 * for i = 0..nrhs-1, buffers stacked [nrhs][spinor].  With
 * diag[i] = 4 m^2 + sigma_i and y = the even vectors that in = D_oe y was
 * formed from, this is (A + sigma_i) y_i.  For FP16S the epilogue output is
 * written as FP16S too.  The RHS tile and block shape come from the
 * autotuner's table (defaults if the shape was never tuned).  The stacks in
 * and out (and y and out) must not overlap.  diag is copied to a buffer of
 * the handle (grown, with a synchronisation, only for nrhs > 64); calls on
 * different streams are ordered on the device around that buffer.
 * Errors: -1 bad arguments (nrhs < 1, y without diag, overlapping stacks),
 * -4 precision not packed.
 */
int hisq_dslash_multi_rhs(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in,
                          void *out, const double *diag, const void *y, void *stream);

/*
 * hisq_dslash_multi_rhs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, semantics and output.  The per-RHS epilogue
 * coefficients are staged in a fixed device array of HISQ_NOALLOC_MAX_RHS
 * doubles per GPU, set up by hisq_gauge_create and kept until the process
 * ends, so the call allocates nothing.  Every call on one GPU shares that
 * array: calls with diag that overlap in time on one GPU (different streams
 * or threads without ordering) race on it; calls ordered on one stream do
 * not.  diag is read during the call (host), y/in/out as for
 * hisq_dslash_multi_rhs.
 * Errors: those of hisq_dslash_multi_rhs, and -1 if diag is given with nrhs >
 * HISQ_NOALLOC_MAX_RHS.
 */
#define HISQ_NOALLOC_MAX_RHS 4096
int hisq_dslash_multi_rhs_noalloc(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in,
                                  void *out, const double *diag, const void *y, void *stream);

/*
 * Autotune the Dslash launch shape (RHS tile per thread: 1, 2, 4, 8 or 16, at
 * most 4 with FP64 links; block size 64, 128 or 256; order: bits 0-23 the
 * traversal - 0 memory order, 1 t-fastest planes, 2 | BY << 8 | BZ << 16 XCD
 * bricks, 3 memory order with the x-rows of a workgroup staged in LDS (block
 * 64-256 threads of whole rows, tiles up to 8), 4 | K << 8 a t-march of K
 * sites per thread (tiles up to 4) - and bits 24-25 log2 of the number of
 * waves a site's RHS tiles are split over) for the kernels a solve in `prec`
 * with `nrhs` right-hand sides launches: plain and epilogue Dslash in `prec`
 * and, if FP64 links are packed, the FP64 kernels of the reliable updates.
 * Each candidate must write bit-identical output to the default shape before
 * it is timed (HIP events, the handle's own links, synthetic inputs).
 *   cache_path  NULL, or a file of JSON lines {"key", "tile", "block",
 *               "order", "ms"} keyed by GPU architecture, formats, lattice and
 *               nrhs: a key found there is installed without timing, a new
 *               result is appended.
 * Installed shapes apply to later Dslash calls and solves on this handle.
 * Synchronous.  Errors: -1 bad arguments (nrhs outside 1..64), -4 precision
 * not packed.
 */
int hisq_autotune(hisq_gauge_t g, int prec, int nrhs, const char *cache_path, void *stream);

/* Launch shape in use for (prec, nrhs, epilogue): epilogue 0 = plain Dslash,
 * 1 = diag*y - D in with output in prec, 2 = the solver's form (FP16S input
 * with FP32 output).  out[0] = RHS tile, out[1] = block size, out[2] = order. */
int hisq_dslash_shape(hisq_gauge_t g, int prec, int nrhs, int epilogue, int out[3]);

/* Solver controls (host struct).  Zero-initialise and set what you need;
 * hisq_solver_params_default() fills the defaults noted below. */
typedef struct {
    double tol;        /* target true relative residual |b - A x| / |b| (1e-10) */
    int max_iter;      /* iteration cap per right-hand side (100000) */
    int sloppy_prec;   /* HISQ_PREC_FP64: plain CG; FP32 / FP16S / FP16L: mixed
                          precision with FP64 reliable updates (FP64).  FP16S
                          rounds the Krylov direction to FP16 as well, FP16L
                          keeps every vector in FP32 and only the links in FP16 */
    int ru_period;     /* iterations between reliable updates (100) */
    int graph_chunk;   /* iterations per replay of a captured hipGraph; 0 = eager
                          kernel launches (32) */
    int warm_start;    /* nonzero: x holds the initial guess on entry (0) */
    int fallback;      /* nonzero: after a breakdown or stagnation of a mixed or
                          preconditioned solve, finish with plain FP64 CG (1) */
    hisq_nn_t precond; /* NULL, or a network: flexible CG with z = N(r) (NULL) */
    double ru_delta;   /* mixed precision: a reliable update also when the iterated
                          residual norm has fallen by this factor since the last
                          one, in [0, 1); 0 = by ru_period and convergence only
                          (0.1) */
} hisq_solver_params;

/* Per right-hand side (or per shift) solver report. */
typedef struct {
    int status;            /* 0 / HISQ_NOT_CONVERGED / HISQ_BREAKDOWN / ..._AFTER_FALLBACK */
    int iterations;        /* operator applications in the Krylov loop */
    int reliable_updates;  /* FP64 residual recomputations */
    int fallback_used;     /* 1 if plain FP64 CG finished the solve */
    double true_residual;  /* final |b - A x| / |b| computed in FP64 */
    double wall_ms;        /* wall time of the whole call */
    double dslash_bytes;   /* algorithmic bytes moved by Dslash launches */
} hisq_solver_stats;

void hisq_solver_params_default(hisq_solver_params *p);

/*
 * CG solve of (D^+ D + 4 m^2)_ee x_i = b_i for i = 0..nrhs-1 (the paper's CG,
 * Sec. 2-3, with its multi-RHS and mixed-precision forms).
 *   mass  m > 0
 *   b, x  device, FP64 spinors [nrhs][3][Vh] (even sites); x is overwritten
 *         with the solution (and read as the initial guess if warm_start).
 *   p     host params (NULL = defaults); st host array of nrhs stats (or NULL).
 * nrhs > 1 runs nrhs independent CGs in lockstep sharing multi-RHS Dslash
 * launches.  Stops on the FP64 true residual.  Synchronous.
 * With p->precond set, each right-hand side is solved in turn by flexible CG
 * (Notay, SIAM J. Sci. Comput. 22 (2000), FCG(1): the learned preconditioner
 * beside the paper's solver family, which is an extension of it) with z = N(r) in FP32, complex step sizes and FP64 reliable updates every
 * ru_period iterations, after which the iteration continues from the
 * recomputed residual with the current search direction; the network
 * must belong to g and the handle needs FP64 and FP32 links plus thin links.
 * A breakdown, or three reliable updates in a row that fail to halve the true
 * residual, hands the solve to plain FP64 CG from the current x when
 * p->fallback is set (status HISQ_CONVERGED_AFTER_FALLBACK on success); a
 * mixed-precision solve that breaks down is finished the same way.
 * Returns the worst per-RHS status in the order 0 < CONVERGED_AFTER_FALLBACK
 * < NOT_CONVERGED < BREAKDOWN (0 if all converged).
 */
int hisq_cg_solve(hisq_gauge_t g, double mass, int nrhs, const double *b, double *x,
                  const hisq_solver_params *p, hisq_solver_stats *st, void *stream);

/*
 * Multi-shift CG (the paper's multiple-shift CG, Sec. 2): (A + sigma_k) x_k = b
 * for k = 0..nshift-1 from one Krylov space, each shift stopped on its own
 * residual, then every shift checked (and if needed refined by CG) on its
 * FP64 true residual.
 *   shifts host double[nshift], every sigma_k + 4 m^2 > 0
 *   b      device FP64 spinor [3][Vh];  x device FP64 [nshift][3][Vh]
 *   st     host array of nshift stats (or NULL)
 */
int hisq_multishift_cg(hisq_gauge_t g, double mass, int nshift, const double *shifts,
                       const double *b, double *x, const hisq_solver_params *p,
                       hisq_solver_stats *st, void *stream);

/*
 * Multi-shift CG for several sources with the same shifts (the paper's
 * multi-RHS and multiple-shift CG together, Sec. 2): (A + sigma_k) x_jk = b_j.
 * The sources run in lockstep: their base directions form one multi-RHS
 * stack, so every link load of the Dslash serves all of them, and the final
 * verification / refinement is one batched solve over all (source, shift)
 * pairs.  The Krylov vectors are FP32 for any sloppy precision other than
 * FP64, FP64 otherwise; nsrc = 1 is hisq_multishift_cg.
 *   b   device FP64 spinors [nsrc][3][Vh];  x device FP64 [nsrc][nshift][3][Vh]
 *   st  host array of nsrc * nshift stats, [source][shift] (or NULL)
 *   1 <= nsrc <= 64, 1 <= nshift <= 256, nsrc * nshift <= 1024; b and x must
 *   not overlap.  Returns the worst status over all (source, shift) pairs.
 * Workspace (allocated by the call): nsrc * nshift * (2 FP64 + 2 Krylov-
 * precision) spinors for the iteration, a few per source, and the vectors of
 * the refinement's batched CG on top; HISQ_ERR_OOM if the device cannot hold
 * them (at 96^3 x 24 an FP64 spinor is 510 MB).
 */
int hisq_multishift_cg_batched(hisq_gauge_t g, double mass, int nsrc, int nshift,
                               const double *shifts, const double *b, double *x,
                               const hisq_solver_params *p, hisq_solver_stats *st, void *stream);

/*
 * Rational functions of A, the solver-side part of rational hybrid Monte
 * Carlo (the paper's RHMC for 2+1 flavours and its multiple-shift CG, Sec. 2;
 * most of the RHMC time goes into these CG solves, Sec. 3): with a rational
 * approximation in partial fractions,
 *     out = alpha0 b + sum_k alpha[k] (A + shift[k])^(-1) b
 * computed by one multi-shift CG (hisq_multishift_cg, each shift to p->tol on
 * its FP64 true residual) and one FP64 linear combination.
 *   alpha, shift host double[nterm] (0 <= nterm <= 256; nterm = 0 gives
 *                alpha0 b), every shift + 4 m^2 > 0
 *   b, out       device FP64 spinors [3][Vh] (even sites), not overlapping
 *   st           host array of nterm stats (or NULL)
 * Needs FP64 links in the handle.  Returns the worst multi-shift status.
 */
int hisq_rational_apply(hisq_gauge_t g, double mass, double alpha0, int nterm, const double *alpha,
                        const double *shift, const double *b, double *out,
                        const hisq_solver_params *p, hisq_solver_stats *st, void *stream);

/*
 * hisq_rational_apply for nsrc sources (several pseudofermion fields) through
 * one hisq_multishift_cg_batched solve: out_j = alpha0 b_j + sum_k alpha[k]
 * (A + shift[k])^(-1) b_j.
 *   b, out  device FP64 spinors [nsrc][3][Vh], not overlapping
 *   st      host array of nsrc * nterm stats, [source][term] (or NULL)
 *   1 <= nsrc <= 64, nsrc * nterm <= 1024.
 */
int hisq_rational_apply_batched(hisq_gauge_t g, double mass, int nsrc, double alpha0, int nterm,
                                const double *alpha, const double *shift, const double *b,
                                double *out, const hisq_solver_params *p, hisq_solver_stats *st,
                                void *stream);

/*
 * Zolotarev's optimal rational approximation of x^(-1/2) on [lmin, lmax]
 * (minimax relative error; E. I. Zolotarev 1877, in the partial-fraction form
 * used for rooted staggered pseudofermions): on return
 *     x^(-1/2) ~ *alpha0 + sum_k alpha[k] / (x + shift[k]),  k < npole,
 * with 0 < shift[0] < ... < shift[npole-1], every alpha[k] > 0, and *delta
 * (may be NULL) the largest relative error over the interval; the error
 * equioscillates 2 npole + 2 times (down to ~1e-13, where the rounding of
 * the FP64 coefficients takes over).  Host only (no GPU).
 *   0 < lmin < lmax, lmax / lmin <= 1e14, 1 <= npole <= 64; alpha and shift
 *   are host double[npole] arrays that must not overlap
 */
int hisq_zolotarev_inv_sqrt(double lmin, double lmax, int npole, double *alpha0, double *alpha,
                            double *shift, double *delta);

/*
 * Minimax relative rational approximation of x^power on [lmin, lmax], the
 * coefficients of the RHMC rational functions for other roots than the
 * square root (e.g. x^(1/4) for the two-flavour pseudofermion heat bath, and
 * x^(-1/4), x^(1/8) for the strange quark; the paper's RHMC for 2+1 flavours,
 * Sec. 2): on return
 *     x^power ~ *alpha0 + sum_k alpha[k] / (x + shift[k]),  k < npole,
 * with 0 < shift[0] < ... < shift[npole-1] and *delta (may be NULL) the
 * largest relative error over the interval, at which the error equioscillates
 * 2 npole + 2 times (Chebyshev's alternation theorem).  Remez exchange on the
 * product form, started from Zolotarev's x^(-1/2) and continued along the
 * power.  Every alpha[k] is positive for power < 0 and negative for
 * power > 0.  Host only (no GPU).
 *   alpha, shift host double[npole] arrays that must not overlap;
 *   0.05 <= |power| <= 0.95; 0 < lmin < lmax, lmax / lmin <= 1e14;
 *   1 <= npole <= 64, and a pole count for which the x^(-1/2) error on the
 *   same interval lies in [1e-12, 0.5] (HISQ_ERR_INVALID otherwise: below,
 *   the error would drown in rounding; above, the approximation is useless)
 * Returns HISQ_ERR_UNSUPPORTED if the exchange finds no equioscillating
 * solution, or if the partial fractions in FP64 lose the approximation to
 * cancellation against alpha0 (positive powers close to 1 over many
 * decades, e.g. x^0.95 on [1e-4, 40]).  Host time: milliseconds for 16
 * poles, up to ~2 s for 40-64 poles over 1e14.
 */
int hisq_rational_remez(double power, double lmin, double lmax, int npole, double *alpha0,
                        double *alpha, double *shift, double *delta);

/*
 * Spectrum bounds of A for a rational approximation: *lmin = 4 m^2 (a lower
 * bound, since (D^+ D)_ee >= 0) and *lmax = the Rayleigh quotient of A after
 * `iters` FP64 power iterations from a fixed pseudo-random vector, an
 * estimate from below of the largest eigenvalue (enlarge it by a margin
 * before use).  Synchronous; needs FP64 links.
 */
int hisq_spectral_bounds(hisq_gauge_t g, double mass, int iters, double *lmin, double *lmax, void *stream);

/*
 * Gauge-covariant preconditioner network, z = N(r) (not part of the paper's
 * method: the learned preconditioner beside its CG family).  The layers are
 * the linear parallel-transport layers of lattice gauge-equivariant networks
 * (Favoni et al., Phys. Rev. Lett. 128 (2022) 032003), used as a
 * preconditioner of the Dirac normal equations as by Lehner and Wettig
 * (Phys. Rev. D 108 (2023) 034503): a stack of linear layers
 * psi'_a(x) = sum_b [ W0_ab psi_b(x) + sum_mu ( Wf_mu,ab U_mu(x) psi_b(x+mu)
 *                                            + Wb_mu,ab U_mu(x-mu)^+ psi_b(x-mu) ) ]
 * on the full lattice (the even input embedded with zeros on odd sites, the
 * output projected back to even sites), channel counts 1 -> C -> ... -> 1.
 *   in, out  device FP32 spinors (public FP32 layout, even parity)
 * The layer weights are complex; the channel mixing runs as a BF16 matrix-core
 * product with FP32 accumulation, the parallel transport in FP32 on FP16
 * links, and hidden activations are stored in BF16.
 * Errors: -1 bad arguments, -4 the handle has no thin links.
 */
int hisq_precond_apply(hisq_gauge_t g, hisq_nn_t net, const void *in, void *out, void *stream);

/* Thin links for the network: device, complex double [V][4][3][3] in the same
 * canonical layout as the fat links, phases and boundary signs folded in.
 * Packed to FP16 inside the handle (entries of unitary links are at most 1 in
 * magnitude); only read during the call.  Synchronous.
 * Errors: -1 if an entry is not finite or |entry| >= 32768. */
int hisq_gauge_set_thin(hisq_gauge_t g, const double *thin, void *stream);

/*
 * Create a network with `nlayers` layers and channel counts channels[0..nlayers]
 * (first and last 1, the others 1..8).  Weights: host complex double,
 * layer after layer, each [9][C_out][C_in] with path index 0 = identity,
 * 1 + mu = forward hop (U_mu(x) psi(x+mu)), 5 + mu = backward hop
 * (U_mu(x-mu)^+ psi(x-mu)); NULL = all zero.  The network owns its weights,
 * Adam state and activation buffers (sized for the handle's lattice).
 */
int hisq_nn_create(hisq_nn_t *out, hisq_gauge_t g, int nlayers, const int *channels, const double *weights,
                   void *stream);
int hisq_nn_destroy(hisq_nn_t net);
/* Number of complex weights (the length of the arrays below, in complex numbers). */
int hisq_nn_num_weights(hisq_nn_t net, size_t *n_complex);
/* Copy the weights to / from a host array of 2 * n_complex doubles. */
int hisq_nn_get_weights(hisq_nn_t net, double *weights, void *stream);
int hisq_nn_set_weights(hisq_nn_t net, const double *weights, void *stream);

/*
 * Loss and gradient over a batch of pairs (A v_i, v_i), i < batch:
 *   L = (1/batch) sum_i |N(A v_i) - v_i|^2 / |v_i|^2
 * av, v: device FP32 spinors [batch][one buffer] (even parity).  *loss gets L;
 * grad (host, 2 * n_complex doubles, or NULL) gets dL/dRe W + i dL/dIm W in the
 * weight layout.  Synchronous.
 */
int hisq_nn_loss_grad(hisq_nn_t net, int batch, const void *av, const void *v, double *loss, double *grad,
                      void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on the
 * gradient of the batch; *loss gets the loss before the step.  Synchronous. */
int hisq_nn_train_step(hisq_nn_t net, int batch, const void *av, const void *v, double lr, double *loss,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
