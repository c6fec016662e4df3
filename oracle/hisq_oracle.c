/*
 * FP64 CPU oracle for the even/odd HISQ staggered operator and its solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * Written for clarity, not speed: one site at a time, the natural
 * lexicographic site order lex = x + Lx*(y + Ly*(z + Lz*t)), an
 * array-of-structures layout and C99 complex arithmetic.  OpenMP only splits
 * the site loop.
 *
 * Layouts (complex values as interleaved re,im doubles):
 *   links  [V][4][3][3]  U[s][mu][a][b]; U_mu(s) maps colour at s+mu to s
 *   vector [V][3]        full lattice; the sites of the other parity are 0
 *
 * The operator (HISQ, Follana et al. 2007, cited in the paper's introduction;
 * the paper calls its application "the most performance-critical kernel"
 * inside CG, Sec. 3):
 *   (D chi)(x) = sum_mu [ F_mu(x) chi(x+mu) - F_mu(x-mu)^+ chi(x-mu)
 *                       + L_mu(x) chi(x+3mu) - L_mu(x-3mu)^+ chi(x-3mu) ]
 * with the staggered phases and boundary signs already folded into the fat
 * links F and the Naik links L.  D connects sites of opposite parity only.
 * Even/odd normal operator: A = 4 m^2 + sigma - D_eo D_oe on even sites,
 * which is (D^+ D + 4 m^2 + sigma) restricted to them because D^+ = -D.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

/* Site loops run on several threads only on lattices large enough to pay for
 * them (on the tiny test lattices the thread start-up costs more than the
 * work, and a busy host makes it far worse). */
#define OMP_MIN_SITES 32768

static long site_volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void lex_to_coords(const int L[4], long s, int c[4]) {
    c[0] = (int)(s % L[0]); s /= L[0];
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)s;
}

static long coords_to_lex(const int L[4], const int c[4]) {
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* Site reached from s by `dist` steps along mu, periodic wrap. */
static long neighbour(const int L[4], long s, int mu, int dist) {
    int c[4];
    lex_to_coords(L, s, c);
    c[mu] = ((c[mu] + dist) % L[mu] + L[mu]) % L[mu];
    return coords_to_lex(L, c);
}

static int parity_of(const int L[4], long s) {
    int c[4];
    lex_to_coords(L, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static const cplx *link_at(const cplx *U, long s, int mu) { return U + (s * 4 + mu) * 9; }

/* acc += sign * M v */
static void add_mv(cplx acc[3], const cplx *M, const cplx *v, double sign) {
    for (int a = 0; a < 3; ++a) {
        cplx t = 0;
        for (int b = 0; b < 3; ++b) t += M[a * 3 + b] * v[b];
        acc[a] += sign * t;
    }
}

/* acc += sign * M^+ v */
static void add_mdag_v(cplx acc[3], const cplx *M, const cplx *v, double sign) {
    for (int a = 0; a < 3; ++a) {
        cplx t = 0;
        for (int b = 0; b < 3; ++b) t += conj(M[b * 3 + a]) * v[b];
        acc[a] += sign * t;
    }
}

/* out = D in on the sites of out_parity; out = 0 on the other parity. */
void oracle_dslash(const int L[4], const double *fat_, const double *lng_,
                   const double *in_, double *out_, int out_parity) {
    const cplx *F = (const cplx *)fat_, *N = (const cplx *)lng_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = site_volume(L);
#pragma omp parallel for schedule(static) if (V >= OMP_MIN_SITES)
    for (long s = 0; s < V; ++s) {
        cplx acc[3] = {0, 0, 0};
        if (parity_of(L, s) == out_parity) {
            for (int mu = 0; mu < 4; ++mu) {
                long f1 = neighbour(L, s, mu, +1), b1 = neighbour(L, s, mu, -1);
                long f3 = neighbour(L, s, mu, +3), b3 = neighbour(L, s, mu, -3);
                add_mv(acc, link_at(F, s, mu), in + f1 * 3, +1.0);
                add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, -1.0);
                add_mv(acc, link_at(N, s, mu), in + f3 * 3, +1.0);
                add_mdag_v(acc, link_at(N, b3, mu), in + b3 * 3, -1.0);
            }
        }
        for (int a = 0; a < 3; ++a) out[s * 3 + a] = acc[a];
    }
}

/* The same sum evaluated only at the listed sites (any parity): out[i][3] =
 * (D in)(sites[i]).  Lets a huge lattice be checked at sampled outputs. */
void oracle_dslash_sites(const int L[4], const double *fat_, const double *lng_, const double *in_,
                         const int64_t *sites, long nsites, double *out_) {
    const cplx *F = (const cplx *)fat_, *N = (const cplx *)lng_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
#pragma omp parallel for schedule(static) if (nsites >= 256)
    for (long i = 0; i < nsites; ++i) {
        const long s = (long)sites[i];
        cplx acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            long f1 = neighbour(L, s, mu, +1), b1 = neighbour(L, s, mu, -1);
            long f3 = neighbour(L, s, mu, +3), b3 = neighbour(L, s, mu, -3);
            add_mv(acc, link_at(F, s, mu), in + f1 * 3, +1.0);
            add_mdag_v(acc, link_at(F, b1, mu), in + b1 * 3, -1.0);
            add_mv(acc, link_at(N, s, mu), in + f3 * 3, +1.0);
            add_mdag_v(acc, link_at(N, b3, mu), in + b3 * 3, -1.0);
        }
        for (int a = 0; a < 3; ++a) out[i * 3 + a] = acc[a];
    }
}

/* Staggered phase eta_mu(x): 1, (-1)^x, (-1)^(x+y), (-1)^(x+y+z). */
static double eta_of(const int c[4], int mu) {
    int e = 0;
    for (int nu = 0; nu < mu; ++nu) e += c[nu];
    return (e & 1) ? -1.0 : 1.0;
}

/*
 * The same operator on links WITHOUT phases or boundary signs: the phases
 * eta_mu and, if antiperiodic_t, a factor -1 on every hop that crosses the
 * time boundary are applied here explicitly.  Used to pin the folding done
 * by the input generator.
 */
void oracle_dslash_phased(const int L[4], const double *fat_, const double *lng_,
                          const double *in_, double *out_, int out_parity, int antiperiodic_t) {
    const cplx *F = (const cplx *)fat_, *N = (const cplx *)lng_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = site_volume(L);
#pragma omp parallel for schedule(static) if (V >= OMP_MIN_SITES)
    for (long s = 0; s < V; ++s) {
        cplx acc[3] = {0, 0, 0};
        int c[4];
        lex_to_coords(L, s, c);
        if (((c[0] + c[1] + c[2] + c[3]) & 1) == out_parity) {
            for (int mu = 0; mu < 4; ++mu) {
                const double eta = eta_of(c, mu); /* same at x - k mu: eta_mu ignores x_mu */
                for (int k = 1; k <= 3; k += 2) {
                    const cplx *links = (k == 1) ? F : N;
                    long fw = neighbour(L, s, mu, +k), bw = neighbour(L, s, mu, -k);
                    double sf = eta, sb = eta;
                    if (antiperiodic_t && mu == 3) {
                        if (c[3] + k >= L[3]) sf = -sf; /* forward path wraps */
                        if (c[3] - k < 0) sb = -sb;     /* backward path wraps */
                    }
                    add_mv(acc, link_at(links, s, mu), in + fw * 3, sf);
                    add_mdag_v(acc, link_at(links, bw, mu), in + bw * 3, -sb);
                }
            }
        }
        for (int a = 0; a < 3; ++a) out[s * 3 + a] = acc[a];
    }
}

/* out_e = (4 m^2 + sigma) in_e - D_eo (D_oe in_e); odd sites of out = 0.
 * tmp: caller scratch of the same size as a vector. */
void oracle_normal_op(const int L[4], const double *fat, const double *lng, double mass,
                      double sigma, const double *in_, double *out_, double *tmp) {
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    const long V = site_volume(L);
    oracle_dslash(L, fat, lng, in_, tmp, 1);
    oracle_dslash(L, fat, lng, tmp, out_, 0);
    const double diag = 4.0 * mass * mass + sigma;
#pragma omp parallel for schedule(static) if (V >= OMP_MIN_SITES)
    for (long s = 0; s < V; ++s) {
        if (parity_of(L, s) != 0) continue;
        for (int a = 0; a < 3; ++a) out[s * 3 + a] = diag * in[s * 3 + a] - out[s * 3 + a];
    }
}

/* <u, v> = sum conj(u) v over all components (odd sites are zero). */
static cplx vdot(long n, const cplx *u, const cplx *v) {
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static) if (n >= 3 * OMP_MIN_SITES)
    for (long i = 0; i < n; ++i) {
        cplx t = conj(u[i]) * v[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

/* Relative true residual |b - A x| / |b|. */
double oracle_true_residual(const int L[4], const double *fat, const double *lng, double mass,
                            double sigma, const double *b_, const double *x_) {
    const long n = site_volume(L) * 3;
    cplx *Ax = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    const cplx *b = (const cplx *)b_;
    oracle_normal_op(L, fat, lng, mass, sigma, x_, (double *)Ax, (double *)tmp);
    for (long i = 0; i < n; ++i) Ax[i] = b[i] - Ax[i];
    double r = sqrt(creal(vdot(n, Ax, Ax))), bn = sqrt(creal(vdot(n, b, b)));
    free(Ax);
    free(tmp);
    return bn > 0 ? r / bn : r;
}

/*
 * Conjugate gradient on A + sigma (Hestenes-Stiefel), started from x = 0.
 * Stops when the TRUE residual |b - A x| <= tol |b|: whenever the iterated
 * residual reaches tol, r is recomputed from x and the loop continues from it
 * if the true residual has not.
 * Returns 0 converged, 1 not converged in max_iter, 2 breakdown.
 */
int oracle_cg(const int L[4], const double *fat, const double *lng, double mass, double sigma,
              const double *b_, double *x_, double tol, int max_iter, int *iters_out,
              double *true_res_out) {
    const long n = site_volume(L) * 3;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *tmp = malloc(sizeof(cplx) * n);
    for (long i = 0; i < n; ++i) { x[i] = 0; r[i] = b[i]; p[i] = b[i]; }
    const double bnorm = sqrt(creal(vdot(n, b, b)));
    double rho = creal(vdot(n, r, r));
    int status = 1, k = 0;
    if (bnorm == 0.0) { status = 0; goto done; }
    for (k = 0; k < max_iter;) {
        oracle_normal_op(L, fat, lng, mass, sigma, (double *)p, (double *)q, (double *)tmp);
        double pq = creal(vdot(n, p, q));
        if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
        double alpha = rho / pq;
        for (long i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rho_new = creal(vdot(n, r, r));
        ++k;
        if (sqrt(rho_new) <= tol * bnorm) {
            oracle_normal_op(L, fat, lng, mass, sigma, (double *)x, (double *)q, (double *)tmp);
            for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
            rho_new = creal(vdot(n, r, r));
            if (sqrt(rho_new) <= tol * bnorm) { status = 0; break; }
        }
        double beta = rho_new / rho;
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
done:
    if (iters_out) *iters_out = k;
    if (true_res_out) *true_res_out = oracle_true_residual(L, fat, lng, mass, sigma, b_, x_);
    free(r); free(p); free(q); free(tmp);
    return status;
}

/* Number of OpenMP threads the oracle's loops use. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
