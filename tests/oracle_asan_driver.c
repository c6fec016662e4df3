/* Memory-safety drive of the FP64 oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code; built and run by
 * tests/test_oracle_asan.py).  Random, non-unitary fields are enough: the
 * point is every index the oracle computes on a ragged lattice. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_dslash(const int L[4], const double *fat, const double *lng, const double *in, double *out,
                   int out_parity);
void oracle_dslash_sites(const int L[4], const double *fat, const double *lng, const double *in,
                         const int64_t *sites, long nsites, double *out);
void oracle_dslash_phased(const int L[4], const double *fat, const double *lng, const double *in, double *out,
                          int out_parity, int antiperiodic_t);
void oracle_normal_op(const int L[4], const double *fat, const double *lng, double mass, double sigma,
                      const double *in, double *out, double *tmp);
double oracle_true_residual(const int L[4], const double *fat, const double *lng, double mass, double sigma,
                            const double *b, const double *x);
int oracle_cg(const int L[4], const double *fat, const double *lng, double mass, double sigma, const double *b,
              double *x, double tol, int max_iter, int *iters_out, double *true_res_out);

static uint64_t state = 0x2111103540ull;
static double rnd(void) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static int parity(const int L[4], long s) {
    int c[4];
    for (int i = 0; i < 4; ++i) {
        c[i] = (int)(s % L[i]);
        s /= L[i];
    }
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static int run(const int L[4]) {
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    double *fat = malloc(sizeof(double) * V * 4 * 18), *lng = malloc(sizeof(double) * V * 4 * 18);
    double *in = calloc(V * 6, sizeof(double)), *out = calloc(V * 6, sizeof(double));
    double *tmp = calloc(V * 6, sizeof(double)), *x = calloc(V * 6, sizeof(double));
    for (long i = 0; i < V * 4 * 18; ++i) {
        fat[i] = 0.3 * rnd();
        lng[i] = 0.1 * rnd();
    }
    for (int i = 0; i < 4; ++i) {  /* diagonal: keep A well conditioned */
        for (long s = 0; s < V; ++s) fat[(s * 4 + i) * 18 + 0] += 0.5;
    }
    for (long s = 0; s < V; ++s)
        if (parity(L, s) == 1)
            for (int c = 0; c < 6; ++c) in[s * 6 + c] = rnd();
    oracle_dslash(L, fat, lng, in, out, 0);
    oracle_dslash_phased(L, fat, lng, in, out, 0, 1);
    int64_t sites[5] = {0, 2, 4, 6, 8};
    double sout[5 * 6];
    oracle_dslash_sites(L, fat, lng, in, sites, 5, sout);
    for (long s = 0; s < V; ++s)
        for (int c = 0; c < 6; ++c) in[s * 6 + c] = parity(L, s) == 0 ? rnd() : 0.0;
    oracle_normal_op(L, fat, lng, 0.5, 0.0, in, out, tmp);
    int iters = 0;
    double tr = 0.0;
    oracle_cg(L, fat, lng, 0.5, 0.1, in, x, 1e-8, 200, &iters, &tr);
    const double r = oracle_true_residual(L, fat, lng, 0.5, 0.1, in, x);
    printf("L = %d %d %d %d: cg %d iterations, true residual %.2e / %.2e\n", L[0], L[1], L[2], L[3], iters, tr, r);
    free(fat);
    free(lng);
    free(in);
    free(out);
    free(tmp);
    free(x);
    return isfinite(r) ? 0 : 1;
}

int main(void) {
    const int shapes[3][4] = {{4, 4, 4, 4}, {6, 4, 4, 10}, {4, 6, 8, 6}};
    int rc = 0;
    for (int k = 0; k < 3; ++k) rc |= run(shapes[k]);
    return rc;
}
