// The C ABI from a plain host program, without Python or torch: device
// memory from the HIP runtime, the entry points of include/hisq.h, and the C
// oracle (oracle/hisq_oracle.c) as the arbiter.  On an 8^4 lattice with random
// (non-unitary) fat and Naik links it checks
//  * hisq_dslash_eo (FP64, both output parities) against oracle_dslash;
//  * hisq_dslash_multi_rhs with the (A + sigma_i) epilogue (FP64, 3 RHS)
//    against oracle_normal_op;
//  * hisq_cg_solve (plain FP64 and mixed FP32, 2 RHS) and hisq_multishift_cg
//    (FP64 and mixed, 3 shifts) on the oracle's true residual, and
//    hisq_multishift_cg_batched (FP64 and mixed, 2 sources x 2 shifts);
//  * that bad arguments return HISQ_ERR_INVALID with a message.
// Prints one line per check and exits non-zero on the first failure.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hisq.h"

extern "C" {
void oracle_dslash(const int L[4], const double *fat, const double *lng, const double *in, double *out,
                   int out_parity);
void oracle_normal_op(const int L[4], const double *fat, const double *lng, double mass, double sigma,
                      const double *in, double *out, double *tmp);
double oracle_true_residual(const int L[4], const double *fat, const double *lng, double mass, double sigma,
                            const double *b, const double *x);
}

static int fails = 0;
#define CHECK(cond, ...)                       \
    do {                                       \
        if (!(cond)) {                         \
            std::fprintf(stderr, "FAIL: ");    \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");        \
            ++fails;                           \
        }                                      \
    } while (0)
#define HIP(x)                                                                           \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            std::exit(2);                                                                \
        }                                                                                \
    } while (0)

// deterministic uniform numbers in [-1, 1) (a 64-bit LCG, Knuth's constants)
static unsigned long long lcg_state = 0x2111103542ULL;
static double uniform() {
    lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static const int L[4] = {8, 8, 8, 8};
static const long V = 8L * 8 * 8 * 8, VH = V / 2;

static int parity_of(long s) {
    const int x = (int)(s % L[0]), y = (int)(s / L[0] % L[1]), z = (int)(s / (L[0] * L[1]) % L[2]),
              t = (int)(s / (L[0] * L[1] * L[2]));
    return (x + y + z + t) & 1;
}

// full lattice [V][3] complex <-> the library's FP64 parity layout [3][Vh] complex (h = lex / 2)
static std::vector<double> to_parity(const std::vector<double> &full, int parity) {
    std::vector<double> p(6 * VH);
    for (long s = 0; s < V; ++s)
        if (parity_of(s) == parity)
            for (int c = 0; c < 3; ++c) {
                p[2 * (c * VH + s / 2)] = full[2 * (3 * s + c)];
                p[2 * (c * VH + s / 2) + 1] = full[2 * (3 * s + c) + 1];
            }
    return p;
}
static std::vector<double> from_parity(const std::vector<double> &p, int parity) {
    std::vector<double> full(6 * V, 0.0);
    for (long s = 0; s < V; ++s)
        if (parity_of(s) == parity)
            for (int c = 0; c < 3; ++c) {
                full[2 * (3 * s + c)] = p[2 * (c * VH + s / 2)];
                full[2 * (3 * s + c) + 1] = p[2 * (c * VH + s / 2) + 1];
            }
    return full;
}
static std::vector<double> random_field(int parity) {
    std::vector<double> f(6 * V, 0.0);
    for (long s = 0; s < V; ++s)
        if (parity_of(s) == parity)
            for (int k = 0; k < 6; ++k) f[6 * s + k] = uniform();
    return f;
}
static double rel_l2(const std::vector<double> &a, const std::vector<double> &b) {
    double d = 0, n = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        d += (a[i] - b[i]) * (a[i] - b[i]);
        n += b[i] * b[i];
    }
    return std::sqrt(d / n);
}

struct Dev {
    void *p = nullptr;
    explicit Dev(size_t n) { HIP(hipMalloc(&p, n)); }
    ~Dev() { (void)hipFree(p); }
};

int main() {
    const size_t nlink = (size_t)V * 4 * 9 * 2;
    std::vector<double> fat(nlink), lng(nlink);
    for (size_t i = 0; i < nlink; ++i) fat[i] = 0.3 * uniform();
    for (size_t i = 0; i < nlink; ++i) lng[i] = 0.1 * uniform();
    Dev dfat(nlink * 8), dlng(nlink * 8);
    HIP(hipMemcpy(dfat.p, fat.data(), nlink * 8, hipMemcpyHostToDevice));
    HIP(hipMemcpy(dlng.p, lng.data(), nlink * 8, hipMemcpyHostToDevice));
    hisq_gauge_t g = nullptr;
    int rc = hisq_gauge_create(&g, L, (const double *)dfat.p, (const double *)dlng.p,
                               HISQ_PREC_MASK(HISQ_PREC_FP64) | HISQ_PREC_MASK(HISQ_PREC_FP32), nullptr);
    CHECK(rc == HISQ_OK && g, "hisq_gauge_create: %d %s", rc, hisq_last_error());
    if (!g) return 1;
    CHECK(hisq_version() == HISQ_VERSION, "hisq_version %d, header %d", hisq_version(), HISQ_VERSION);
    const size_t sb = 6 * VH * sizeof(double);

    // single-parity Dslash, both output parities
    for (int par = 0; par < 2; ++par) {
        const std::vector<double> chi = random_field(1 - par);
        const std::vector<double> in = to_parity(chi, 1 - par);
        Dev din(sb), dout(sb);
        HIP(hipMemcpy(din.p, in.data(), sb, hipMemcpyHostToDevice));
        rc = hisq_dslash_eo(g, par, HISQ_PREC_FP64, din.p, dout.p, nullptr);
        CHECK(rc == HISQ_OK, "hisq_dslash_eo: %d %s", rc, hisq_last_error());
        HIP(hipDeviceSynchronize());
        std::vector<double> got(6 * VH), want(6 * V);
        HIP(hipMemcpy(got.data(), dout.p, sb, hipMemcpyDeviceToHost));
        oracle_dslash(L, fat.data(), lng.data(), chi.data(), want.data(), par);
        const double err = rel_l2(from_parity(got, par), want);
        std::printf("dslash_eo FP64 parity %d: rel L2 %.2e\n", par, err);
        CHECK(err <= 1e-13, "dslash_eo parity %d: %.3e", par, err);
    }

    // multi-RHS Dslash with the (A + sigma_i) epilogue: out_i = diag_i y_i - D_eo (D_oe y_i)
    {
        const int n = 3;
        const double mass = 0.1, sig[n] = {0.0, 0.05, 0.3};
        double diag[n];
        for (int i = 0; i < n; ++i) diag[i] = 4 * mass * mass + sig[i];
        std::vector<std::vector<double>> ys(n);
        std::vector<double> stack(n * 6 * VH);
        for (int i = 0; i < n; ++i) {
            ys[i] = random_field(0);
            const std::vector<double> p = to_parity(ys[i], 0);
            std::memcpy(stack.data() + i * 6 * VH, p.data(), sb);
        }
        Dev dy(n * sb), dt(n * sb), dout(n * sb);
        HIP(hipMemcpy(dy.p, stack.data(), n * sb, hipMemcpyHostToDevice));
        rc = hisq_dslash_multi_rhs(g, 1, HISQ_PREC_FP64, n, dy.p, dt.p, nullptr, nullptr, nullptr);
        CHECK(rc == HISQ_OK, "multi_rhs plain: %d %s", rc, hisq_last_error());
        rc = hisq_dslash_multi_rhs(g, 0, HISQ_PREC_FP64, n, dt.p, dout.p, diag, dy.p, nullptr);
        CHECK(rc == HISQ_OK, "multi_rhs epilogue: %d %s", rc, hisq_last_error());
        HIP(hipDeviceSynchronize());
        std::vector<double> got(n * 6 * VH), want(6 * V), tmp(6 * V);
        HIP(hipMemcpy(got.data(), dout.p, n * sb, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) {
            oracle_normal_op(L, fat.data(), lng.data(), mass, sig[i], ys[i].data(), want.data(), tmp.data());
            std::vector<double> gi(got.begin() + i * 6 * VH, got.begin() + (i + 1) * 6 * VH);
            const double err = rel_l2(from_parity(gi, 0), want);
            std::printf("multi_rhs epilogue RHS %d: rel L2 %.2e\n", i, err);
            CHECK(err <= 1e-13, "multi_rhs epilogue RHS %d: %.3e", i, err);
        }
    }

    // CG: plain FP64 and mixed FP32, two RHS in one batch
    const double mass = 0.1;
    for (int sloppy : {HISQ_PREC_FP64, HISQ_PREC_FP32}) {
        const int n = 2;
        std::vector<std::vector<double>> bs(n);
        std::vector<double> stack(n * 6 * VH);
        for (int i = 0; i < n; ++i) {
            bs[i] = random_field(0);
            const std::vector<double> p = to_parity(bs[i], 0);
            std::memcpy(stack.data() + i * 6 * VH, p.data(), sb);
        }
        Dev db(n * sb), dx(n * sb);
        HIP(hipMemcpy(db.p, stack.data(), n * sb, hipMemcpyHostToDevice));
        hisq_solver_params prm;
        hisq_solver_params_default(&prm);
        prm.sloppy_prec = sloppy;
        hisq_solver_stats st[n];
        rc = hisq_cg_solve(g, mass, n, (const double *)db.p, (double *)dx.p, &prm, st, nullptr);
        CHECK(rc == HISQ_OK, "cg sloppy %d: %d %s", sloppy, rc, hisq_last_error());
        HIP(hipMemcpy(stack.data(), dx.p, n * sb, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) {
            std::vector<double> xi(stack.begin() + i * 6 * VH, stack.begin() + (i + 1) * 6 * VH);
            const double res = oracle_true_residual(L, fat.data(), lng.data(), mass, 0.0, bs[i].data(),
                                                    from_parity(xi, 0).data());
            std::printf("cg sloppy %d RHS %d: %d iterations, oracle true residual %.2e\n", sloppy, i,
                        st[i].iterations, res);
            CHECK(res <= 1e-10 && st[i].status == HISQ_OK, "cg sloppy %d RHS %d: %.3e", sloppy, i, res);
        }
    }

    // multi-shift CG, FP64 and mixed
    for (int sloppy : {HISQ_PREC_FP64, HISQ_PREC_FP32}) {
        const int ns = 3;
        const double shifts[ns] = {0.2, 0.0, 0.01};
        const std::vector<double> b = random_field(0), bp = to_parity(b, 0);
        Dev db(sb), dx(ns * sb);
        HIP(hipMemcpy(db.p, bp.data(), sb, hipMemcpyHostToDevice));
        hisq_solver_params prm;
        hisq_solver_params_default(&prm);
        prm.sloppy_prec = sloppy;
        hisq_solver_stats st[ns];
        rc = hisq_multishift_cg(g, mass, ns, shifts, (const double *)db.p, (double *)dx.p, &prm, st, nullptr);
        CHECK(rc == HISQ_OK, "multishift sloppy %d: %d %s", sloppy, rc, hisq_last_error());
        std::vector<double> xs(ns * 6 * VH);
        HIP(hipMemcpy(xs.data(), dx.p, ns * sb, hipMemcpyDeviceToHost));
        for (int k = 0; k < ns; ++k) {
            std::vector<double> xk(xs.begin() + k * 6 * VH, xs.begin() + (k + 1) * 6 * VH);
            const double res = oracle_true_residual(L, fat.data(), lng.data(), mass, shifts[k], b.data(),
                                                    from_parity(xk, 0).data());
            std::printf("multishift sloppy %d shift %g: oracle true residual %.2e\n", sloppy, shifts[k], res);
            CHECK(res <= 1e-10, "multishift sloppy %d shift %d: %.3e", sloppy, k, res);
        }
    }

    // two sources with the same shifts in one call, in lockstep through the
    // 2-RHS Dslash (FP32 Krylov vectors in the mixed form, FP64 otherwise)
    for (int sloppy : {HISQ_PREC_FP32, HISQ_PREC_FP64}) {
        const int ns = 2, m = 2;
        const double shifts[ns] = {0.05, 0.0};
        std::vector<std::vector<double>> bs;
        std::vector<double> stack;
        for (int j = 0; j < m; ++j) {
            bs.push_back(random_field(0));
            const std::vector<double> bp = to_parity(bs[j], 0);
            stack.insert(stack.end(), bp.begin(), bp.end());
        }
        Dev db(m * sb), dx(m * ns * sb);
        HIP(hipMemcpy(db.p, stack.data(), m * sb, hipMemcpyHostToDevice));
        hisq_solver_params prm;
        hisq_solver_params_default(&prm);
        prm.sloppy_prec = sloppy;
        hisq_solver_stats st[m * ns];
        rc = hisq_multishift_cg_batched(g, mass, m, ns, shifts, (const double *)db.p, (double *)dx.p, &prm, st,
                                        nullptr);
        CHECK(rc == HISQ_OK, "batched multishift sloppy %d: %d %s", sloppy, rc, hisq_last_error());
        std::vector<double> xs(m * ns * 6 * VH);
        HIP(hipMemcpy(xs.data(), dx.p, m * ns * sb, hipMemcpyDeviceToHost));
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < ns; ++k) {
                const size_t at = (size_t)(j * ns + k) * 6 * VH;
                std::vector<double> xk(xs.begin() + at, xs.begin() + at + 6 * VH);
                const double res = oracle_true_residual(L, fat.data(), lng.data(), mass, shifts[k], bs[j].data(),
                                                        from_parity(xk, 0).data());
                std::printf("batched multishift sloppy %d source %d shift %g: oracle true residual %.2e\n", sloppy, j,
                            shifts[k], res);
                CHECK(res <= 1e-10 && st[j * ns + k].status == HISQ_OK, "batched multishift %d %d: %.3e", j, k, res);
            }
        rc = hisq_multishift_cg_batched(g, mass, 0, ns, shifts, (const double *)db.p, (double *)dx.p, &prm, st,
                                        nullptr);
        CHECK(rc == HISQ_ERR_INVALID, "nsrc 0: %d", rc);
    }

    // error paths
    {
        Dev a(sb), b(sb);
        rc = hisq_dslash_eo(g, 2, HISQ_PREC_FP64, a.p, b.p, nullptr);
        CHECK(rc == HISQ_ERR_INVALID && std::strlen(hisq_last_error()) > 0, "bad parity: %d", rc);
        rc = hisq_dslash_eo(g, 0, HISQ_PREC_FP64, a.p, a.p, nullptr);
        CHECK(rc == HISQ_ERR_INVALID, "in == out: %d", rc);
        hisq_solver_params prm;
        hisq_solver_params_default(&prm);
        prm.ru_delta = 1.5;
        rc = hisq_cg_solve(g, 0.1, 1, (const double *)a.p, (double *)b.p, &prm, nullptr, nullptr);
        CHECK(rc == HISQ_ERR_INVALID, "ru_delta 1.5: %d", rc);
        std::printf("error paths: %s\n", fails ? "FAILED" : "ok");
    }
    CHECK(hisq_gauge_destroy(g) == HISQ_OK, "destroy");
    std::printf("%s\n", fails ? "FAILED" : "all C-ABI checks passed");
    return fails ? 1 : 0;
}
