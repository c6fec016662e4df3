// C ABI of the library: argument validation, handle life cycle, error codes.
// Every entry point validates its arguments on the host before touching the
// GPU; invalid arguments return HISQ_ERR_INVALID without any HIP call.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "solver_internal.h"

namespace hisq {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *get_error() { return g_last_error.c_str(); }

static int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

static bool valid_prec(int p) { return p == HISQ_PREC_FP64 || p == HISQ_PREC_FP32 || p == HISQ_PREC_FP16S; }
// sloppy modes of the solvers: a spinor precision, or FP16 links with FP32 vectors
static bool valid_sloppy(int p) { return valid_prec(p) || p == HISQ_PREC_FP16L; }

static int check_dims(const int *dims) {
    if (!dims) return fail(HISQ_ERR_INVALID, "dims is NULL");
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        if (dims[i] < 4 || (dims[i] & 1))
            return fail(HISQ_ERR_INVALID, "every lattice extent must be even and >= 4");
        v *= dims[i];
    }
    if (v >= ((int64_t)1 << 31)) return fail(HISQ_ERR_INVALID, "lattice volume must be below 2^31");
    return HISQ_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static int check_spinors(const void *a, const void *b, const void *c = nullptr) {
    if (!aligned16(a) || !aligned16(b) || (c && !aligned16(c)))
        return fail(HISQ_ERR_INVALID, "spinor buffers must be 16-byte aligned");
    return HISQ_OK;
}

// Two device buffers of na and nb bytes share memory (compared as addresses).
static bool bytes_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    return pa < pb + nb && pb < pa + na;
}

static int check_handle(hisq_gauge_t g) {
    if (!g) return fail(HISQ_ERR_INVALID, "gauge handle is NULL");
    return HISQ_OK;
}

static int check_params(const hisq_solver_params &p) {
    if (!(p.tol > 0.0) || !std::isfinite(p.tol)) return fail(HISQ_ERR_INVALID, "tol must be positive");
    if (p.max_iter < 1) return fail(HISQ_ERR_INVALID, "max_iter must be >= 1");
    if (!valid_sloppy(p.sloppy_prec)) return fail(HISQ_ERR_INVALID, "bad sloppy_prec");
    if (p.graph_chunk < 0 || p.graph_chunk > 4096) return fail(HISQ_ERR_INVALID, "graph_chunk out of range");
    if (!(p.ru_delta >= 0.0 && p.ru_delta < 1.0)) return fail(HISQ_ERR_INVALID, "ru_delta must be in [0, 1)");
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

TraceRange::TraceRange(const char *name) { roctxRangePush(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

hisq_gauge_s::~hisq_gauge_s() {
    cg_ws.clear();
    fcg_ws.reset();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    if (diag_event) (void)hipEventDestroy(diag_event);
}

extern "C" {

int hisq_version(void) { return HISQ_VERSION; }

const char *hisq_last_error(void) { return get_error(); }

size_t hisq_spinor_bytes(int prec, int64_t vh) {
    if (!valid_prec(prec) || vh < 0) return 0;
    return spinor_bytes(prec, vh);
}

void hisq_solver_params_default(hisq_solver_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-10;
    p->max_iter = 100000;
    p->sloppy_prec = HISQ_PREC_FP64;
    p->ru_period = 100;
    p->graph_chunk = 32;
    p->warm_start = 0;
    p->fallback = 1;
    p->precond = nullptr;
    p->ru_delta = 0.1;
}

int hisq_gauge_create(hisq_gauge_t *out, const int dims[4], const double *fat, const double *lng,
                      unsigned prec_mask, void *stream) {
    TraceRange tr_("hisq_gauge_create");
    if (!out) return fail(HISQ_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!fat || !lng) return fail(HISQ_ERR_INVALID, "fat and long link pointers are required");
    if ((prec_mask & HISQ_PREC_MASK_ALL) == 0 || (prec_mask & ~(HISQ_PREC_MASK_ALL | HISQ_LINKS_FULL)))
        return fail(HISQ_ERR_INVALID, "prec_mask must be a nonzero combination of HISQ_PREC_MASK bits "
                                      "(plus optionally HISQ_LINKS_FULL)");
    hipStream_t s = (hipStream_t)stream;
    hisq_gauge_s *g = new (std::nothrow) hisq_gauge_s();
    if (!g) return fail(HISQ_ERR_OOM, "host allocation failed");
    std::memcpy(g->dims, dims, sizeof(g->dims));
    g->geom = make_geom(dims);
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) {
        delete g;
        return fail(HISQ_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    DevBuf maxabs;
    if ((rc = maxabs.alloc(2 * sizeof(float)))) {
        delete g;
        return rc;
    }
    if (!(prec_mask & HISQ_LINKS_FULL)) {
        // compress the long links when every one is unitary with det +-1
        // (sign bits), or else when every one is a positive multiple of a
        // unitary matrix (complex factor per link)
        e = hipMemsetAsync(maxabs.p, 0, 2 * sizeof(float), s);
        float defect[2] = {1.f, 1.f};
        if (e == hipSuccess) {
            launch_long_link_defect(g->geom, lng, (unsigned *)maxabs.p, s);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(defect, maxabs.p, 2 * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete g;
            return fail(HISQ_ERR_HIP, std::string("long-link check: ") + hipGetErrorString(e));
        }
        g->comp_mode = defect[0] <= 1e-12f ? COMP_SIGN : defect[1] <= 1e-12f ? COMP_KAPPA : COMP_NONE;
    }
    for (int f = 0; f < 3; ++f) {
        if (!(prec_mask & HISQ_PREC_MASK(f))) continue;
        const size_t bytes = link_parity_bytes(f, g->geom.vh, links_compressed(g, f));
        if ((rc = g->links[f][0].alloc(bytes)) || (rc = g->links[f][1].alloc(bytes))) {
            delete g;
            return rc;
        }
        float *mb = nullptr;
        if (f == H16) {
            e = hipMemsetAsync(maxabs.p, 0, sizeof(float), s);
            mb = (float *)maxabs.p;
        }
        if (e == hipSuccess)
            rc = launch_pack_links(g->geom, f, fat, lng, g->links[f][0].p, g->links[f][1].p, mb,
                                   links_compressed(g, f), s);
        if (e != hipSuccess || rc) {
            delete g;
            return rc ? rc : fail(HISQ_ERR_HIP, hipGetErrorString(e));
        }
        if (f == H16) {
            float m = 0.f;
            e = hipMemcpyAsync(&m, maxabs.p, sizeof(float), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                delete g;
                return fail(HISQ_ERR_HIP, hipGetErrorString(e));
            }
            if (!(m < 16384.f)) {
                delete g;
                return fail(HISQ_ERR_INVALID, "link entries too large (or non-finite) for FP16 storage");
            }
        }
    }
    e = hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->diag_event, hipEventDisableTiming);
    // epilogue coefficients of up to 64 right-hand sides without a later allocation
    if (e == hipSuccess && (rc = g->diag_buf.alloc(sizeof(double) * 64))) {
        delete g;
        return rc;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete g;
        return fail(HISQ_ERR_HIP, std::string("create: ") + hipGetErrorString(e));
    }
    *out = g;
    return HISQ_OK;
}

int hisq_smear_links(const int dims[4], const double *thin, double *fat, double *lng, unsigned flags,
                     void *stream) {
    TraceRange tr_("hisq_smear_links");
    int rc = check_dims(dims);
    if (rc) return rc;
    if (!thin || !fat || !lng) return fail(HISQ_ERR_INVALID, "thin, fat and lng are required");
    if (flags & ~HISQ_SMEAR_ANTIPERIODIC_T) return fail(HISQ_ERR_INVALID, "unknown smearing flags");
    if (!aligned16(thin) || !aligned16(fat) || !aligned16(lng))
        return fail(HISQ_ERR_INVALID, "link fields must be 16-byte aligned");
    const size_t n = (size_t)dims[0] * dims[1] * dims[2] * dims[3] * 4 * 9 * 16;
    if (bytes_overlap(thin, n, fat, n) || bytes_overlap(thin, n, lng, n) || bytes_overlap(fat, n, lng, n))
        return fail(HISQ_ERR_INVALID, "thin, fat and lng must not overlap");
    return smear_links(dims, thin, fat, lng, flags, (hipStream_t)stream);
}

int hisq_gauge_destroy(hisq_gauge_t g) {
    if (!g) return HISQ_OK;
    (void)hipDeviceSynchronize();
    delete g;
    return HISQ_OK;
}

int hisq_gauge_links_compressed(hisq_gauge_t g) {
    int rc = check_handle(g);
    if (rc) return rc;
    return g->comp_mode;
}

int hisq_gauge_device_bytes(hisq_gauge_t g, size_t *bytes) {
    int rc = check_handle(g);
    if (rc) return rc;
    if (!bytes) return fail(HISQ_ERR_INVALID, "bytes is NULL");
    size_t n = g->diag_buf.bytes;
    for (auto &f : g->links)
        for (auto &b : f) n += b.bytes;
    *bytes = n;
    return HISQ_OK;
}

int hisq_dslash_eo(hisq_gauge_t g, int out_parity, int prec, const void *in, void *out, void *stream) {
    int rc = check_handle(g);
    if (rc) return rc;
    if (out_parity != 0 && out_parity != 1) return fail(HISQ_ERR_INVALID, "out_parity must be 0 or 1");
    if (!valid_prec(prec)) return fail(HISQ_ERR_INVALID, "bad precision");
    if (!in || !out) return fail(HISQ_ERR_INVALID, "in and out are required");
    if ((rc = check_spinors(in, out))) return rc;
    const size_t sb = spinor_bytes(prec, g->geom.vh);
    if (bytes_overlap(in, sb, out, sb)) return fail(HISQ_ERR_INVALID, "in and out must not overlap");
    return gauge_dslash(g, out_parity, prec, prec, prec, 1, in, out, nullptr, nullptr, nullptr, nullptr,
                        (hipStream_t)stream);
}

}  // extern "C"

// Argument checks of the multi-RHS entry points.
int hisq::check_multi_rhs(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in, void *out,
                           const double *diag, const void *y) {
    int rc = check_handle(g);
    if (rc) return rc;
    if (out_parity != 0 && out_parity != 1) return fail(HISQ_ERR_INVALID, "out_parity must be 0 or 1");
    if (!valid_prec(prec)) return fail(HISQ_ERR_INVALID, "bad precision");
    if (nrhs < 1) return fail(HISQ_ERR_INVALID, "nrhs must be >= 1");
    if (!in || !out) return fail(HISQ_ERR_INVALID, "in and out are required");
    if ((diag == nullptr) != (y == nullptr)) return fail(HISQ_ERR_INVALID, "diag and y go together");
    if ((rc = check_spinors(in, out, y))) return rc;
    const size_t stack = spinor_bytes(prec, g->geom.vh) * (size_t)nrhs;
    if (bytes_overlap(in, stack, out, stack)) return fail(HISQ_ERR_INVALID, "in and out must not overlap");
    if (y && bytes_overlap(y, stack, out, stack)) return fail(HISQ_ERR_INVALID, "y and out must not overlap");
    if (diag)
        for (int i = 0; i < nrhs; ++i)
            if (!std::isfinite(diag[i])) return fail(HISQ_ERR_INVALID, "diag must be finite");
    return HISQ_OK;
}

extern "C" {

int hisq_dslash_multi_rhs(hisq_gauge_t g, int out_parity, int prec, int nrhs, const void *in, void *out,
                          const double *diag, const void *y, void *stream) {
    int rc = check_multi_rhs(g, out_parity, prec, nrhs, in, out, diag, y);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!diag) return gauge_dslash(g, out_parity, prec, prec, prec, nrhs, in, out, nullptr, nullptr, nullptr, nullptr, s);
    // The handle's coefficient buffer is reused by every epilogue call.  The
    // lock covers copy and launch, and each call's copy waits (on the device)
    // for the previous call's kernel, whatever stream either was issued on.
    std::lock_guard<std::mutex> lk(g->mu);
    const size_t need = sizeof(double) * nrhs;
    if (g->diag_buf.bytes < need) {
        HISQ_HIP_CHECK(hipEventSynchronize(g->diag_event));  // the old buffer may still be read
        if ((rc = g->diag_buf.alloc(need))) return rc;
    }
    HISQ_HIP_CHECK(hipStreamWaitEvent(s, g->diag_event, 0));
    HISQ_HIP_CHECK(hipMemcpyAsync(g->diag_buf.p, diag, need, hipMemcpyHostToDevice, s));
    if ((rc = gauge_dslash(g, out_parity, prec, prec, prec, nrhs, in, out, y, (const double *)g->diag_buf.p,
                           nullptr, nullptr, s)))
        return rc;
    HISQ_HIP_CHECK(hipEventRecord(g->diag_event, s));
    return HISQ_OK;
}

int hisq_cg_solve(hisq_gauge_t g, double mass, int nrhs, const double *b, double *x,
                  const hisq_solver_params *p, hisq_solver_stats *st, void *stream) {
    TraceRange tr_("hisq_cg_solve");
    int rc = check_handle(g);
    if (rc) return rc;
    hisq_solver_params prm;
    if (p) prm = *p;
    else hisq_solver_params_default(&prm);
    if ((rc = check_params(prm))) return rc;
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(HISQ_ERR_INVALID, "mass must be positive");
    if (nrhs < 1) return fail(HISQ_ERR_INVALID, "nrhs must be >= 1");
    if (!b || !x) return fail(HISQ_ERR_INVALID, "b and x are required");
    if ((rc = check_spinors(b, x))) return rc;
    const size_t stack = spinor_bytes(F64, g->geom.vh) * (size_t)nrhs;
    if (bytes_overlap(b, stack, x, stack)) return fail(HISQ_ERR_INVALID, "b and x must not overlap");
    std::lock_guard<std::mutex> lk(g->mu);
    if (prm.precond) {
        // flexible CG: one right-hand side after another
        const size_t sb = spinor_bytes(F64, g->geom.vh);
        int worst = HISQ_OK;
        for (int i = 0; i < nrhs; ++i) {
            rc = fcg_solve(g, mass, (const double *)((const char *)b + sb * i), (double *)((char *)x + sb * i),
                           prm, st ? st + i : nullptr, (hipStream_t)stream);
            if (rc < 0) return rc;
            if (status_severity(rc) > status_severity(worst)) worst = rc;
        }
        return worst;
    }
    return cg_solve_fallback(g, mass, nrhs, b, x, prm, st, (hipStream_t)stream);
}

// validation shared by the single- and multi-source multi-shift entry points
static int check_multishift(hisq_gauge_t g, double mass, int nsrc, int nshift, const double *shifts,
                            const double *b, double *x, const hisq_solver_params &prm) {
    int rc = check_params(prm);
    if (rc) return rc;
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(HISQ_ERR_INVALID, "mass must be positive");
    if (prm.precond) return fail(HISQ_ERR_UNSUPPORTED, "multi-shift CG takes no preconditioner");
    if (nsrc < 1 || nsrc > 64) return fail(HISQ_ERR_INVALID, "1 <= nsrc <= 64");
    if (nshift < 1 || nshift > 256 || !shifts)
        return fail(HISQ_ERR_INVALID, "1 <= nshift <= 256 and shifts are required");
    if (nsrc * nshift > 1024) return fail(HISQ_ERR_INVALID, "nsrc * nshift must not exceed 1024");
    for (int k = 0; k < nshift; ++k)
        if (!std::isfinite(shifts[k]) || !(shifts[k] + 4.0 * mass * mass > 0.0))
            return fail(HISQ_ERR_INVALID, "every shift must be finite with sigma + 4 m^2 > 0");
    if (!b || !x) return fail(HISQ_ERR_INVALID, "b and x are required");
    if ((rc = check_spinors(b, x))) return rc;
    const size_t sb = spinor_bytes(F64, g->geom.vh);
    if (bytes_overlap(b, sb * nsrc, x, sb * (size_t)nshift * nsrc)) return fail(HISQ_ERR_INVALID, "b and x must not overlap");
    if (!g->links[F64][0].p) return fail(HISQ_ERR_UNSUPPORTED, "the handle lacks packed FP64 links");
    return HISQ_OK;
}

int hisq_multishift_cg(hisq_gauge_t g, double mass, int nshift, const double *shifts, const double *b,
                       double *x, const hisq_solver_params *p, hisq_solver_stats *st, void *stream) {
    TraceRange tr_("hisq_multishift_cg");
    int rc = check_handle(g);
    if (rc) return rc;
    hisq_solver_params prm;
    if (p) prm = *p;
    else hisq_solver_params_default(&prm);
    if ((rc = check_multishift(g, mass, 1, nshift, shifts, b, x, prm))) return rc;
    std::lock_guard<std::mutex> lk(g->mu);
    return multishift_solve(g, mass, nshift, shifts, b, x, prm, st, (hipStream_t)stream);
}

int hisq_multishift_cg_batched(hisq_gauge_t g, double mass, int nsrc, int nshift, const double *shifts,
                               const double *b, double *x, const hisq_solver_params *p, hisq_solver_stats *st,
                               void *stream) {
    TraceRange tr_("hisq_multishift_cg_batched");
    int rc = check_handle(g);
    if (rc) return rc;
    hisq_solver_params prm;
    if (p) prm = *p;
    else hisq_solver_params_default(&prm);
    if ((rc = check_multishift(g, mass, nsrc, nshift, shifts, b, x, prm))) return rc;
    std::lock_guard<std::mutex> lk(g->mu);
    return multishift_solve_batched(g, mass, nsrc, nshift, shifts, b, x, prm, st, (hipStream_t)stream);
}

// The coefficient outputs of the rational-approximation routines are written
// one after another: none may share memory with another (alpha0 and delta are
// single doubles, alpha and shift npole each).
static int check_coefficient_outputs(int npole, const double *alpha0, const double *alpha, const double *shift,
                                     const double *delta) {
    const size_t one = sizeof(double), arr = sizeof(double) * (size_t)npole;
    if (bytes_overlap(alpha, arr, shift, arr)) return fail(HISQ_ERR_INVALID, "alpha and shift must not overlap");
    for (const double *a : {alpha, shift}) {
        if (bytes_overlap(alpha0, one, a, arr)) return fail(HISQ_ERR_INVALID, "alpha0 must not overlap alpha or shift");
        if (delta && bytes_overlap(delta, one, a, arr))
            return fail(HISQ_ERR_INVALID, "delta must not overlap alpha or shift");
    }
    if (delta && bytes_overlap(delta, one, alpha0, one)) return fail(HISQ_ERR_INVALID, "delta must not overlap alpha0");
    return HISQ_OK;
}

int hisq_zolotarev_inv_sqrt(double lmin, double lmax, int npole, double *alpha0, double *alpha, double *shift,
                            double *delta) {
    if (!(lmin > 0.0) || !std::isfinite(lmin) || !std::isfinite(lmax) || !(lmax > lmin))
        return fail(HISQ_ERR_INVALID, "need 0 < lmin < lmax, both finite");
    if (lmax / lmin > 1e14) return fail(HISQ_ERR_INVALID, "lmax / lmin must not exceed 1e14");
    if (npole < 1 || npole > 64) return fail(HISQ_ERR_INVALID, "1 <= npole <= 64");
    if (!alpha0 || !alpha || !shift) return fail(HISQ_ERR_INVALID, "alpha0, alpha and shift are required");
    int rc = check_coefficient_outputs(npole, alpha0, alpha, shift, delta);
    if (rc) return rc;
    return zolotarev_inv_sqrt(lmin, lmax, npole, alpha0, alpha, shift, delta);
}

int hisq_rational_remez(double power, double lmin, double lmax, int npole, double *alpha0, double *alpha,
                        double *shift, double *delta) {
    if (!std::isfinite(power) || !(std::fabs(power) >= 0.05 && std::fabs(power) <= 0.95))
        return fail(HISQ_ERR_INVALID, "the power must satisfy 0.05 <= |p| <= 0.95");
    if (!(lmin > 0.0) || !std::isfinite(lmin) || !std::isfinite(lmax) || !(lmax > lmin))
        return fail(HISQ_ERR_INVALID, "need 0 < lmin < lmax, both finite");
    if (lmax / lmin > 1e14) return fail(HISQ_ERR_INVALID, "lmax / lmin must not exceed 1e14");
    if (npole < 1 || npole > 64) return fail(HISQ_ERR_INVALID, "1 <= npole <= 64");
    if (!alpha0 || !alpha || !shift) return fail(HISQ_ERR_INVALID, "alpha0, alpha and shift are required");
    int rc = check_coefficient_outputs(npole, alpha0, alpha, shift, delta);
    if (rc) return rc;
    // below ~1e-12 relative error the alternation drowns in rounding: the
    // x^(-1/2) optimum on the same interval measures how close that is
    {
        std::vector<double> za(npole), zs(npole);
        double z0 = 0.0, zd = 0.0;
        int rc = zolotarev_inv_sqrt(lmin, lmax, npole, &z0, za.data(), zs.data(), &zd);
        if (rc) return rc;
        if (zd < 1e-12)
            return fail(HISQ_ERR_INVALID, "too many poles for this interval: the error would fall below 1e-12");
        if (zd > 0.5)
            return fail(HISQ_ERR_INVALID, "too few poles for this interval: the error would exceed 0.5");
    }
    return remez_power(power, lmin, lmax, npole, alpha0, alpha, shift, delta);
}

static int rational_apply_checked(hisq_gauge_t g, double mass, int nsrc, double alpha0, int nterm,
                                  const double *alpha, const double *shift, const double *b, double *out,
                                  const hisq_solver_params *p, hisq_solver_stats *st, void *stream) {
    int rc = check_handle(g);
    if (rc) return rc;
    hisq_solver_params prm;
    if (p) prm = *p;
    else hisq_solver_params_default(&prm);
    if ((rc = check_params(prm))) return rc;
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(HISQ_ERR_INVALID, "mass must be positive");
    if (prm.precond) return fail(HISQ_ERR_UNSUPPORTED, "rational apply takes no preconditioner");
    if (nsrc < 1 || nsrc > 64) return fail(HISQ_ERR_INVALID, "1 <= nsrc <= 64");
    if (nterm < 0 || nterm > 256) return fail(HISQ_ERR_INVALID, "0 <= nterm <= 256");
    if (nsrc * nterm > 1024) return fail(HISQ_ERR_INVALID, "nsrc * nterm must not exceed 1024");
    if (nterm > 0 && (!alpha || !shift)) return fail(HISQ_ERR_INVALID, "alpha and shift are required");
    if (!std::isfinite(alpha0)) return fail(HISQ_ERR_INVALID, "alpha0 must be finite");
    for (int k = 0; k < nterm; ++k)
        if (!std::isfinite(alpha[k]) || !std::isfinite(shift[k]) || !(shift[k] + 4.0 * mass * mass > 0.0))
            return fail(HISQ_ERR_INVALID, "every alpha and shift must be finite with shift + 4 m^2 > 0");
    if (!b || !out) return fail(HISQ_ERR_INVALID, "b and out are required");
    if ((rc = check_spinors(b, out))) return rc;
    const size_t sb = spinor_bytes(F64, g->geom.vh) * nsrc;
    if (bytes_overlap(b, sb, out, sb)) return fail(HISQ_ERR_INVALID, "b and out must not overlap");
    if (!g->links[F64][0].p) return fail(HISQ_ERR_UNSUPPORTED, "the handle lacks packed FP64 links");
    std::lock_guard<std::mutex> lk(g->mu);
    return rational_apply(g, mass, nsrc, alpha0, nterm, alpha, shift, b, out, prm, st, (hipStream_t)stream);
}

int hisq_rational_apply(hisq_gauge_t g, double mass, double alpha0, int nterm, const double *alpha,
                        const double *shift, const double *b, double *out, const hisq_solver_params *p,
                        hisq_solver_stats *st, void *stream) {
    TraceRange tr_("hisq_rational_apply");
    return rational_apply_checked(g, mass, 1, alpha0, nterm, alpha, shift, b, out, p, st, stream);
}

int hisq_rational_apply_batched(hisq_gauge_t g, double mass, int nsrc, double alpha0, int nterm,
                                const double *alpha, const double *shift, const double *b, double *out,
                                const hisq_solver_params *p, hisq_solver_stats *st, void *stream) {
    TraceRange tr_("hisq_rational_apply_batched");
    return rational_apply_checked(g, mass, nsrc, alpha0, nterm, alpha, shift, b, out, p, st, stream);
}

int hisq_spectral_bounds(hisq_gauge_t g, double mass, int iters, double *lmin, double *lmax, void *stream) {
    TraceRange tr_("hisq_spectral_bounds");
    int rc = check_handle(g);
    if (rc) return rc;
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(HISQ_ERR_INVALID, "mass must be positive");
    if (iters < 1 || iters > 100000) return fail(HISQ_ERR_INVALID, "1 <= iters <= 100000");
    if (!lmin || !lmax) return fail(HISQ_ERR_INVALID, "lmin and lmax are required");
    std::lock_guard<std::mutex> lk(g->mu);
    return spectral_bounds(g, mass, iters, lmin, lmax, (hipStream_t)stream);
}

int hisq_autotune(hisq_gauge_t g, int prec, int nrhs, const char *cache_path, void *stream) {
    TraceRange tr_("hisq_autotune");
    int rc = check_handle(g);
    if (rc) return rc;
    if (!valid_sloppy(prec)) return fail(HISQ_ERR_INVALID, "bad precision");
    if (nrhs < 1 || nrhs > 64) return fail(HISQ_ERR_INVALID, "nrhs must be in 1..64");
    const int fl = sloppy_link_fmt(prec), fv = sloppy_vec_fmt(prec);
    if (!g->links[fl][0].p) return fail(HISQ_ERR_UNSUPPORTED, "links of this precision were not packed");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g->mu);
    const int fq = fv == H16 ? F32 : fv;
    struct Job { int fl, fi, fo; bool epi; };
    std::vector<Job> jobs = {{fl, fv, fv, false}, {fl, fv, fq, true}};
    if (fq != fv) jobs.push_back({fl, fv, fv, true});
    if (prec != F64 && g->links[F64][0].p) {  // FP64 kernels of the reliable updates
        jobs.push_back({F64, F64, F64, false});
        jobs.push_back({F64, F64, F64, true});
    }
    for (const Job &j : jobs)
        if ((rc = tune_dslash(g, j.fl, j.fi, j.fo, nrhs, j.epi, cache_path, s, nullptr, nullptr))) return rc;
    return HISQ_OK;
}

int hisq_dslash_shape(hisq_gauge_t g, int prec, int nrhs, int epilogue, int out[3]) {
    int rc = check_handle(g);
    if (rc) return rc;
    if (!valid_sloppy(prec) || nrhs < 1 || epilogue < 0 || epilogue > 2 || !out)
        return fail(HISQ_ERR_INVALID, "bad arguments");
    const int fl = sloppy_link_fmt(prec), fv = sloppy_vec_fmt(prec);
    const int fo = (epilogue == 2 && fv == H16) ? F32 : fv;
    const DslashShape sh = pick_shape(g, fl, fv, fo, nrhs, epilogue != 0);
    out[0] = sh.tile;
    out[1] = sh.block;
    out[2] = sh.order;
    return HISQ_OK;
}

}  // extern "C"
