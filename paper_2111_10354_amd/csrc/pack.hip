// Packing of the caller's canonical links into the Dslash layout.
//
// For output parity p and output site h the 16 slots k = 4 mu + j hold the
// matrix that multiplies the neighbour colour vector:
//   j = 0: F_mu(x)            (neighbour x + mu)
//   j = 1: -F_mu(x - mu)^+    (neighbour x - mu)
//   j = 2: L_mu(x)            (neighbour x + 3 mu)
//   j = 3: -L_mu(x - 3 mu)^+  (neighbour x - 3 mu)
// so the kernel is a plain 16-term gather/mat-vec sum.  Every link therefore
// appears twice in memory (once per parity it serves), which trades HBM
// capacity for fully contiguous per-site reads.

#include "solver_internal.h"

namespace hisq {

__device__ __forceinline__ int64_t lex_of(const Geom &g, int x, int y, int z, int t) {
    return x + (int64_t)g.L[0] * (y + (int64_t)g.L[1] * (z + (int64_t)g.L[2] * t));
}

// Write the 9 complex entries of slot k of site h into the tiled group layout.
template <int F>
__device__ void store_slot(void *dst, int k, int h, const cx<double> w[9]) {
    constexpr int G = LinkGroup<F>::G;
    constexpr int NG = 16 / G;
    constexpr int CSIZE = 144 / (9 * G);  // bytes per complex entry: 16, 8, 4
    const int gi = k / G, sl = k % G;
    char *rec = (char *)dst + ((size_t)((h >> 6) * NG + gi) * 9) * 1024 + (size_t)(h & 63) * 16;
    for (int c = 0; c < 9; ++c) {
        const int off = (sl * 9 + c) * CSIZE;
        char *q = rec + (size_t)(off >> 4) * 1024 + (off & 15);
        if constexpr (F == F64) {
            *(d2v *)q = d2v{w[c].re, w[c].im};
        } else if constexpr (F == F32) {
            *(f2v *)q = f2v{(float)w[c].re, (float)w[c].im};
        } else {
            // double -> float -> half, round to nearest even at each step
            *(h2v *)q = __builtin_convertvector((f2v{(float)w[c].re, (float)w[c].im}), h2v);
        }
    }
}

// Compressed layouts: fat slots whole, long slots as rows 0 and 1 plus the
// determinant sign bit (COMP_SIGN) or the complex factor kappa = det / s^4,
// s^2 = tr(M M^+) / 3 (COMP_KAPPA), see CompGeom.
__device__ inline cx<double> det3(const cx<double> w[9]) {
    const cx<double> a = cmul(w[4], w[8]), b = cmul(w[5], w[7]);
    const cx<double> c2 = cmul(w[3], w[8]), d2 = cmul(w[5], w[6]);
    const cx<double> e2 = cmul(w[3], w[7]), f2 = cmul(w[4], w[6]);
    const cx<double> t0 = cmul(w[0], {a.re - b.re, a.im - b.im}), t1 = cmul(w[1], {c2.re - d2.re, c2.im - d2.im}),
                     t2 = cmul(w[2], {e2.re - f2.re, e2.im - f2.im});
    return {t0.re - t1.re + t2.re, t0.im - t1.im + t2.im};
}

template <int F>
__device__ void store_entry(char *q, cx<double> v) {
    if constexpr (F == F64) {
        *(d2v *)q = d2v{v.re, v.im};
    } else if constexpr (F == F32) {
        *(f2v *)q = f2v{(float)v.re, (float)v.im};
    } else {
        *(h2v *)q = __builtin_convertvector((f2v{(float)v.re, (float)v.im}), h2v);
    }
}

template <int F>
__device__ void store_slot_comp(void *dst, int vh, int k, int h, const cx<double> w[9], int mode) {
    constexpr int MC = CompGeom<F>::MC, NC = CompGeom<F>::NC, UF = CompGeom<F>::UF, UL = CompGeom<F>::UL;
    constexpr int CSIZE = F == F64 ? 16 : F == F32 ? 8 : 4;  // bytes per complex entry
    const int UC = comp_chunk_units<F>(mode);
    const int mu = k >> 2, j = k & 3, c = mu / MC, sm = mu % MC;
    char *rec = (char *)dst + ((size_t)((h >> 6) * NC + c) * UC) * 1024 + (size_t)(h & 63) * 16;
    const int n = j < 2 ? 9 : 6;
    const int first = j < 2 ? (2 * sm + j) * 9 * CSIZE : UF * 16 + (2 * sm + j - 2) * 6 * CSIZE;
    for (int e = 0; e < n; ++e) {
        const int off = first + e * CSIZE;
        store_entry<F>(rec + (size_t)(off >> 4) * 1024 + (off & 15), w[e]);
    }
    if (j < 2) return;
    const cx<double> det = det3(w);
    if (mode == COMP_KAPPA) {
        double s2 = 0.0;
        for (int e = 0; e < 9; ++e) s2 += w[e].re * w[e].re + w[e].im * w[e].im;
        s2 /= 3.0;
        const double inv = 1.0 / (s2 * s2);
        const int off = (UF + UL) * 16 + (2 * sm + j - 2) * CSIZE;
        store_entry<F>(rec + (size_t)(off >> 4) * 1024 + (off & 15), cx<double>{det.re * inv, det.im * inv});
    } else if (det.re < 0.0) {  // determinant +-1
        const size_t tiles = (size_t)(vh + LINK_TILE - 1) / LINK_TILE;
        unsigned *sg = (unsigned *)((char *)dst + tiles * comp_units_per_site(F, COMP_SIGN) * 1024);
        atomicOr(sg + h, 1u << (2 * mu + j - 2));
    }
}

template <int F>
__global__ __launch_bounds__(256) void k_pack_links(Geom g, const double *__restrict__ fat,
                                                    const double *__restrict__ lng, void *dst,
                                                    int parity, unsigned int *maxabs_bits, int comp_mode) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (h >= g.vh) return;
    const int mu = k >> 2, j = k & 3;
    const SiteCoord s = decode_site(g, h, parity);
    int c[4] = {s.x, s.y, s.z, s.t};
    const int d = (j == 1) ? -1 : (j == 3) ? -3 : 0;  // link sits at x + d mu
    c[mu] = wrap(c[mu] + d, g.L[mu]);
    const int64_t src = lex_of(g, c[0], c[1], c[2], c[3]);
    const double *U = ((j < 2) ? fat : lng) + (size_t)(src * 4 + mu) * 18;
    cx<double> w[9];
    float m = 0.f;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            if (j & 1) {  // -U^+ : entry (a,b) = -conj(U(b,a))
                w[3 * a + b] = {-U[(3 * b + a) * 2], U[(3 * b + a) * 2 + 1]};
            } else {
                w[3 * a + b] = {U[(3 * a + b) * 2], U[(3 * a + b) * 2 + 1]};
            }
            m = fmaxf(m, fmaxf(fabsf((float)w[3 * a + b].re), fabsf((float)w[3 * a + b].im)));
        }
    if (comp_mode != COMP_NONE) store_slot_comp<F>(dst, g.vh, k, h, w, comp_mode);
    else store_slot<F>(dst, k, h, w);
    if (maxabs_bits) atomicMax(maxabs_bits, __float_as_uint(m));  // m >= 0: bit order = value order
}

// Deviation of each long link L from a unitary matrix with determinant +-1
// (bits[0]) and from a positive multiple of a unitary matrix (bits[1]).
__global__ __launch_bounds__(256) void k_long_defect(int64_t V, const double *__restrict__ lng, unsigned *bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (site, mu)
    if (i >= 4 * V) return;
    const double *U = lng + (size_t)i * 18;
    cx<double> m[9];
    for (int e = 0; e < 9; ++e) m[e] = {U[2 * e], U[2 * e + 1]};
    double ll[9][2];
    double s2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {  // (L L^+)_ab
            double re = 0.0, im = 0.0;
            for (int c = 0; c < 3; ++c) {
                const cx<double> x = m[3 * a + c], y = m[3 * b + c];
                re += x.re * y.re + x.im * y.im;
                im += x.im * y.re - x.re * y.im;
            }
            ll[3 * a + b][0] = re;
            ll[3 * a + b][1] = im;
            if (a == b) s2 += re;
        }
    s2 /= 3.0;
    double dev1 = 0.0, dev2 = 0.0;
    for (int e = 0; e < 9; ++e) {
        const double d = (e % 4 == 0) ? 1.0 : 0.0;
        dev1 = fmax(dev1, fmax(fabs(ll[e][0] - d), fabs(ll[e][1])));
        dev2 = fmax(dev2, fmax(fabs(ll[e][0] - d * s2), fabs(ll[e][1])));
    }
    dev2 = s2 > 0.0 ? dev2 / s2 : 1e30;
    const cx<double> det = det3(m);
    dev1 = fmax(dev1, fmax(fabs(fabs(det.re) - 1.0), fabs(det.im)));
    if (!(dev1 == dev1)) dev1 = 1e30;  // NaN: not compressible
    if (!(dev2 == dev2)) dev2 = 1e30;
    atomicMax(bits, __float_as_uint((float)fmin(dev1, 1e30)));
    atomicMax(bits + 1, __float_as_uint((float)fmin(dev2, 1e30)));
}

void launch_long_link_defect(const Geom &g, const double *lng, unsigned *defect_bits, hipStream_t s) {
    const int64_t V = 2 * (int64_t)g.vh;
    hipLaunchKernelGGL(k_long_defect, dim3((unsigned)((4 * V + 255) / 256)), dim3(256), 0, s, V, lng, defect_bits);
}

int launch_pack_links(const Geom &g, int fmt, const double *fat, const double *lng, void *dst_even,
                      void *dst_odd, float *maxabs_dev, int comp_mode, hipStream_t s) {
    dim3 grid((g.vh + 255) / 256, 16);
    for (int par = 0; par < 2; ++par) {
        void *dst = par ? dst_odd : dst_even;
        if (comp_mode == COMP_SIGN) {  // determinant sign words start at zero
            const size_t tiles = (size_t)(g.vh + LINK_TILE - 1) / LINK_TILE;
            HISQ_HIP_CHECK(hipMemsetAsync((char *)dst + tiles * comp_units_per_site(fmt, COMP_SIGN) * 1024, 0,
                                          tiles * LINK_TILE * 4, s));
        }
        unsigned int *mb = (unsigned int *)maxabs_dev;
        switch (fmt) {
            case F64:
                hipLaunchKernelGGL(k_pack_links<F64>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb, comp_mode);
                break;
            case F32:
                hipLaunchKernelGGL(k_pack_links<F32>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb, comp_mode);
                break;
            case H16:
                hipLaunchKernelGGL(k_pack_links<H16>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb, comp_mode);
                break;
            default: return HISQ_ERR_INVALID;
        }
    }
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
