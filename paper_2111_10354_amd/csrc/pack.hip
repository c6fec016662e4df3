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

template <int F>
__global__ __launch_bounds__(256) void k_pack_links(Geom g, const double *__restrict__ fat,
                                                    const double *__restrict__ lng, void *dst,
                                                    int parity, unsigned int *maxabs_bits) {
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
    store_slot<F>(dst, k, h, w);
    if (maxabs_bits) atomicMax(maxabs_bits, __float_as_uint(m));  // m >= 0: bit order = value order
}

int launch_pack_links(const Geom &g, int fmt, const double *fat, const double *lng, void *dst_even,
                      void *dst_odd, float *maxabs_dev, hipStream_t s) {
    dim3 grid((g.vh + 255) / 256, 16);
    for (int par = 0; par < 2; ++par) {
        void *dst = par ? dst_odd : dst_even;
        unsigned int *mb = (unsigned int *)maxabs_dev;
        switch (fmt) {
            case F64: hipLaunchKernelGGL(k_pack_links<F64>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb); break;
            case F32: hipLaunchKernelGGL(k_pack_links<F32>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb); break;
            case H16: hipLaunchKernelGGL(k_pack_links<H16>, grid, dim3(256), 0, s, g, fat, lng, dst, par, mb); break;
            default: return HISQ_ERR_INVALID;
        }
    }
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

}  // namespace hisq
