// Internal declarations of the HISQ library: device types, lattice geometry,
// spinor/link storage formats and the host-side launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hisq.h"

namespace hisq {

// ------------------------------------------------------------------ types
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

template <class T>
struct cx {
    T re, im;
};

template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc += a * b
template <class T>
__device__ __forceinline__ void cmac(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}

// ------------------------------------------------------------------ geometry
// Checkerboard geometry.  A site of parity p with coordinates (x,y,z,t) has
// index h = (x >> 1) + lxh*(y + Ly*(z + Lz*t)), lxh = Lx/2.
struct Geom {
    int L[4];
    int lxh;
    int vh;
    int sy, sz, st;  // index strides of one step in y, z, t
};

Geom make_geom(const int dims[4]);

__device__ __forceinline__ int wrap(int c, int L) {
    c = c < 0 ? c + L : c;
    return c >= L ? c - L : c;
}

struct SiteCoord {
    int x, y, z, t, base;  // base = h - (x >> 1)
};

__device__ __forceinline__ SiteCoord decode_site(const Geom &g, int h, int parity) {
    SiteCoord s;
    int xh = h % g.lxh;
    int r = h / g.lxh;
    s.y = r % g.L[1];
    r /= g.L[1];
    s.z = r % g.L[2];
    s.t = r / g.L[2];
    s.x = 2 * xh + ((s.y + s.z + s.t + parity) & 1);
    s.base = h - xh;
    return s;
}

// Index of the site reached by `d` steps along mu (|d| <= 3 < L_mu).
__device__ __forceinline__ int hop_index(const Geom &g, const SiteCoord &s, int h, int mu, int d) {
    switch (mu) {
        case 0: return s.base + (wrap(s.x + d, g.L[0]) >> 1);
        case 1: return h + (wrap(s.y + d, g.L[1]) - s.y) * g.sy;
        case 2: return h + (wrap(s.z + d, g.L[2]) - s.z) * g.sz;
        default: return h + (wrap(s.t + d, g.L[3]) - s.t) * g.st;
    }
}

// Hop of link slot k = 4*mu + j: j = 0 -> +1, 1 -> -1, 2 -> +3, 3 -> -3.
__device__ __forceinline__ constexpr int slot_dist(int j) { return j == 0 ? 1 : j == 1 ? -1 : j == 2 ? 3 : -3; }

// Workgroups are dealt round-robin to the 8 XCDs; remap so each XCD walks a
// contiguous range of sites and its L2 sees the x/y/z neighbours it reuses.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
    const int per = nblocks >> 3;
    if (per == 0 || (nblocks & 7)) return bid;
    return (bid & 7) * per + (bid >> 3);
}

// ------------------------------------------------------------------ formats
enum Fmt { F64 = HISQ_PREC_FP64, F32 = HISQ_PREC_FP32, H16 = HISQ_PREC_FP16S };

template <int F> struct RealOf { typedef float T; };
template <> struct RealOf<F64> { typedef double T; };

// Spinor field of one parity in colour-major planes (public layout).
template <int F> struct Spinor;

template <> struct Spinor<F64> {
    d2v *p;
    int vh;
    // view of buffer i of a stack [n][3][vh]
    __device__ __forceinline__ Spinor rhs(int i) const { return {p + (size_t)i * 3 * vh, vh}; }
    __device__ __forceinline__ void load(int h, cx<double> v[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d2v a = p[(size_t)c * vh + h];
            v[c] = {a.x, a.y};
        }
    }
    __device__ __forceinline__ void store(int h, const cx<double> v[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) p[(size_t)c * vh + h] = d2v{v[c].re, v[c].im};
    }
};

template <> struct Spinor<F32> {
    f2v *p;
    int vh;
    __device__ __forceinline__ Spinor rhs(int i) const { return {p + (size_t)i * 3 * vh, vh}; }
    __device__ __forceinline__ void load(int h, cx<float> v[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f2v a = p[(size_t)c * vh + h];
            v[c] = {a.x, a.y};
        }
    }
    __device__ __forceinline__ void store(int h, const cx<float> v[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) p[(size_t)c * vh + h] = f2v{v[c].re, v[c].im};
    }
};

// FP16 values with one FP32 scale per site: value = scale * half.
template <> struct Spinor<H16> {
    h2v *p;      // [3][vh]
    float *s;    // [vh], right after the planes
    int vh;
    // one buffer = 16*vh bytes = 4*vh words, planes and scales move together
    __device__ __forceinline__ Spinor rhs(int i) const {
        return {p + (size_t)i * 4 * vh, s + (size_t)i * 4 * vh, vh};
    }
    __device__ __forceinline__ void load(int h, cx<float> v[3]) const {
        const float sc = s[h];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f2v a = __builtin_convertvector(p[(size_t)c * vh + h], f2v);
            v[c] = {a.x * sc, a.y * sc};
        }
    }
    __device__ __forceinline__ void store(int h, const cx<float> v[3]) const {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            p[(size_t)c * vh + h] = __builtin_convertvector((f2v{v[c].re * inv, v[c].im * inv}), h2v);
        s[h] = m;
    }
};

template <int F>
inline Spinor<F> spinor_view(void *ptr, int vh);
template <>
inline Spinor<F64> spinor_view<F64>(void *ptr, int vh) { return {(d2v *)ptr, vh}; }
template <>
inline Spinor<F32> spinor_view<F32>(void *ptr, int vh) { return {(f2v *)ptr, vh}; }
template <>
inline Spinor<H16> spinor_view<H16>(void *ptr, int vh) {
    return {(h2v *)ptr, (float *)((char *)ptr + (size_t)12 * vh), vh};
}

inline size_t spinor_bytes(int f, int64_t vh) {
    switch (f) {
        case F64: return (size_t)48 * vh;
        case F32: return (size_t)24 * vh;
        case H16: return (size_t)16 * vh;
        default: return 0;
    }
}

// Packed links for one output parity: 16 slots (k = 4 mu + j), each slot a
// block of 9 complex entries per output site, stored so that one wavefront
// reads whole contiguous planes:
//   F64: [16][9][vh] double2
//   F32: [16] { float4 [4][vh] (entries 0..7), float2 [vh] (entry 8) }
//   H16: [16] { 8-half [2][vh] (entries 0..7), half2  [vh] (entry 8) }
// Slot k of output site x already holds the factor that multiplies the
// neighbour spinor: F_mu(x), -F_mu(x-mu)^+, L_mu(x), -L_mu(x-3mu)^+.
inline size_t link_slot_bytes(int f, int64_t vh) {
    switch (f) {
        case F64: return (size_t)144 * vh;
        case F32: return (size_t)72 * vh;
        case H16: return (size_t)36 * vh;
        default: return 0;
    }
}
inline size_t link_parity_bytes(int f, int64_t vh) { return 16 * link_slot_bytes(f, vh); }

template <int F> struct Links;

template <> struct Links<F64> {
    const d2v *p;  // parity block
    int vh;
    __device__ __forceinline__ void load(int k, int h, cx<double> w[9]) const {
        const d2v *b = p + (size_t)k * 9 * vh + h;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            d2v a = __builtin_nontemporal_load(b + (size_t)e * vh);
            w[e] = {a.x, a.y};
        }
    }
};

template <> struct Links<F32> {
    const float *p;
    int vh;
    __device__ __forceinline__ void load(int k, int h, cx<float> w[9]) const {
        const float *b = p + (size_t)k * 18 * vh;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f4v a = __builtin_nontemporal_load((const f4v *)(b + (size_t)q * 4 * vh) + h);
            w[2 * q] = {a.x, a.y};
            w[2 * q + 1] = {a.z, a.w};
        }
        f2v a = __builtin_nontemporal_load((const f2v *)(b + (size_t)16 * vh) + h);
        w[8] = {a.x, a.y};
    }
};

template <> struct Links<H16> {
    const unsigned int *p;  // in 32-bit words; one word = one complex half
    int vh;
    __device__ __forceinline__ void load(int k, int h, cx<float> w[9]) const {
        const unsigned int *b = p + (size_t)k * 9 * vh;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            u4v a = __builtin_nontemporal_load((const u4v *)(b + (size_t)q * 4 * vh) + h);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                unsigned int wd = a[e];
                f2v f = __builtin_convertvector(__builtin_bit_cast(h2v, wd), f2v);
                w[4 * q + e] = {f.x, f.y};
            }
        }
        unsigned int wd = __builtin_nontemporal_load(b + (size_t)8 * vh + h);
        f2v f = __builtin_convertvector(__builtin_bit_cast(h2v, wd), f2v);
        w[8] = {f.x, f.y};
    }
};

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
const char *get_error();

#define HISQ_HIP_CHECK(expr)                                                           \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::hisq::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));      \
            return e_ == hipErrorOutOfMemory ? HISQ_ERR_OOM : HISQ_ERR_HIP;            \
        }                                                                              \
    } while (0)

// ------------------------------------------------------------------ launch wrappers
// Link packing: canonical [V][4][3][3] complex double -> packed per parity.
int launch_pack_links(const Geom &g, int fmt, const double *fat, const double *lng, void *dst_even,
                      void *dst_odd, float *maxabs_dev, hipStream_t s);

struct CgState;

// Dslash with optional epilogue out = diag_i * y_i - D in_i and per-block
// partial sums of Re<y_i, out_i> (FP64).  nrhs >= 1, tile = RHS per thread.
struct DslashLaunch {
    const void *links;  // packed block of the output parity
    const void *in;
    void *out;
    const void *y;          // epilogue input (null = plain Dslash)
    const double *diag;     // device, per RHS (null = plain Dslash)
    double *partials;       // device [nrhs][nblocks] (null = no dot)
    const CgState *skip;    // device per-RHS solver state: a tile whose RHS are all
                            // not running is skipped (null = compute all)
    int nrhs;
    int parity;
    int fmt_links, fmt_in, fmt_out;
    int tile;
    int block;
};
int launch_dslash(const Geom &g, const DslashLaunch &a, hipStream_t s);
int dslash_grid_blocks(const Geom &g, int block);

}  // namespace hisq
