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
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
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

__host__ __device__ __forceinline__ int wrap(int c, int L) {
    c = c < 0 ? c + L : c;
    return c >= L ? c - L : c;
}

struct SiteCoord {
    int x, y, z, t, base;  // base = h - (x >> 1)
};

__host__ __device__ __forceinline__ SiteCoord decode_site(const Geom &g, int h, int parity) {
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
__host__ __device__ __forceinline__ int hop_index(const Geom &g, const SiteCoord &s, int h, int mu, int d) {
    switch (mu) {
        case 0: return s.base + (wrap(s.x + d, g.L[0]) >> 1);
        case 1: return h + (wrap(s.y + d, g.L[1]) - s.y) * g.sy;
        case 2: return h + (wrap(s.z + d, g.L[2]) - s.z) * g.sz;
        default: return h + (wrap(s.t + d, g.L[3]) - s.t) * g.st;
    }
}

// Hop of link slot k = 4*mu + j: j = 0 -> +1, 1 -> -1, 2 -> +3, 3 -> -3.
__host__ __device__ __forceinline__ constexpr int slot_dist(int j) { return j == 0 ? 1 : j == 1 ? -1 : j == 2 ? 3 : -3; }

// Output site of thread `tid` of workgroup `blk` (of `nb`, `bdim` threads each)
// in the processing order of the 64-site tiles (the low byte of `order`).
//
// 0: memory order (x, y, z, t).
// 1: (z, t) planes with t fastest, which brings the time-direction neighbours
//    16x closer in processing order.  Needs whole tiles per plane.
// 2: XCD bricks.  Workgroup b runs on XCD b % 8 (workgroups are dealt to the
//    eight XCDs in turn), so logical block (b % 8) * nb/8 + b/8 hands every XCD
//    one contiguous eighth of the processing order and its own L2 sees every
//    neighbour gather of that eighth.  The order walks columns of BY y-rows by
//    BZ z-planes (BY = bits 8-15 of `order`, BZ = bits 16-23), with z-block
//    slowest, then y-block, then t, then z inside the block, then the column's
//    tiles.  While a column is swept along t, all sixteen hops of the sites in
//    flight (+-1 and +-3 in every direction) fall inside a window of seven
//    t-slices of the column, which is sized to stay in one L2; only the column
//    faces are fetched twice.
// 3: memory order with workgroups of whole x-rows (block a multiple of the
//    row length Lx/2): the workgroup stages the input colour vectors of its
//    rows in LDS and the four x-direction hops read them there.
// 4: t-march (K = bits 8-15 of `order`): each thread computes K sites of one
//    (x, y, z) column, t advancing by 2 (tmarch_first_site below).
__host__ __device__ __forceinline__ int site_of_thread(const Geom &g, int blk, int nb, int bdim, int tid,
                                                       int order) {
    const int kind = order & 0xff;
    if (kind == 2) blk = (blk & 7) * (nb >> 3) + (blk >> 3);
    const int i = blk * bdim + tid;
    // grid tail: keep it out of range (the permutations below would map an
    // index past the last tile back onto a valid one)
    if (kind == 0 || kind == 3 || i >= g.vh) return i;
    const int tpp = (g.lxh * g.L[1]) >> 6;  // tiles per (z, t) plane
    int wt = i >> 6;
    if (kind == 1) {
        const int q = wt / tpp, p = wt - q * tpp;
        const int z = q / g.L[3], t = q - z * g.L[3];
        return ((t * g.L[2] + z) * tpp + p) * 64 + (i & 63);
    }
    const int by = (order >> 8) & 0xff, bz = (order >> 16) & 0xff;
    const int ty = (g.lxh * by) >> 6;  // tiles per column row block
    const int nyb = g.L[1] / by;
    const int within = wt % ty;
    wt /= ty;
    const int zz = wt % bz;
    wt /= bz;
    const int t = wt % g.L[3];
    wt /= g.L[3];
    const int yb = wt % nyb, zb = wt / nyb;
    return ((t * g.L[2] + zb * bz + zz) * tpp + yb * ty + within) * 64 + (i & 63);
}

// Order 4: thread i computes the K output sites h0, h0 + 2 st, ...,
// h0 + 2 st (K - 1) of one (x, y, z) column, h0 = the value returned (Vh for
// the grid tail).  The columns are the 2 st sites of t-slices 0 and 1;
// consecutive threads take consecutive columns of one segment of K steps,
// segment q covering t-slices 2 q K .. 2 q K + 2 K - 1.  K divides Lt / 2.
__host__ __device__ __forceinline__ int tmarch_first_site(const Geom &g, int i, int K) {
    const int cols = 2 * g.st;
    if (i >= g.vh / K) return g.vh;
    const int q = i / cols;
    return (i - q * cols) + q * K * cols;
}

// ------------------------------------------------------------------ formats
enum Fmt { F64 = HISQ_PREC_FP64, F32 = HISQ_PREC_FP32, H16 = HISQ_PREC_FP16S };

template <int F> struct RealOf { typedef float T; };
template <> struct RealOf<F64> { typedef double T; };

// Spinor field of one parity in the public layouts (include/hisq.h).
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
    // streaming store: the written field is not re-read by this kernel
    __device__ __forceinline__ void store_nt(int h, const cx<double> v[3]) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(d2v{v[c].re, v[c].im}, p + (size_t)c * vh + h);
    }
};

// FP32: plane A = colours 0,1 as float4 [vh], plane B = colour 2 as float2 [vh]
// (two loads per site instead of three).
template <> struct Spinor<F32> {
    float *p;
    int vh;
    __device__ __forceinline__ Spinor rhs(int i) const { return {p + (size_t)i * 6 * vh, vh}; }
    __device__ __forceinline__ void load(int h, cx<float> v[3]) const {
        const f4v a = ((const f4v *)p)[h];
        const f2v b = ((const f2v *)(p + (size_t)4 * vh))[h];
        v[0] = {a.x, a.y};
        v[1] = {a.z, a.w};
        v[2] = {b.x, b.y};
    }
    __device__ __forceinline__ void store(int h, const cx<float> v[3]) const {
        ((f4v *)p)[h] = f4v{v[0].re, v[0].im, v[1].re, v[1].im};
        ((f2v *)(p + (size_t)4 * vh))[h] = f2v{v[2].re, v[2].im};
    }
    __device__ __forceinline__ void store_nt(int h, const cx<float> v[3]) const {
        __builtin_nontemporal_store(f4v{v[0].re, v[0].im, v[1].re, v[1].im}, (f4v *)p + h);
        __builtin_nontemporal_store(f2v{v[2].re, v[2].im}, (f2v *)(p + (size_t)4 * vh) + h);
    }
};

// FP16S: one 16-byte record per site, {c0, c1, c2 as half2, scale as float};
// value = scale * half, scale = max |re|,|im| over the site (one load per site).
template <> struct Spinor<H16> {
    u4v *p;
    int vh;
    __device__ __forceinline__ Spinor rhs(int i) const { return {p + (size_t)i * vh, vh}; }
    __device__ __forceinline__ void load(int h, cx<float> v[3]) const {
        const u4v rec = p[h];
        const h8v a = __builtin_bit_cast(h8v, rec);
        // element to a scalar first: bit-casting rec.w directly reads element 0
        const unsigned int sw = rec.w;
        const float sc = __builtin_bit_cast(float, sw);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = {(float)a[2 * c] * sc, (float)a[2 * c + 1] * sc};
    }
    static __device__ __forceinline__ u4v encode(const cx<float> v[3]) {
        float m = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
        unsigned int wd[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            wd[c] = __builtin_bit_cast(unsigned int, __builtin_convertvector((f2v{v[c].re * inv, v[c].im * inv}), h2v));
        return u4v{wd[0], wd[1], wd[2], __builtin_bit_cast(unsigned int, m)};
    }
    __device__ __forceinline__ void store(int h, const cx<float> v[3]) const { p[h] = encode(v); }
    __device__ __forceinline__ void store_nt(int h, const cx<float> v[3]) const {
        __builtin_nontemporal_store(encode(v), p + h);
    }
};

template <int F>
inline Spinor<F> spinor_view(void *ptr, int vh);
template <>
inline Spinor<F64> spinor_view<F64>(void *ptr, int vh) { return {(d2v *)ptr, vh}; }
template <>
inline Spinor<F32> spinor_view<F32>(void *ptr, int vh) { return {(float *)ptr, vh}; }
template <>
inline Spinor<H16> spinor_view<H16>(void *ptr, int vh) { return {(u4v *)ptr, vh}; }

inline size_t spinor_bytes(int f, int64_t vh) {
    switch (f) {
        case F64: return (size_t)48 * vh;
        case F32: return (size_t)24 * vh;
        case H16: return (size_t)16 * vh;
        default: return 0;
    }
}

// Packed links for one output parity.  Slot k = 4 mu + j of output site x
// holds the matrix that multiplies the neighbour colour vector:
//   j = 0: F_mu(x), 1: -F_mu(x-mu)^+, 2: L_mu(x), 3: -L_mu(x-3mu)^+.
// Consecutive slots are grouped so that one group is 144 bytes = nine 16-byte
// units per site: a group is 1 link in FP64, 2 links in FP32, 4 links in FP16
// (the group's links' complex entries concatenated, row-major).  Sites are
// tiled by 64 (one wavefront), and a tile stores, group by group and unit by
// unit, the 64 sites' 16-byte units back to back:
//   byte offset of (site h, group gi, unit e) =
//       (((h / 64) * NG + gi) * 9 + e) * 1024 + (h % 64) * 16,   NG = 16 / G.
// One load instruction of a wavefront reads 1 KiB contiguously and the whole
// wavefront's 16 links are one contiguous stream: every link byte is read
// exactly once per Dslash, at the pattern a plain streaming read uses.
constexpr int LINK_TILE = 64;
template <int F> struct LinkGroup { static constexpr int G = 1; };
template <> struct LinkGroup<F32> { static constexpr int G = 2; };
template <> struct LinkGroup<H16> { static constexpr int G = 4; };

inline int link_group_size(int f) { return f == F64 ? 1 : f == F32 ? 2 : 4; }

// Compressed layouts (the gauge-field compression of the D-slash: only part of
// a link is stored and the rest recomputed from its unitarity).  Slots
// j = 2, 3 (long links) keep rows 0 and 1; row 2 is rebuilt in the kernel as
// kappa * conj(row 0 x row 1), which holds for every multiple M = s U of a
// unitary U (s > 0) with kappa = det(M) / s^4.  Two modes:
//   COMP_SIGN  kappa = +-1 (unitary links with determinant +-1, e.g. products
//              of SU(3) links with the staggered signs folded in), one bit
//              per slot in a 32-bit word per site after the last tile;
//   COMP_KAPPA kappa complex (any multiple of a U(3) link, e.g. the HISQ
//              Naik links -W W W / 24 of U(3)-projected W), stored per slot
//              in one extra 16-byte unit per chunk.
// The fat links (not unitary in general) stay whole.  The sites of a 64-site
// tile are stored chunk by chunk; chunk c covers MC directions
// mu = c MC .. c MC + MC - 1 and holds first the fat slots (mu, j = 0, 1 for
// each mu of the chunk, 9 complex entries each), then the long slots (mu,
// j = 2, 3, rows 0 and 1 = 6 complex entries each), entries row-major, slots
// in that order, packed into 16-byte units, and in COMP_KAPPA mode one unit of
// the chunk's 2 MC kappas (slot order):
//   byte offset of (site h, chunk c, unit e) = (((h / 64) * NC + c) * UC + e) * 1024 + (h % 64) * 16,
//   UC = UF + UL (+ 1 in COMP_KAPPA mode)
//   FP64: MC 1, NC 4, 18 fat + 12 long units;  FP32: MC 1, NC 4, 9 + 6;  FP16: MC 2, NC 2, 9 + 6.
// COMP_SIGN: after the last tile, one 32-bit word per site holds the
// determinant signs: bit 2 mu + (j - 2) set when the determinant of slot
// (mu, j) is -1.
enum CompMode { COMP_NONE = 0, COMP_SIGN = 1, COMP_KAPPA = 2 };
template <int F> struct CompGeom { static constexpr int MC = 1, NC = 4, UF = 18, UL = 12; };
template <> struct CompGeom<F32> { static constexpr int MC = 1, NC = 4, UF = 9, UL = 6; };
template <> struct CompGeom<H16> { static constexpr int MC = 2, NC = 2, UF = 9, UL = 6; };
// 16-byte units per chunk and per site (per 64-site tile, in units of 1 KiB)
template <int F>
__host__ __device__ constexpr int comp_chunk_units(int mode) {
    return CompGeom<F>::UF + CompGeom<F>::UL + (mode == COMP_KAPPA ? 1 : 0);
}
template <int F>
__host__ __device__ constexpr int comp_units(int mode = COMP_SIGN) {
    return CompGeom<F>::NC * comp_chunk_units<F>(mode);
}
__host__ __device__ inline int comp_units_per_site(int f, int mode = COMP_SIGN) {
    return f == F64 ? comp_units<F64>(mode) : f == F32 ? comp_units<F32>(mode) : comp_units<H16>(mode);
}
static_assert(comp_units<F64>() == 120 && comp_units<F32>() == 60 && comp_units<H16>() == 30,
              "compressed layouts: 15 or 30 units per direction chunk");
static_assert(comp_units<F32>(COMP_KAPPA) == 64 && comp_units<H16>(COMP_KAPPA) == 32,
              "kappa layouts: one extra unit per chunk");

inline size_t link_parity_bytes(int f, int64_t vh, int mode = COMP_NONE) {
    const int64_t tiles = (vh + LINK_TILE - 1) / LINK_TILE;
    if (mode == COMP_SIGN) return (size_t)tiles * (comp_units_per_site(f, mode) * 1024 + LINK_TILE * 4);
    if (mode == COMP_KAPPA) return (size_t)tiles * comp_units_per_site(f, mode) * 1024;
    return (size_t)tiles * (16 / link_group_size(f)) * 9 * 1024;
}

__host__ __device__ __forceinline__ const u4v *link_unit_ptr(const void *base, int ng, int gi, int h) {
    return (const u4v *)base + ((size_t)((h >> 6) * ng + gi) * 9) * 64 + (h & 63);
}

// Link loads: non-temporal (streamed past the caches) when each link byte is
// read once per launch; cached when several waves of a workgroup read the same
// links (the RHS of a site split over waves).
template <bool NT, class T>
__device__ __forceinline__ T ldlink(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <int F, bool NT = true> struct Links;

template <bool NT> struct Links<F64, NT> {
    const void *p;
    // the G*9 = 9 complex entries of group gi (= slot gi)
    __device__ __forceinline__ void load_group(int gi, int h, cx<double> w[9]) const {
        const u4v *b = link_unit_ptr(p, 16, gi, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            d2v a = __builtin_bit_cast(d2v, ldlink<NT>(b + e * 64));
            w[e] = {a.x, a.y};
        }
    }
};

template <bool NT> struct Links<F32, NT> {
    const void *p;
    // 18 complex entries: slots 2 gi and 2 gi + 1
    __device__ __forceinline__ void load_group(int gi, int h, cx<float> w[18]) const {
        const u4v *b = link_unit_ptr(p, 8, gi, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            f4v a = __builtin_bit_cast(f4v, ldlink<NT>(b + e * 64));
            w[2 * e] = {a.x, a.y};
            w[2 * e + 1] = {a.z, a.w};
        }
    }
};

template <bool NT> struct Links<H16, NT> {
    const void *p;
    // 36 complex entries: slots 4 gi .. 4 gi + 3
    __device__ __forceinline__ void load_group(int gi, int h, cx<float> w[36]) const {
        const u4v *b = link_unit_ptr(p, 4, gi, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            // reinterpret all 16 bytes at once: bit-casting a single element
            // of the loaded vector (a[q]) was compiled as if q were 0
            const h8v a = __builtin_bit_cast(h8v, ldlink<NT>(b + e * 64));
#pragma unroll
            for (int q = 0; q < 4; ++q) w[4 * e + q] = {(float)a[2 * q], (float)a[2 * q + 1]};
        }
    }
};

// Loaders of the compressed layouts: fat part (2 MC slots, 9 entries each),
// long part (2 MC slots, rows 0 and 1 = 6 entries each) and, in COMP_KAPPA
// mode, the 2 MC kappas of chunk c.
template <int F, int CM, bool NT = true> struct LinksC;

template <int F, int CM>
__host__ __device__ __forceinline__ const u4v *comp_unit_ptr(const void *base, int c, int h) {
    constexpr int NC = CompGeom<F>::NC, UC = comp_chunk_units<F>(CM);
    return (const u4v *)base + ((size_t)((h >> 6) * NC + c) * UC) * 64 + (h & 63);
}

template <int F>
__device__ __forceinline__ unsigned comp_signs(const void *base, int vh, int h) {
    const size_t tiles = (size_t)(vh + LINK_TILE - 1) / LINK_TILE;
    const unsigned *sg = (const unsigned *)((const char *)base + tiles * comp_units_per_site(F, COMP_SIGN) * 1024);
    return __builtin_nontemporal_load(sg + h);
}

template <int CM, bool NT> struct LinksC<F64, CM, NT> {
    const void *p;
    int vh;
    __device__ __forceinline__ unsigned signs(int h) const { return comp_signs<F64>(p, vh, h); }
    __device__ __forceinline__ void load_fat(int c, int h, cx<double> w[18]) const {
        const u4v *b = comp_unit_ptr<F64, CM>(p, c, h);
#pragma unroll
        for (int e = 0; e < 18; ++e) {
            d2v a = __builtin_bit_cast(d2v, ldlink<NT>(b + e * 64));
            w[e] = {a.x, a.y};
        }
    }
    __device__ __forceinline__ void load_long(int c, int h, cx<double> r[12]) const {
        const u4v *b = comp_unit_ptr<F64, CM>(p, c, h) + 18 * 64;
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            d2v a = __builtin_bit_cast(d2v, ldlink<NT>(b + e * 64));
            r[e] = {a.x, a.y};
        }
    }
};

template <int CM, bool NT> struct LinksC<F32, CM, NT> {
    const void *p;
    int vh;
    __device__ __forceinline__ unsigned signs(int h) const { return comp_signs<F32>(p, vh, h); }
    __device__ __forceinline__ void load_fat(int c, int h, cx<float> w[18]) const {
        const u4v *b = comp_unit_ptr<F32, CM>(p, c, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            f4v a = __builtin_bit_cast(f4v, ldlink<NT>(b + e * 64));
            w[2 * e] = {a.x, a.y};
            w[2 * e + 1] = {a.z, a.w};
        }
    }
    __device__ __forceinline__ void load_long(int c, int h, cx<float> r[12]) const {
        const u4v *b = comp_unit_ptr<F32, CM>(p, c, h) + 9 * 64;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            f4v a = __builtin_bit_cast(f4v, ldlink<NT>(b + e * 64));
            r[2 * e] = {a.x, a.y};
            r[2 * e + 1] = {a.z, a.w};
        }
    }
    __device__ __forceinline__ void load_kappa(int c, int h, cx<float> k[2]) const {
        const f4v a = __builtin_bit_cast(f4v, ldlink<NT>(comp_unit_ptr<F32, CM>(p, c, h) + 15 * 64));
        k[0] = {a.x, a.y};
        k[1] = {a.z, a.w};
    }
};

template <int CM, bool NT> struct LinksC<H16, CM, NT> {
    const void *p;
    int vh;
    __device__ __forceinline__ unsigned signs(int h) const { return comp_signs<H16>(p, vh, h); }
    __device__ __forceinline__ void load_fat(int c, int h, cx<float> w[36]) const {
        const u4v *b = comp_unit_ptr<H16, CM>(p, c, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const h8v a = __builtin_bit_cast(h8v, ldlink<NT>(b + e * 64));
#pragma unroll
            for (int q = 0; q < 4; ++q) w[4 * e + q] = {(float)a[2 * q], (float)a[2 * q + 1]};
        }
    }
    __device__ __forceinline__ void load_long(int c, int h, cx<float> r[24]) const {
        const u4v *b = comp_unit_ptr<H16, CM>(p, c, h) + 9 * 64;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const h8v a = __builtin_bit_cast(h8v, ldlink<NT>(b + e * 64));
#pragma unroll
            for (int q = 0; q < 4; ++q) r[4 * e + q] = {(float)a[2 * q], (float)a[2 * q + 1]};
        }
    }
    __device__ __forceinline__ void load_kappa(int c, int h, cx<float> k[4]) const {
        const h8v a = __builtin_bit_cast(h8v, ldlink<NT>(comp_unit_ptr<H16, CM>(p, c, h) + 15 * 64));
#pragma unroll
        for (int q = 0; q < 4; ++q) k[q] = {(float)a[2 * q], (float)a[2 * q + 1]};
    }
};

// Row 2 of a multiple of a unitary matrix from rows 0 and 1:
// m[6..8] = kappa * conj(row0 x row1) with kappa = +-1 (real d) or complex.
template <class R>
__device__ __forceinline__ void rebuild_row2(cx<R> m[9], R d) {
    const cx<R> *a = m, *b = m + 3;
    const cx<R> c0 = cmul(a[1], b[2]), c1 = cmul(a[2], b[1]);
    const cx<R> c2 = cmul(a[2], b[0]), c3 = cmul(a[0], b[2]);
    const cx<R> c4 = cmul(a[0], b[1]), c5 = cmul(a[1], b[0]);
    m[6] = {d * (c0.re - c1.re), -d * (c0.im - c1.im)};
    m[7] = {d * (c2.re - c3.re), -d * (c2.im - c3.im)};
    m[8] = {d * (c4.re - c5.re), -d * (c4.im - c5.im)};
}
template <class R>
__device__ __forceinline__ void rebuild_row2(cx<R> m[9], cx<R> k) {
    const cx<R> *a = m, *b = m + 3;
    const cx<R> c0 = cmul(a[1], b[2]), c1 = cmul(a[2], b[1]);
    const cx<R> c2 = cmul(a[2], b[0]), c3 = cmul(a[0], b[2]);
    const cx<R> c4 = cmul(a[0], b[1]), c5 = cmul(a[1], b[0]);
    m[6] = cmul(k, cx<R>{c0.re - c1.re, c1.im - c0.im});
    m[7] = cmul(k, cx<R>{c2.re - c3.re, c3.im - c2.im});
    m[8] = cmul(k, cx<R>{c4.re - c5.re, c5.im - c4.im});
}

// ------------------------------------------------------------------ tracing
// roctx range over a scope: solver phases show up in `rocprofv3 --marker-trace`
// (no-ops when no profiler is attached).
struct TraceRange {
    explicit TraceRange(const char *name);
    ~TraceRange();
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
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
                      void *dst_odd, float *maxabs_dev, int comp_mode, hipStream_t s);
// Largest deviation of any long link from a unitary matrix with determinant
// +-1 (max |L L^+ - 1| entry or | det - round(det) |) into defect_bits[0], and
// from a positive multiple s U of a unitary U (max |L L^+ - s^2| entry / s^2,
// s^2 = tr(L L^+) / 3) into defect_bits[1], as float bits (atomic max; zero
// both first).
void launch_long_link_defect(const Geom &g, const double *lng, unsigned *defect_bits, hipStream_t s);

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
    int order;  // tile processing order: 0 memory order, 1 t-fastest planes,
                // 2 | BY << 8 | BZ << 16 XCD bricks (dslash.hip); bits 24-25:
                // log2 of the waves a site's RHS tiles are split over
    int compressed;  // links in a compressed layout (CompMode)
};
int launch_dslash(const Geom &g, const DslashLaunch &a, hipStream_t s);
bool order_supported(const Geom &g, int order, int block);
// Workgroups along the sites of a launch with `block` threads and tile order
// `order` (bits 24-25: the RHS split over waves).
int dslash_grid_blocks(const Geom &g, int block, int order);

}  // namespace hisq
