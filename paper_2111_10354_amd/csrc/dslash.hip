// HISQ single-parity Dslash for gfx950, single- and multi-RHS.
//
// One thread owns one output site h and a tile of TILE right-hand sides.  For
// each of the 16 link slots it streams the 9 complex entries of the slot's
// link once (non-temporal: each link is read exactly once per application and
// must not evict the spinors that neighbouring sites still reuse), gathers the
// neighbour colour vector of every RHS in the tile and accumulates the 3x3
// complex mat-vec.  All 16 slots are laid out per output site, so every link
// load of a wavefront is one contiguous plane segment; the neighbour gathers
// of a wavefront touch a contiguous run of sites shifted by the hop.
//
// Epilogue (optional): out_i = diag_i * y_i - (D in)_i and, if a partials
// buffer is given, a per-block FP64 partial of Re <y_i, out_i>, which is what
// CG needs for <p, A p>.
//
// The stencil is a 3x3 complex mat-vec per hop: 1146 flop per site against
// 1200 bytes (FP32), far below the ridge point, so it is written for memory
// throughput on the vector ALUs; matrix cores would gain nothing here.

#include <type_traits>

#include "solver_internal.h"

namespace hisq {

Geom make_geom(const int dims[4]) {
    Geom g;
    for (int i = 0; i < 4; ++i) g.L[i] = dims[i];
    g.lxh = dims[0] / 2;
    g.vh = (int)((int64_t)dims[0] * dims[1] * dims[2] * dims[3] / 2);
    g.sy = g.lxh;
    g.sz = g.lxh * dims[1];
    g.st = g.lxh * dims[1] * dims[2];
    return g;
}

// Bits 24-25 of a launch's `order`: log2 of the number of waves a site's RHS
// tiles are split over (RS = 1, 2, 4).  A workgroup of `block` threads then
// covers block / RS sites, and its RS waves of the same sites apply one RHS
// tile each: they read the same link units (the later ones from the caches),
// so each thread holds the accumulators and gathers of one tile only.
static inline int order_rsplit(int order) { return 1 << ((order >> 24) & 3); }
static inline int order_tiles(int order) { return order & 0xffffff; }

int dslash_grid_blocks(const Geom &g, int block, int order) {
    const int sb = block / order_rsplit(order);
    const int k = (order_tiles(order) & 0xff) == 4 ? (order >> 8) & 0xff : 1;  // t-march: K sites per thread
    const int threads = k > 0 ? g.vh / k : g.vh;
    return (threads + sb - 1) / sb;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Kernel variants (MODE; each a template instance of its own, so that the
// others keep their branch-free hop loops):
//  MODE_PLAIN:  one output site per thread, every hop gathered through the
//               caches;
//  MODE_XROW:   traversal order 3 (RS = 1): the workgroup's sites are whole
//               x-rows in memory order; it stages the input colour vectors of
//               those rows (its RHS tile) in LDS, and the four x-direction
//               hops of every site read LDS;
//  MODE_TMARCH: traversal order 4: each thread computes K output sites of one
//               (x, y, z) column, t advancing by 2, and keeps the input
//               vectors at t - 3, t - 1, t + 1 and t + 3 of its RHS tile in
//               registers.  Three of the four t-direction hops of the next
//               site are hops of the current one, so one t-hop is gathered
//               per site instead of four, and the t-hop reuse no longer needs
//               the caches to hold seven t-slices of input.
enum { MODE_PLAIN = 0, MODE_XROW = 1, MODE_TMARCH = 2 };

template <int LF, int SI, int SO, int TILE, bool EPI, int CM, int RS, int MODE = MODE_PLAIN>
__global__ __launch_bounds__(256) void dslash_kernel(Geom g, const void *__restrict__ lptr, Spinor<SI> in,
                                                     Spinor<SO> out, Spinor<SI> y,
                                                     const double *__restrict__ diag,
                                                     double *__restrict__ partials,
                                                     const CgState *__restrict__ skip, int parity,
                                                     int nrhs, int order) {
    typedef typename RealOf<LF>::T R;
    constexpr int G = LinkGroup<LF>::G;
    constexpr bool NT = RS == 1;  // links read once per launch: stream them
    const int nb = gridDim.x;
    const int blk = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rsub = wave % RS;  // this wave's RHS tile among the RS sharing its sites
    const int sb = (int)blockDim.x / RS, tloc = (wave / RS) * 64 + lane;
    const int ksteps = MODE == MODE_TMARCH ? (order >> 8) & 0xff : 1;
    const int h0 = MODE == MODE_TMARCH ? tmarch_first_site(g, blk * sb + tloc, ksteps)
                                       : site_of_thread(g, blk, nb, sb, tloc, order & 0xffffff);
    const int rb = blockIdx.y * RS * TILE;  // first RHS of the workgroup
    const int r0 = rb + rsub * TILE;
    if (skip) {
        bool idle = true;
        for (int r = rb; r < rb + RS * TILE && r < nrhs; ++r)
            if (skip[r].flag == CG_RUNNING) idle = false;
        if (idle) return;  // uniform over the block
    }
    // RHS r of the tile; a ragged last tile repeats its last RHS (those results
    // are never stored): no branch, so the compiler can issue the gathers of
    // every RHS of the tile before the first one returns
    auto rhs_of = [&](int r) { return (TILE > 1 && r0 + r >= nrhs) ? nrhs - 1 : r0 + r; };

    // x-row staging: thread t loads the input vectors of site base + t (the
    // same row index in the input parity), for every RHS of its tile
    extern __shared__ unsigned char xr_lds[];
    cx<R> *xs = reinterpret_cast<cx<R> *>(xr_lds);  // [TILE][3][blockDim.x]
    const int xbase = blk * (int)blockDim.x;
    if constexpr (MODE == MODE_XROW) {
        static_assert(RS == 1, "x-row staging needs one wave per site");
        if (h0 < g.vh) {
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                cx<R> v[3];
                in.rhs(rhs_of(r)).load(h0, v);
#pragma unroll
                for (int c = 0; c < 3; ++c) xs[(r * 3 + c) * (int)blockDim.x + threadIdx.x] = v[c];
            }
        }
        __syncthreads();
    }

    double part[TILE];
#pragma unroll
    for (int r = 0; r < TILE; ++r) part[r] = 0.0;

    // t-march window: input vectors at t - 3, t - 1, t + 1, t + 3 of the site
    cx<R> tw[MODE == MODE_TMARCH ? 4 : 1][TILE][3];
    auto load_in = [&](int nbh, cx<R> (*dst)[3]) {
#pragma unroll
        for (int r = 0; r < TILE; ++r) in.rhs(rhs_of(r)).load(nbh, dst[r]);
    };

    // the whole stencil of output site h (decoded as sc)
    auto site = [&](const int h, const SiteCoord &sc) {
        cx<R> acc[TILE][3];
#pragma unroll
        for (int r = 0; r < TILE; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] = {R(0), R(0)};

        auto mac = [&](int r, const cx<R> *m, const cx<R> *v) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) cmac(acc[r][a], m[3 * a + b], v[b]);
        };
        // acc += m * (neighbour of slot k), for every RHS of the tile
        auto apply = [&](int k, const cx<R> *m) {
            const int nbh = hop_index(g, sc, h, k >> 2, slot_dist(k & 3));
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                cx<R> v[3];
                in.rhs(rhs_of(r)).load(nbh, v);
                mac(r, m, v);
            }
        };
        // x-direction slot (k < 4) from the staged rows
        auto apply_x = [&](int k, const cx<R> *m) {
            const int li = hop_index(g, sc, h, 0, slot_dist(k & 3)) - xbase;
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                cx<R> v[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) v[b] = xs[(r * 3 + b) * (int)blockDim.x + li];
                mac(r, m, v);
            }
        };
        // t-direction slot (k >= 12) from the window: slots +1, -1, +3, -3
        auto apply_t = [&](int k, const cx<R> *m) {
            const int wi = (k & 3) == 0 ? 2 : (k & 3) == 1 ? 1 : (k & 3) == 2 ? 3 : 0;
#pragma unroll
            for (int r = 0; r < TILE; ++r) mac(r, m, tw[MODE == MODE_TMARCH ? wi : 0][r]);
        };
        // slot k through the path its variant takes (F: 1 = the x-slots of
        // this call are staged, 2 = its t-slots are in the window)
        auto slot = [&](int k, const cx<R> *m, auto fl) {
            constexpr int F = decltype(fl)::value;
            if constexpr (F == 1) {
                if ((k >> 2) == 0) return apply_x(k, m);  // k is unrolled: folded
            }
            if constexpr (F == 2) {
                if ((k >> 2) == 3) return apply_t(k, m);
            }
            apply(k, m);
        };
        using Plain = std::integral_constant<int, 0>;
        using XSlots = std::integral_constant<int, MODE == MODE_XROW ? 1 : 0>;
        using TSlots = std::integral_constant<int, MODE == MODE_TMARCH ? 2 : 0>;
        // One RHS: every slot unrolled, the compiler interleaves the loads of
        // neighbouring slots.  Several RHS: one link group (or compressed
        // chunk) per loop trip with the gathers of all its RHS in flight
        // together; unrolled, the compiler hoists every gather of the site and
        // spills them to scratch.  The groups (chunks) holding x- or t-slots
        // of the staged / windowed variants are peeled off the loop.
        if constexpr (CM == COMP_NONE) {
            const Links<LF, NT> links{lptr};
            auto group = [&](int gi, auto fl) {
                cx<R> w[9 * G];
                links.load_group(gi, h, w);
#pragma unroll
                for (int sl = 0; sl < G; ++sl) slot(gi * G + sl, w + 9 * sl, fl);
            };
            constexpr int NG = 16 / G;
            constexpr int GX = MODE == MODE_XROW ? 4 / G : 0;     // leading groups of x-slots
            constexpr int GT = MODE == MODE_TMARCH ? 4 / G : 0;   // trailing groups of t-slots
#pragma unroll
            for (int gi = 0; gi < GX; ++gi) group(gi, XSlots{});
            if constexpr (TILE == 1) {
#pragma unroll
                for (int gi = GX; gi < NG - GT; ++gi) group(gi, Plain{});
            } else {
#pragma unroll 1
                for (int gi = GX; gi < NG - GT; ++gi) group(gi, Plain{});
            }
#pragma unroll
            for (int gi = NG - GT; gi < NG; ++gi) group(gi, TSlots{});
        } else {
            // fat slots whole; long slots from rows 0, 1 and the determinant
            // sign (COMP_SIGN) or the complex factor kappa (COMP_KAPPA)
            constexpr int MC = CompGeom<LF>::MC, NC = CompGeom<LF>::NC;
            const LinksC<LF, CM, NT> cl{lptr, g.vh};
            unsigned sg = 0;
            if constexpr (CM == COMP_SIGN) sg = cl.signs(h);
            auto chunk = [&](int c, auto fl) {
                {
                    cx<R> w[18 * MC];
                    cl.load_fat(c, h, w);
#pragma unroll
                    for (int s2 = 0; s2 < 2 * MC; ++s2) slot(4 * (c * MC + (s2 >> 1)) + (s2 & 1), w + 9 * s2, fl);
                }
                {
                    cx<R> lr[12 * MC];
                    cl.load_long(c, h, lr);
                    cx<R> kap[2 * MC];
                    if constexpr (CM == COMP_KAPPA) cl.load_kappa(c, h, kap);
#pragma unroll
                    for (int s2 = 0; s2 < 2 * MC; ++s2) {
                        const int mu = c * MC + (s2 >> 1), bit = 2 * mu + (s2 & 1);
                        cx<R> m[9];
#pragma unroll
                        for (int e = 0; e < 6; ++e) m[e] = lr[6 * s2 + e];
                        if constexpr (CM == COMP_KAPPA) rebuild_row2(m, kap[s2]);
                        else rebuild_row2(m, ((sg >> bit) & 1u) ? R(-1) : R(1));
                        slot(4 * mu + 2 + (s2 & 1), m, fl);
                    }
                }
            };
            // (a chunk's fat and long slots in separate loop trips halve the
            // registers but measured 5-10 % slower: fewer gathers in flight)
            constexpr int CX = MODE == MODE_XROW ? 1 : 0;    // chunk 0 holds the x-slots
            constexpr int CT = MODE == MODE_TMARCH ? 1 : 0;  // the last chunk, the t-slots
            if constexpr (CX) chunk(0, XSlots{});
            if constexpr (TILE == 1) {
#pragma unroll
                for (int c = CX; c < NC - CT; ++c) chunk(c, Plain{});
            } else {
#pragma unroll 1
                for (int c = CX; c < NC - CT; ++c) chunk(c, Plain{});
            }
            if constexpr (CT) chunk(NC - 1, TSlots{});
        }

#pragma unroll
        for (int r = 0; r < TILE; ++r) {
            if (TILE > 1 && r0 + r >= nrhs) break;
            cx<R> o[3];
            if constexpr (EPI) {
                const Spinor<SI> ys = y.rhs(r0 + r);
                cx<R> yv[3];
                ys.load(h, yv);
                const R d = (R)diag[r0 + r];
                double pr = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    o[c] = {d * yv[c].re - acc[r][c].re, d * yv[c].im - acc[r][c].im};
                    pr += (double)yv[c].re * (double)o[c].re + (double)yv[c].im * (double)o[c].im;
                }
                part[r] += pr;
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) o[c] = acc[r][c];
            }
            const Spinor<SO> dst = out.rhs(r0 + r);
            typedef typename RealOf<SO>::T RO;
            cx<RO> oo[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) oo[c] = {(RO)o[c].re, (RO)o[c].im};
            // streaming store: interleaving ordinary write-backs with the link
            // stream costs far more HBM time than the 2% of bytes they carry
            dst.store_nt(h, oo);
        }
    };

    if (h0 < g.vh && r0 < nrhs) {
        if constexpr (MODE == MODE_TMARCH) {
            // sites h0, h0 + 2 st, ...: t advances by 2, the window by one hop
            for (int s = 0; s < ksteps; ++s) {
                const int h = h0 + s * 2 * g.st;
                const SiteCoord sc = decode_site(g, h, parity);
                if (s == 0) {
                    load_in(hop_index(g, sc, h, 3, -3), tw[0]);
                    load_in(hop_index(g, sc, h, 3, -1), tw[1]);
                    load_in(hop_index(g, sc, h, 3, 1), tw[2]);
                } else {
#pragma unroll
                    for (int r = 0; r < TILE; ++r)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            tw[0][r][c] = tw[1][r][c];
                            tw[1][r][c] = tw[2][r][c];
                            tw[2][r][c] = tw[3][r][c];
                        }
                }
                load_in(hop_index(g, sc, h, 3, 3), tw[3]);
                site(h, sc);
            }
        } else {
            site(h0, decode_site(g, h0, parity));
        }
    }

    if constexpr (EPI) {
        if (!partials) return;  // uniform: the caller wants no <y, out>
        // deterministic block reduction: wave shuffles, then the waves of each
        // RHS tile in order
        __shared__ double red[4][TILE];
#pragma unroll
        for (int r = 0; r < TILE; ++r) {
            double s = wave_sum(part[r]);
            if (lane == 0) red[wave][r] = s;
        }
        __syncthreads();
        const int t = threadIdx.x;
        if (t < RS * TILE && rb + t < nrhs) {
            const int rs = t / TILE, r = t % TILE;
            double s = 0.0;
            for (int w = rs; w < (int)(blockDim.x >> 6); w += RS) s += red[w][r];
            partials[(size_t)(rb + t) * nb + blk] = s;
        }
    }
}

template <int LF, int SI, int SO, int TILE, bool EPI, int RS, int MODE>
static void launch_mode(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    dim3 block(a.block);
    const int ntiles = (a.nrhs + TILE - 1) / TILE;
    dim3 grid(dslash_grid_blocks(g, a.block, a.order), (ntiles + RS - 1) / RS);
    const size_t lds = MODE == MODE_XROW ? (size_t)TILE * 3 * a.block * 2 * sizeof(typename RealOf<LF>::T) : 0;
    Spinor<SI> in = spinor_view<SI>(const_cast<void *>(a.in), g.vh);
    Spinor<SO> out = spinor_view<SO>(a.out, g.vh);
    Spinor<SI> y = spinor_view<SI>(const_cast<void *>(a.y ? a.y : a.in), g.vh);
    if constexpr (LF != F64) {  // FP64 links are always stored whole
        if (a.compressed == COMP_SIGN) {
            hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_SIGN, RS, MODE>), grid, block, lds, s, g,
                               a.links, in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
            return;
        }
        if (a.compressed == COMP_KAPPA) {
            hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_KAPPA, RS, MODE>), grid, block, lds, s, g,
                               a.links, in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
            return;
        }
    }
    hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_NONE, RS, MODE>), grid, block, lds, s, g, a.links,
                       in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
}

// LDS of the x-row staging per workgroup: TILE x 3 colours x block sites
static size_t xrow_lds_bytes(int fl, int tile, int block) {
    return (size_t)tile * 3 * block * 2 * (fl == F64 ? 8 : 4);
}
static constexpr size_t kXrowLdsMax = 64 * 1024;

template <int LF, int SI, int SO, int TILE, bool EPI, int RS>
static void launch_rs(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    const int kind = order_tiles(a.order) & 0xff;
    if constexpr (RS == 1 && TILE <= 8) {
        if (kind == 3) {
            launch_mode<LF, SI, SO, TILE, EPI, 1, MODE_XROW>(g, a, s);
            return;
        }
    }
    if constexpr (TILE <= 4) {
        if (kind == 4) {
            launch_mode<LF, SI, SO, TILE, EPI, RS, MODE_TMARCH>(g, a, s);
            return;
        }
    }
    launch_mode<LF, SI, SO, TILE, EPI, RS, MODE_PLAIN>(g, a, s);
}

template <int LF, int SI, int SO, int TILE, bool EPI>
static void launch_one(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    switch (order_rsplit(a.order)) {
        case 2: launch_rs<LF, SI, SO, TILE, EPI, 2>(g, a, s); break;
        case 4: launch_rs<LF, SI, SO, TILE, EPI, 4>(g, a, s); break;
        default: launch_rs<LF, SI, SO, TILE, EPI, 1>(g, a, s); break;
    }
}

template <int LF, int SI, int SO, bool EPI>
static int launch_tile(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    switch (a.tile) {
        case 1: launch_one<LF, SI, SO, 1, EPI>(g, a, s); return 0;
        case 2: launch_one<LF, SI, SO, 2, EPI>(g, a, s); return 0;
        case 4: launch_one<LF, SI, SO, 4, EPI>(g, a, s); return 0;
        case 8:
            if constexpr (LF != F64) {
                launch_one<LF, SI, SO, 8, EPI>(g, a, s);
                return 0;
            }
            [[fallthrough]];
        case 16:
            if constexpr (LF != F64) {
                if (a.tile == 16) {
                    launch_one<LF, SI, SO, 16, EPI>(g, a, s);
                    return 0;
                }
            }
            [[fallthrough]];
        default: return -1;
    }
}

template <int LF, int SI, int SO>
static int launch_epi(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    return a.diag ? launch_tile<LF, SI, SO, true>(g, a, s) : launch_tile<LF, SI, SO, false>(g, a, s);
}

bool order_supported(const Geom &g, int order, int block) {
    if (order < 0 || (order >> 26)) return false;
    const int rs = order_rsplit(order);
    if (rs == 8 || block / rs < 64) return false;  // whole waves of sites
    // x-row staging: one wave per site, workgroups of whole rows
    if (order == 3) return (block == 64 || block == 128 || block == 192 || block == 256) && block % g.lxh == 0;
    if (block != 64 && block != 128 && block != 256) return false;
    block /= rs;
    order = order_tiles(order);
    const int kind = order & 0xff;
    if (kind == 0) return order == 0;
    if (kind == 4) {  // t-march: K sites per thread, K dividing Lt / 2
        const int k = (order >> 8) & 0xff;
        return (order >> 16) == 0 && k >= 1 && (g.L[3] / 2) % k == 0;
    }
    if (g.vh % 64 || (g.lxh * g.L[1]) % 64) return false;
    if (kind == 1) return order == 1;
    if (kind != 2 || (order >> 24)) return false;
    // whole tiles per column row block, whole blocks, and a grid of whole
    // eighths (the XCD remap is a permutation only then)
    const int by = (order >> 8) & 0xff, bz = (order >> 16) & 0xff;
    if (by < 1 || bz < 1 || g.L[1] % by || g.L[2] % bz || (g.lxh * by) % 64) return false;
    if (block < 64 || g.vh % block) return false;
    return (g.vh / block) % 8 == 0;
}

int launch_dslash(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    const bool xrow = a.order == 3;
    if (a.block != 64 && a.block != 128 && a.block != 256 && !(xrow && a.block == 192)) {
        set_error("dslash: block size must be 64, 128 or 256 (or 192 with x-row staging)");
        return HISQ_ERR_INVALID;
    }
    if (!order_supported(g, a.order, a.block)) {
        set_error("dslash: traversal order not supported for this lattice");
        return HISQ_ERR_INVALID;
    }
    if (xrow && (a.tile > 8 || xrow_lds_bytes(a.fmt_links, a.tile, a.block) > kXrowLdsMax)) {
        set_error("dslash: x-row staging takes RHS tiles of at most 8 and 64 KiB of LDS");
        return HISQ_ERR_INVALID;
    }
    if ((order_tiles(a.order) & 0xff) == 4 && a.tile > 4) {
        set_error("dslash: the t-march takes RHS tiles of at most 4");
        return HISQ_ERR_INVALID;
    }
    int rc = -1;
    if (a.fmt_links == F64 && a.fmt_in == F64 && a.fmt_out == F64)
        rc = launch_epi<F64, F64, F64>(g, a, s);
    else if (a.fmt_links == F32 && a.fmt_in == F32 && a.fmt_out == F32)
        rc = launch_epi<F32, F32, F32>(g, a, s);
    else if (a.fmt_links == H16 && a.fmt_in == H16 && a.fmt_out == H16)
        rc = launch_epi<H16, H16, H16>(g, a, s);
    else if (a.fmt_links == H16 && a.fmt_in == H16 && a.fmt_out == F32)
        rc = launch_epi<H16, H16, F32>(g, a, s);
    else if (a.fmt_links == H16 && a.fmt_in == F32 && a.fmt_out == F32)
        rc = launch_epi<H16, F32, F32>(g, a, s);
    if (rc != 0) {
        set_error("dslash: unsupported precision / tile combination");
        return HISQ_ERR_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("dslash launch: ") + hipGetErrorString(e));
        return HISQ_ERR_HIP;
    }
    return HISQ_OK;
}

}  // namespace hisq
