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
    return (g.vh + sb - 1) / sb;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// XR (traversal order 3, RS = 1): the workgroup's sites are whole x-rows in
// memory order; it stages the input colour vectors of those rows (its RHS
// tile) in LDS, and the four x-direction hops of every site read LDS instead
// of gathering through the caches.  A separate instance, so that the other
// kernels keep their branch-free hop loops.
template <int LF, int SI, int SO, int TILE, bool EPI, int CM, int RS, bool XR = false>
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
    const int h = site_of_thread(g, blk, nb, (int)blockDim.x / RS, (wave / RS) * 64 + lane, order & 0xffffff);
    const int rb = blockIdx.y * RS * TILE;  // first RHS of the workgroup
    const int r0 = rb + rsub * TILE;
    if (skip) {
        bool idle = true;
        for (int r = rb; r < rb + RS * TILE && r < nrhs; ++r)
            if (skip[r].flag == CG_RUNNING) idle = false;
        if (idle) return;  // uniform over the block
    }

    // x-row staging: thread t loads the input vectors of site base + t (the
    // same row index in the input parity), for every RHS of its tile
    extern __shared__ unsigned char xr_lds[];
    cx<R> *xs = reinterpret_cast<cx<R> *>(xr_lds);  // [TILE][3][blockDim.x]
    const int xbase = blk * (int)blockDim.x;
    if constexpr (XR) {
        static_assert(RS == 1, "x-row staging needs one wave per site");
        if (h < g.vh) {
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                const int rr = (TILE > 1 && r0 + r >= nrhs) ? nrhs - 1 : r0 + r;
                cx<R> v[3];
                in.rhs(rr).load(h, v);
#pragma unroll
                for (int c = 0; c < 3; ++c) xs[(r * 3 + c) * (int)blockDim.x + threadIdx.x] = v[c];
            }
        }
        __syncthreads();
    }

    double part[TILE];
#pragma unroll
    for (int r = 0; r < TILE; ++r) part[r] = 0.0;

    if (h < g.vh && r0 < nrhs) {
        const SiteCoord sc = decode_site(g, h, parity);
        cx<R> acc[TILE][3];
#pragma unroll
        for (int r = 0; r < TILE; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[r][c] = {R(0), R(0)};

        // acc += m * (neighbour of slot k), for every RHS of the tile
        auto apply = [&](int k, const cx<R> *m) {
            const int nbh = hop_index(g, sc, h, k >> 2, slot_dist(k & 3));
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                // a ragged last tile repeats its last RHS (those results are
                // never stored): no branch, so the compiler can issue the
                // gathers of every RHS of the tile before the first one returns
                const int rr = (TILE > 1 && r0 + r >= nrhs) ? nrhs - 1 : r0 + r;
                const Spinor<SI> src = in.rhs(rr);
                cx<R> v[3];
                src.load(nbh, v);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) cmac(acc[r][a], m[3 * a + b], v[b]);
            }
        };
        // the same for an x-direction slot (k < 4) from the staged rows
        auto apply_x = [&](int k, const cx<R> *m) {
            const int li = hop_index(g, sc, h, 0, slot_dist(k & 3)) - xbase;
#pragma unroll
            for (int r = 0; r < TILE; ++r) {
                cx<R> v[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) v[b] = xs[(r * 3 + b) * (int)blockDim.x + li];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) cmac(acc[r][a], m[3 * a + b], v[b]);
            }
        };
        // One RHS: every slot unrolled, the compiler interleaves the loads of
        // neighbouring slots.  Several RHS: one link group (or compressed
        // chunk) per loop trip with the gathers of all its RHS in flight
        // together; unrolled, the compiler hoists every gather of the site and
        // spills them to scratch.
        if constexpr (CM == COMP_NONE) {
            const Links<LF, NT> links{lptr};
            // xd: the group's slots are x-direction hops read from the staged rows
            auto group = [&](int gi, auto xd) {
                cx<R> w[9 * G];
                links.load_group(gi, h, w);
#pragma unroll
                for (int sl = 0; sl < G; ++sl) {
                    if constexpr (decltype(xd)::value) apply_x(gi * G + sl, w + 9 * sl);
                    else apply(gi * G + sl, w + 9 * sl);
                }
            };
            constexpr int GX = XR ? 4 / G : 0;  // groups of x-direction slots
            if constexpr (TILE == 1) {
#pragma unroll
                for (int gi = 0; gi < GX; ++gi) group(gi, std::true_type{});
#pragma unroll
                for (int gi = GX; gi < 16 / G; ++gi) group(gi, std::false_type{});
            } else {
#pragma unroll
                for (int gi = 0; gi < GX; ++gi) group(gi, std::true_type{});
#pragma unroll 1
                for (int gi = GX; gi < 16 / G; ++gi) group(gi, std::false_type{});
            }
        } else {
            // fat slots whole; long slots from rows 0, 1 and the determinant
            // sign (COMP_SIGN) or the complex factor kappa (COMP_KAPPA)
            constexpr int MC = CompGeom<LF>::MC, NC = CompGeom<LF>::NC;
            const LinksC<LF, CM, NT> cl{lptr, g.vh};
            unsigned sg = 0;
            if constexpr (CM == COMP_SIGN) sg = cl.signs(h);
            // xd: chunk 0, whose mu = 0 slots read the staged rows
            auto chunk = [&](int c, auto xd) {
                {
                    cx<R> w[18 * MC];
                    cl.load_fat(c, h, w);
#pragma unroll
                    for (int s2 = 0; s2 < 2 * MC; ++s2) {
                        const int k = 4 * (c * MC + (s2 >> 1)) + (s2 & 1);
                        if constexpr (decltype(xd)::value) {
                            if (s2 < 2) apply_x(k, w + 9 * s2);  // s2 is unrolled: folded
                            else apply(k, w + 9 * s2);
                        } else {
                            apply(k, w + 9 * s2);
                        }
                    }
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
                        if constexpr (decltype(xd)::value) {
                            if (s2 < 2) apply_x(4 * mu + 2 + (s2 & 1), m);
                            else apply(4 * mu + 2 + (s2 & 1), m);
                        } else {
                            apply(4 * mu + 2 + (s2 & 1), m);
                        }
                    }
                }
            };
            // (a chunk's fat and long slots in separate loop trips halve the
            // registers but measured 5-10 % slower: fewer gathers in flight)
            constexpr int CX = XR ? 1 : 0;  // chunk 0 holds the x-direction slots
            if constexpr (XR) chunk(0, std::true_type{});
            if constexpr (TILE == 1) {
#pragma unroll
                for (int c = CX; c < NC; ++c) chunk(c, std::false_type{});
            } else {
#pragma unroll 1
                for (int c = CX; c < NC; ++c) chunk(c, std::false_type{});
            }
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
                part[r] = pr;
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

template <int LF, int SI, int SO, int TILE, bool EPI, int RS, bool XR>
static void launch_xr(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    dim3 block(a.block);
    const int ntiles = (a.nrhs + TILE - 1) / TILE;
    dim3 grid(dslash_grid_blocks(g, a.block, a.order), (ntiles + RS - 1) / RS);
    const size_t lds = XR ? (size_t)TILE * 3 * a.block * 2 * sizeof(typename RealOf<LF>::T) : 0;
    Spinor<SI> in = spinor_view<SI>(const_cast<void *>(a.in), g.vh);
    Spinor<SO> out = spinor_view<SO>(a.out, g.vh);
    Spinor<SI> y = spinor_view<SI>(const_cast<void *>(a.y ? a.y : a.in), g.vh);
    if constexpr (LF != F64) {  // FP64 links are always stored whole
        if (a.compressed == COMP_SIGN) {
            hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_SIGN, RS, XR>), grid, block, lds, s, g,
                               a.links, in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
            return;
        }
        if (a.compressed == COMP_KAPPA) {
            hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_KAPPA, RS, XR>), grid, block, lds, s, g,
                               a.links, in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
            return;
        }
    }
    hipLaunchKernelGGL((dslash_kernel<LF, SI, SO, TILE, EPI, COMP_NONE, RS, XR>), grid, block, lds, s, g, a.links,
                       in, out, y, a.diag, a.partials, a.skip, a.parity, a.nrhs, a.order);
}

// LDS of the x-row staging per workgroup: TILE x 3 colours x block sites
static size_t xrow_lds_bytes(int fl, int tile, int block) {
    return (size_t)tile * 3 * block * 2 * (fl == F64 ? 8 : 4);
}
static constexpr size_t kXrowLdsMax = 64 * 1024;

template <int LF, int SI, int SO, int TILE, bool EPI, int RS>
static void launch_rs(const Geom &g, const DslashLaunch &a, hipStream_t s) {
    if constexpr (RS == 1 && TILE <= 8) {
        if ((order_tiles(a.order) & 0xff) == 3) {
            launch_xr<LF, SI, SO, TILE, EPI, 1, true>(g, a, s);
            return;
        }
    }
    launch_xr<LF, SI, SO, TILE, EPI, RS, false>(g, a, s);
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
