// Autotuner for the Dslash launch shape.
//
// For one (link precision, input/output formats, number of RHS, epilogue) it
// times every candidate (RHS tile per thread, number of waves a site's RHS
// tiles are split over, block size, tile processing order) on the handle's
// own links with HIP events, after checking that the
// candidate writes exactly the bytes the default shape writes (every shape
// performs the same per-site arithmetic in the same order).  The fastest shape
// is installed in the handle and, if a cache file is given, appended to it as
// one JSON object per line, keyed by device architecture, formats, lattice and
// RHS count; a later call finds it there and skips the timing.

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "solver_internal.h"

namespace hisq {

template <int F>
__global__ __launch_bounds__(256) void k_fill_spinor(Spinor<F> s, unsigned int seed) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= s.vh) return;
    typedef typename RealOf<F>::T R;
    cx<R> v[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        unsigned int x = (unsigned int)(h * 6 + c) * 2654435761u ^ (seed + blockIdx.y * 7919u);
        x ^= x >> 13;
        x *= 0x5bd1e995u;
        x ^= x >> 15;
        const R val = (R)((x & 0xffff) * (1.0 / 65536.0) - 0.5);
        if (c & 1) v[c >> 1].im = val;
        else v[c >> 1].re = val;
    }
    s.rhs(blockIdx.y).store(h, v);
}

__global__ void k_count_diff(const unsigned int *a, const unsigned int *b, size_t n, unsigned int *count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    unsigned int c = 0;
    for (; i < n; i += stride) c += a[i] != b[i];
    if (c) atomicAdd(count, c);
}

static int fill(int fmt, void *p, int vh, int n, unsigned seed, hipStream_t s) {
    dim3 grid((vh + 255) / 256, n);
    switch (fmt) {
        case F64: hipLaunchKernelGGL(k_fill_spinor<F64>, grid, dim3(256), 0, s, spinor_view<F64>(p, vh), seed); break;
        case F32: hipLaunchKernelGGL(k_fill_spinor<F32>, grid, dim3(256), 0, s, spinor_view<F32>(p, vh), seed); break;
        default: hipLaunchKernelGGL(k_fill_spinor<H16>, grid, dim3(256), 0, s, spinor_view<H16>(p, vh), seed); break;
    }
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

static std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static std::string tune_key(hisq_gauge_s *g, int fl, int fi, int fo, int nrhs, bool epi) {
    std::ostringstream k;
    k << arch_name(g->device) << "|" << fl << fi << fo << "|" << g->dims[0] << "x" << g->dims[1] << "x" << g->dims[2]
      << "x" << g->dims[3] << "|n" << nrhs << "|e" << (int)epi << (links_compressed(g, fl) == COMP_SIGN ? "|c" : links_compressed(g, fl) == COMP_KAPPA ? "|u" : "");
    return k.str();
}

// Look the key up in a JSON-lines cache: {"key": "...", "tile": T, "block": B, "order": O, "ms": M}
static bool cache_lookup(const char *path, const std::string &key, DslashShape *out) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const std::string want = "\"key\": \"" + key + "\"";
        if (line.find(want) == std::string::npos) continue;
        DslashShape s;
        char buf[256];
        double ms = 0;
        if (std::sscanf(line.c_str(), "{\"key\": \"%255[^\"]\", \"tile\": %d, \"block\": %d, \"order\": %d, \"ms\": %lf}",
                        buf, &s.tile, &s.block, &s.order, &ms) == 5) {
            *out = s;  // last matching line wins
            found = true;
        }
    }
    return found;
}

static void cache_append(const char *path, const std::string &key, const DslashShape &s, double ms) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    char buf[512];
    std::snprintf(buf, sizeof(buf), "{\"key\": \"%s\", \"tile\": %d, \"block\": %d, \"order\": %d, \"ms\": %.6f}\n",
                  key.c_str(), s.tile, s.block, s.order, ms);
    f << buf;
}

// Candidate traversal orders: memory order, t-fastest planes, and, for window
// budgets of 1, 2 and 4 MiB (one XCD's L2 holds 4 MiB, shared with the link
// stream), the XCD-brick column whose seven-t-slice window of input spinors
// (a tile of RHS) fits the budget with the fewest face re-reads 6/BY + 6/BZ.
static std::vector<int> brick_orders(const Geom &G, int fi, int tile) {
    std::vector<int> o{0, 1};
    const double site_b = (fi == F64 ? 48.0 : fi == F32 ? 24.0 : 16.0) * tile;
    for (double budget : {1.0, 2.0, 4.0}) {
        int best = -1;
        double best_cost = 1e30;
        for (int by = 1; by <= std::min(G.L[1], 255); ++by)
            for (int bz = 1; bz <= std::min(G.L[2], 255); ++bz) {
                if (G.L[1] % by || G.L[2] % bz || (G.lxh * by) % 64) continue;
                if (7.0 * G.lxh * by * bz * site_b > budget * 1024 * 1024) continue;
                const double cost = 6.0 / by + 6.0 / bz;
                if (cost < best_cost) {
                    best_cost = cost;
                    best = 2 | by << 8 | bz << 16;
                }
            }
        if (best >= 0 && std::find(o.begin(), o.end(), best) == o.end()) o.push_back(best);
    }
    return o;
}

// RHS split of a shape (bits 24-25 of its order: waves sharing a site's links)
static int shape_rsplit(const DslashShape &s) { return 1 << ((s.order >> 24) & 3); }

static bool valid_shape(const Geom &geom, int fl, int nrhs, const DslashShape &s) {
    if (s.tile < 1 || s.tile > 16 || (s.tile & (s.tile - 1)) || s.tile > std::max(1, nrhs)) return false;
    if (fl == F64 && s.tile > 4) return false;
    if ((s.order & 0xff) == 4 && s.tile > 4) return false;  // t-march: RHS tiles of up to 4
    if (s.order == 3) {  // x-row staging: RHS tiles of up to 8 in at most 64 KiB of LDS
        if (s.tile > 8 || (size_t)s.tile * 3 * s.block * 2 * (fl == F64 ? 8 : 4) > 64 * 1024) return false;
    } else if (s.block != 64 && s.block != 128 && s.block != 256) {
        return false;
    }
    // a split wider than the RHS count only adds idle waves
    int p2 = 1;
    while (p2 < nrhs) p2 <<= 1;
    if (s.tile * shape_rsplit(s) > p2) return false;
    return order_supported(geom, s.order, s.block);
}

int tune_dslash(hisq_gauge_s *g, int fl, int fi, int fo, int nrhs, bool epi, const char *cache, hipStream_t s,
                DslashShape *chosen, double *chosen_ms) {
    const Geom &G = g->geom;
    const auto map_key = std::make_tuple(fl, fi, fo, nrhs, (int)epi);
    const std::string key = tune_key(g, fl, fi, fo, nrhs, epi);
    DslashShape cached;
    if (cache_lookup(cache, key, &cached) && valid_shape(G, fl, nrhs, cached)) {
        g->shapes[map_key] = cached;
        g->cg_ws.clear();  // captured graphs hold the old shapes
        if (chosen) *chosen = cached;
        if (chosen_ms) *chosen_ms = -1.0;
        return HISQ_OK;
    }
    if (!g->links[fl][0].p) {
        set_error("autotune: links of this precision were not packed");
        return HISQ_ERR_UNSUPPORTED;
    }
    const size_t in_b = spinor_bytes(fi, G.vh) * nrhs, out_b = spinor_bytes(fo, G.vh) * nrhs;
    DevBuf in, y, out, ref, part, diag, cnt;
    int rc;
    if ((rc = in.alloc(in_b)) || (rc = out.alloc(out_b)) || (rc = ref.alloc(out_b)) ||
        (rc = part.alloc(sizeof(double) * (size_t)nrhs * ((G.vh + 63) / 64))) ||
        (rc = diag.alloc(sizeof(double) * nrhs)) || (rc = cnt.alloc(sizeof(unsigned int))))
        return rc;
    if (epi && (rc = y.alloc(in_b))) return rc;
    if ((rc = fill(fi, in.p, G.vh, nrhs, 12345u, s))) return rc;
    if (epi && (rc = fill(fi, y.p, G.vh, nrhs, 777u, s))) return rc;
    std::vector<double> dh(nrhs);
    for (int i = 0; i < nrhs; ++i) dh[i] = 0.01 + 0.1 * i;
    HISQ_HIP_CHECK(hipMemcpyAsync(diag.p, dh.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, s));

    auto launch = [&](const DslashShape &sh, void *dst) {
        DslashLaunch a{};
        a.links = g->links[fl][0].p;
        a.in = in.p;
        a.out = dst;
        a.y = epi ? y.p : nullptr;
        a.diag = epi ? (const double *)diag.p : nullptr;
        a.partials = epi ? (double *)part.p : nullptr;
        a.skip = nullptr;
        a.nrhs = nrhs;
        a.parity = 0;
        a.fmt_links = fl;
        a.fmt_in = fi;
        a.fmt_out = fo;
        a.tile = sh.tile;
        a.block = sh.block;
        a.order = sh.order;
        a.compressed = links_compressed(g, fl);
        return launch_dslash(G, a, s);
    };

    DslashShape ref_shape;  // tile 1, block 256, memory order: always valid
    ref_shape.tile = 1;
    ref_shape.block = 256;
    ref_shape.order = 0;
    if ((rc = launch(ref_shape, ref.p))) return rc;

    std::vector<DslashShape> cands;
    for (int rsl = 0; rsl <= 2; ++rsl)  // RHS tiles of a site on 1, 2 or 4 waves
        for (int tile : {1, 2, 4, 8, 16})
            for (int block : {64, 128, 256})
                for (int order : brick_orders(G, fi, tile << rsl)) {
                    DslashShape c;
                    c.tile = tile;
                    c.block = block;
                    c.order = order | rsl << 24;
                    if (valid_shape(G, fl, nrhs, c)) cands.push_back(c);
                }
    for (int rsl = 0; rsl <= 2; ++rsl)  // t-march: K sites per thread along t
        for (int tile : {1, 2, 4})
            for (int block : {64, 128, 256})
                for (int k = 1; k <= G.L[3] / 2; ++k) {
                    DslashShape c;
                    c.tile = tile;
                    c.block = block;
                    c.order = 4 | k << 8 | rsl << 24;
                    if (valid_shape(G, fl, nrhs, c)) cands.push_back(c);
                }
    for (int tile : {1, 2, 4, 8})  // x-row staging (whole rows per workgroup, one wave per site)
        for (int block : {64, 128, 192, 256}) {
            DslashShape c;
            c.tile = tile;
            c.block = block;
            c.order = 3;
            if (valid_shape(G, fl, nrhs, c)) cands.push_back(c);
        }

    hipEvent_t e0, e1;
    HISQ_HIP_CHECK(hipEventCreate(&e0));
    HISQ_HIP_CHECK(hipEventCreate(&e1));
    const int reps = G.vh >= (1 << 22) ? 4 : 10;
    DslashShape best = ref_shape;
    double best_ms = 1e30;
    for (const DslashShape &c : cands) {
        HISQ_HIP_CHECK(hipMemsetAsync(cnt.p, 0, sizeof(unsigned int), s));
        if ((rc = launch(c, out.p))) break;
        hipLaunchKernelGGL(k_count_diff, dim3(1024), dim3(256), 0, s, (const unsigned int *)ref.p,
                           (const unsigned int *)out.p, out_b / 4, (unsigned int *)cnt.p);
        unsigned int diff = 0;
        HISQ_HIP_CHECK(hipMemcpyAsync(&diff, cnt.p, sizeof(diff), hipMemcpyDeviceToHost, s));
        HISQ_HIP_CHECK(hipStreamSynchronize(s));
        if (diff != 0) continue;  // a shape that changes the result never wins
        if ((rc = launch(c, out.p))) break;
        HISQ_HIP_CHECK(hipEventRecord(e0, s));
        for (int r = 0; r < reps && rc == HISQ_OK; ++r) rc = launch(c, out.p);
        HISQ_HIP_CHECK(hipEventRecord(e1, s));
        HISQ_HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0;
        HISQ_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    g->shapes[map_key] = best;
    g->cg_ws.clear();
    cache_append(cache, key, best, best_ms);
    if (chosen) *chosen = best;
    if (chosen_ms) *chosen_ms = best_ms;
    return HISQ_OK;
}

}  // namespace hisq
