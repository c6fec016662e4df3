// Host-side check of the Dslash kernel's index arithmetic, built from the
// kernel's own helpers (hisq_internal.h: site_of_thread, decode_site,
// hop_index, link_unit_ptr, comp_unit_ptr are host + device).  For every
// thread of the launch grids the kernel uses - block sizes 64, 128, 256 (and
// 192 with x-row staging), every traversal order the launcher accepts - it
// checks that
//  * the threads inside the lattice cover every output site exactly once;
//  * with x-row staging, every x-direction hop stays inside the workgroup's
//    own staged rows;
//  * with the t-march, the K sites of every thread cover each output site
//    once and each step stays in its (x, y, z) column;
//  * the decoded coordinates give back the site and its parity;
//  * each of the 16 hops lands on the site a coordinate-based reference gives,
//    of the other parity, inside [0, Vh);
//  * every 16-byte link unit a thread reads, whole or compressed layout (sign
//    or kappa mode), lies inside the packed buffer, and the sign word inside
//    the sign plane.
// Prints one line per lattice and exits non-zero on the first violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hisq_internal.h"

using namespace hisq;

static int fails = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            if (++fails > 20) std::exit(1);               \
        }                                                 \
    } while (0)

static long lex_of(const int L[4], const int c[4]) { return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3])); }

// units of 16 bytes in one parity's packed links
static long whole_units(int f, long vh) { return (long)link_parity_bytes(f, vh, COMP_NONE) / 16; }
static long comp_units_total(int f, long vh, int mode) { return (long)link_parity_bytes(f, vh, mode) / 16; }

static void check_lattice(const int dims[4], bool quick) {
    const Geom g = make_geom(dims);
    const long vh = g.vh;
    std::vector<int> orders = {0, 1};
    for (int by : {4, 8, 12, 16, 24})
        for (int bz : {2, 4, 8, 12, 16}) orders.push_back(2 | by << 8 | bz << 16);
    long launches = 0;
    for (int parity = 0; parity < 2; ++parity) {
        // x-row staging (order 3): memory order, and every x-direction hop of a
        // site inside the thread's own workgroup (the rows it staged in LDS)
        for (int block : {64, 128, 192, 256}) {
            if (!order_supported(g, 3, block)) continue;
            ++launches;
            const int nbs = dslash_grid_blocks(g, block, 3);
            CHECK(nbs == (int)((vh + block - 1) / block), "x-row grid of %d blocks for block %d", nbs, block);
            for (int blk = 0; blk < nbs; ++blk)
                for (int tid = 0; tid < block; ++tid) {
                    const int h = site_of_thread(g, blk, nbs, block, tid, 3);
                    CHECK(h == blk * block + tid, "x-row order is not memory order at block %d", blk);
                    if (h >= vh) continue;
                    const SiteCoord sc = decode_site(g, h, parity);
                    for (int k = 0; k < 4; ++k) {
                        const int li = hop_index(g, sc, h, 0, slot_dist(k)) - blk * block;
                        CHECK(li >= 0 && li < block && blk * block + li < vh,
                              "x-row hop of site %d slot %d outside its workgroup (block %d)", h, k, block);
                    }
                }
        }
        // t-march (order 4, K sites per thread along t): the K sites of every
        // thread of the grid, split over 1, 2, 4 waves, cover each output
        // site exactly once
        for (int k = 1; k <= dims[3] / 2; ++k)
            for (int block : {64, 128, 256})
                for (int rsl = 0; rsl <= 2; ++rsl) {
                    const int order = 4 | k << 8 | rsl << 24, sb = block >> rsl;
                    if (!order_supported(g, order, block)) continue;
                    if (quick && (rsl || block != 128)) continue;
                    ++launches;
                    const int nbs = dslash_grid_blocks(g, block, order);
                    CHECK(nbs == (int)((vh / k + sb - 1) / sb), "t-march grid of %d blocks (K %d block %d)", nbs, k,
                          block);
                    std::vector<unsigned char> seen(vh, 0);
                    for (int blk = 0; blk < nbs; ++blk)
                        for (int tid = 0; tid < sb; ++tid) {
                            const int h0 = tmarch_first_site(g, blk * sb + tid, k);
                            if (h0 >= vh) continue;
                            for (int s = 0; s < k; ++s) {
                                const long h = h0 + (long)s * 2 * g.st;
                                CHECK(h >= 0 && h < vh, "t-march site %ld out of range (K %d)", h, k);
                                if (h < 0 || h >= vh) continue;
                                CHECK(!seen[h], "t-march site %ld twice (K %d block %d)", h, k, block);
                                seen[h] = 1;
                                if (s > 0) {  // the same column, two t-slices on
                                    const SiteCoord a = decode_site(g, (int)(h - 2 * g.st), parity);
                                    const SiteCoord b = decode_site(g, (int)h, parity);
                                    CHECK(a.x == b.x && a.y == b.y && a.z == b.z && b.t == a.t + 2,
                                          "t-march step of site %ld leaves its column", h);
                                }
                            }
                        }
                    for (long h = 0; h < vh; ++h)
                        CHECK(seen[h], "t-march site %ld never visited (K %d block %d)", h, k, block);
                }
        for (int block : {64, 128, 256}) {
            for (int base : orders)
            for (int rsl = 0; rsl <= 2; ++rsl) {
                // RHS split over 1, 2, 4 waves: the kernel maps its block of
                // `block` threads onto block / RS sites with the tile order bits
                const int order = base | rsl << 24, sb = block >> rsl;
                if (!order_supported(g, order, block)) continue;
                if (quick && (rsl || (base > 1 && base != orders[2 + 7]))) continue;
                ++launches;
                const int nbs = dslash_grid_blocks(g, block, order);
                CHECK(nbs == (int)((vh + sb - 1) / sb), "grid of %d blocks for block %d split %d", nbs, block, 1 << rsl);
                std::vector<unsigned char> seen(vh, 0);
                for (int blk = 0; blk < nbs; ++blk)
                    for (int tid = 0; tid < sb; ++tid) {
                        const int h = site_of_thread(g, blk, nbs, sb, tid, base);
                        if (h >= vh) continue;  // grid tail, skipped by the kernel's guard
                        CHECK(h >= 0, "negative site %d (order %d block %d)", h, order, block);
                        CHECK(!seen[h], "site %d twice (order %d block %d)", h, order, block);
                        seen[h] = 1;
                    }
                for (long h = 0; h < vh; ++h) CHECK(seen[h], "site %ld never visited (order %d block %d)", h, order, block);
            }
        }
        // geometry and hops (independent of the launch shape)
        for (long h = 0; h < vh; ++h) {
            const SiteCoord sc = decode_site(g, (int)h, parity);
            const int c[4] = {sc.x, sc.y, sc.z, sc.t};
            const long lex = lex_of(dims, c);
            CHECK((lex >> 1) == h && ((c[0] + c[1] + c[2] + c[3]) & 1) == parity, "decode of site %ld parity %d", h, parity);
            for (int k = 0; k < 16; ++k) {
                const int mu = k >> 2, d = slot_dist(k & 3);
                const int nbh = hop_index(g, sc, (int)h, mu, d);
                int cn[4] = {c[0], c[1], c[2], c[3]};
                cn[mu] = ((cn[mu] + d) % dims[mu] + dims[mu]) % dims[mu];
                const long ref = lex_of(dims, cn);
                CHECK(nbh >= 0 && nbh < vh, "hop out of range: site %ld slot %d -> %d", h, k, nbh);
                CHECK(nbh == (ref >> 1) && ((cn[0] + cn[1] + cn[2] + cn[3]) & 1) == 1 - parity,
                      "hop of site %ld slot %d: %d, reference %ld", h, k, nbh, ref >> 1);
            }
            // link units of the site: whole layout (groups of 1, 2, 4 slots)
            for (int f : {F64, F32, H16}) {
                const int G = f == F64 ? 1 : f == F32 ? 2 : 4, ng = 16 / G;
                for (int gi = 0; gi < ng; ++gi) {
                    const long u = (long)(link_unit_ptr(nullptr, ng, gi, (int)h) - (const u4v *)nullptr);
                    CHECK(u >= 0 && u + 8 * 64 < whole_units(f, vh), "whole link unit %ld of site %ld fmt %d", u, h, f);
                }
            }
            // compressed layouts (FP32 and FP16): sign mode with its sign word,
            // kappa mode with its kappa unit (the last unit of every chunk)
            {
                constexpr int NC = CompGeom<F32>::NC, UC = comp_chunk_units<F32>(COMP_SIGN);
                for (int cc = 0; cc < NC; ++cc) {
                    const long u = (long)(comp_unit_ptr<F32, COMP_SIGN>(nullptr, cc, (int)h) - (const u4v *)nullptr);
                    CHECK(u >= 0 && u + (UC - 1) * 64 < comp_units_total(F32, vh, COMP_SIGN),
                          "compressed FP32 unit of site %ld", h);
                }
                const long tiles = (vh + LINK_TILE - 1) / LINK_TILE;
                CHECK((long)(tiles * comp_units_per_site(F32, COMP_SIGN) * 1024) + 4 * (h + 1) <=
                          (long)link_parity_bytes(F32, vh, COMP_SIGN),
                      "FP32 sign word of site %ld", h);
            }
            {
                constexpr int NC = CompGeom<H16>::NC, UC = comp_chunk_units<H16>(COMP_SIGN);
                for (int cc = 0; cc < NC; ++cc) {
                    const long u = (long)(comp_unit_ptr<H16, COMP_SIGN>(nullptr, cc, (int)h) - (const u4v *)nullptr);
                    CHECK(u >= 0 && u + (UC - 1) * 64 < comp_units_total(H16, vh, COMP_SIGN),
                          "compressed FP16 unit of site %ld", h);
                }
            }
            {
                constexpr int NC = CompGeom<F32>::NC, UC = comp_chunk_units<F32>(COMP_KAPPA);
                static_assert(UC == 16, "FP32 kappa chunk: 9 fat + 6 long + 1 kappa unit");
                for (int cc = 0; cc < NC; ++cc) {
                    const long u = (long)(comp_unit_ptr<F32, COMP_KAPPA>(nullptr, cc, (int)h) - (const u4v *)nullptr);
                    // the kernel reads units 0 .. 15 of the chunk (kappa at 15)
                    CHECK(u >= 0 && u + 15 * 64 < comp_units_total(F32, vh, COMP_KAPPA),
                          "kappa-compressed FP32 unit of site %ld", h);
                }
            }
            {
                constexpr int NC = CompGeom<H16>::NC, UC = comp_chunk_units<H16>(COMP_KAPPA);
                static_assert(UC == 16, "FP16 kappa chunk: 9 fat + 6 long + 1 kappa unit");
                for (int cc = 0; cc < NC; ++cc) {
                    const long u = (long)(comp_unit_ptr<H16, COMP_KAPPA>(nullptr, cc, (int)h) - (const u4v *)nullptr);
                    CHECK(u >= 0 && u + 15 * 64 < comp_units_total(H16, vh, COMP_KAPPA),
                          "kappa-compressed FP16 unit of site %ld", h);
                }
            }
        }
    }
    std::printf("%dx%dx%dx%d: Vh %ld, %ld launch shapes, %s\n", dims[0], dims[1], dims[2], dims[3], vh, launches,
                fails ? "FAILED" : "ok");
}

int main(int argc, char **argv) {
    const int lattices[][4] = {{4, 4, 4, 4}, {6, 4, 4, 10}, {10, 6, 4, 8}, {8, 8, 8, 8}, {16, 8, 8, 8},
                               {8, 6, 4, 10}, {12, 4, 4, 8}, {8, 12, 8, 16}, {16, 16, 16, 8}, {32, 32, 32, 8},
                               {48, 48, 48, 12}};
    for (const auto &d : lattices) check_lattice(d, false);
    if (argc > 1) {  // the benchmark lattice: Vh = 10.6 M, one traversal order per kind
        const int big[4] = {96, 96, 96, 24};
        check_lattice(big, true);
    }
    return fails ? 1 : 0;
}
