// Gauge-covariant preconditioner network: forward, backward and Adam kernels.
//
// Layer with C_in -> C_out complex channels (C <= 8) on the full lattice:
//   y_a(x) = sum_b [ W0_ab psi_b(x) + sum_mu ( Wf_mu,ab U_mu(x) psi_b(x+mu)
//                                            + Wb_mu,ab U_mu(x-mu)^+ psi_b(x-mu) ) ]
// (linear, gauge covariant; the L-CNN construction of Favoni et al. 2022 used
// as a solver preconditioner as in Lehner and Wettig 2023).
//
// Storage in HBM:
//  * hidden activations and back-propagated gradients: BF16, always 8
//    channels (unused ones hold zeros).  A site is six 16-byte units
//    u = 2 colour + (0: re, 1: im), each holding channels 0..7, tiled by 64
//    sites: unit u of site s at byte ((s / 64) * 6 + u) * 1024 + (s % 64) * 16.
//  * network input and output: FP32 spinors of the public layout, even sites.
//  * thin links: FP16, a 144-byte record per site (links mu = 0..3 of 9
//    complex entries, entry k of link mu in 32-bit word 9 mu + k), tiled by 64
//    sites like the activations, nine units per site.
//
// Kernel: a wavefront owns 32 sites, i.e. 96 (site, colour) columns, and
// builds the layer as the real-block GEMM
//   [Re y; Im y] (16 x 96) = A (16 x K) B (K x 96),  A = [[Wr, -Wi], [Wi, Wr]],
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  B is the transported
// input, produced 32 K rows at a time (two paths x {re, im} x 8 channels) by
// the wave's lanes in FP32 and staged in LDS as BF16: lane pair (site, half)
// loads the neighbour's units and the link once per pair and each half
// transports 4 of the 8 channels.  The result is staged in LDS and written
// as whole 16-byte units.  The adjoint layer needed by back-propagation is
// the same kernel with weights W'_{p'} = W_p^H, p' the adjoint hop.  Weight
// gradients G(W_p[a][b]) = sum_{x,c} g_a(x)_c conj((T_p psi_b)(x)_c) use the
// same MFMA with (site, colour, re/im) as the reduction, per-block partials
// and a fixed-order final sum (deterministic).

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nn_internal.h"

namespace hisq {

typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef __bf16 b4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }

constexpr int NW_SITES = 32;                 // sites per wavefront
constexpr int NW_COLS = 3 * NW_SITES;        // (site, colour) columns per wavefront
constexpr int NN_WAVES = 2;                  // wavefronts per block
constexpr int NB_SITES = NW_SITES * NN_WAVES;
constexpr int BT_LD = 40;                    // bf16 per LDS column of B: 32 K rows + pad
constexpr int GT_LD = 2 * NW_COLS + 8;       // bf16 per LDS row of the gradient operand

enum { IO_FULL = 0, IO_EVEN = 1 };

// K extent of the real-block weight matrix: 9 paths x {re, im} x 8 channels
// padded to 160 for hidden inputs, 9 paths x {re, im} padded to 32 for the
// one-channel even-site input.
__host__ __device__ constexpr int kp_of(int inm) { return inm == IO_EVEN ? 32 : 160; }

// ------------------------------------------------------------------ geometry (full lattice, lex order)
struct Lex {
    int L[4];
    int V;
};

struct SiteGeo {
    int s;     // lex index
    int c[4];  // coordinates
    int par;   // (x + y + z + t) & 1
};

__device__ __forceinline__ SiteGeo site_geo(const Lex &g, int s) {
    SiteGeo o;
    o.s = s;
    int r = s;
    o.c[0] = r % g.L[0];
    r /= g.L[0];
    o.c[1] = r % g.L[1];
    r /= g.L[1];
    o.c[2] = r % g.L[2];
    o.c[3] = r / g.L[2];
    o.par = (o.c[0] + o.c[1] + o.c[2] + o.c[3]) & 1;
    return o;
}

// lex index of x + d mu, d = +1 or -1
template <int MU>
__device__ __forceinline__ int hop(const Lex &g, const SiteGeo &x, int d) {
    int stride = 1;
#pragma unroll
    for (int k = 0; k < MU; ++k) stride *= g.L[k];
    const int c = x.c[MU], Lm = g.L[MU];
    if (d > 0) return c == Lm - 1 ? x.s - (Lm - 1) * stride : x.s + stride;
    return c == 0 ? x.s + (Lm - 1) * stride : x.s - stride;
}

// Enumerated site -> lex index: all sites in lex order, or the even sites in
// checkerboard order (h = lex / 2).
template <int MODE>
__device__ __forceinline__ int site_of(const Lex &g, int idx) {
    if constexpr (MODE == IO_FULL) {
        return idx;
    } else {
        const int lxh = g.L[0] >> 1;
        const int xh = idx % lxh, r = idx / lxh;
        const int y = r % g.L[1], z = (r / g.L[1]) % g.L[2], t = r / (g.L[1] * g.L[2]);
        return 2 * xh + ((y + z + t) & 1) + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
    }
}

// ------------------------------------------------------------------ thin links (FP16)
template <int MU>
__device__ __forceinline__ void load_link(const void *thin, int s, cx<float> w[9]) {
    const u4v *b = (const u4v *)thin + (size_t)(s >> 6) * 9 * 64 + (s & 63);
    constexpr int U0 = (9 * MU) / 4, OFF = (9 * MU) % 4;  // first unit, first word in it
    const u4v r0 = b[U0 * 64], r1 = b[(U0 + 1) * 64], r2 = b[(U0 + 2) * 64];
    const unsigned wd[12] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w, r2.x, r2.y, r2.z, r2.w};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const unsigned v = wd[OFF + k];
        const h2v h = __builtin_bit_cast(h2v, v);
        w[k] = {(float)h.x, (float)h.y};
    }
}

// Pack canonical FP64 thin links [V][4][3][3] complex into the FP16 records;
// *bad is set if an entry is not finite or too large for FP16.
__global__ __launch_bounds__(256) void k_pack_thin(Lex g, const double *__restrict__ U, void *dst, unsigned *bad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= g.V) return;
    unsigned *words = (unsigned *)dst;
    const double *src = U + ((size_t)s * 4 + mu) * 18;
    bool ok = true;
    for (int k = 0; k < 9; ++k) {
        const int wi = 9 * mu + k, e = wi >> 2, q = wi & 3;
        const double re = src[2 * k], im = src[2 * k + 1];
        ok = ok && fabs(re) < 32768.0 && fabs(im) < 32768.0;  // false for NaN as well
        const h2v h = {(_Float16)(float)re, (_Float16)(float)im};
        words[((size_t)(s >> 6) * 9 + e) * 256 + (size_t)(s & 63) * 4 + q] = __builtin_bit_cast(unsigned, h);
    }
    if (!ok) atomicOr(bad, 1u);
}

// ------------------------------------------------------------------ activations
__device__ __forceinline__ float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// Channels 4 h .. 4 h + 3 of the six units of site s: v[u] = 8 bytes of unit u.
__device__ __forceinline__ void load_act_half(const void *buf, int s, int h, u2v v[6]) {
    const u2v *b = (const u2v *)buf + ((size_t)(s >> 6) * 6 * 64 + (s & 63)) * 2 + h;
#pragma unroll
    for (int u = 0; u < 6; ++u) v[u] = b[(size_t)u * 128];
}

// channel q (0..3) of an 8-byte half unit
__device__ __forceinline__ float half_chan(const u2v &v, int q) {
    const unsigned w = (q < 2) ? v.x : v.y;
    return (q & 1) ? bf_hi(w) : bf_lo(w);
}

// ------------------------------------------------------------------ transport into LDS
// Path P (0 identity, 1..4 forward hop mu = P - 1, 5..8 backward hop
// mu = P - 5, 9 = padding) of channels 4h .. 4h + 3 of a hidden input at
// site x; writes the 3 colours x {re, im} x 4 channels to the LDS columns of
// the site at K offset koff (+ 8 ri + 4 h).
template <int P>
__device__ __forceinline__ void transport_hidden(const Lex &g, const void *thin, const void *in, const SiteGeo &x,
                                                 bool valid, int h, __bf16 *col, int koff) {
    float tr[3][4], ti[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) tr[a][q] = ti[a][q] = 0.f;
    if (P < 9 && valid) {
        int nb = x.s;
        cx<float> w[9];
        if constexpr (P >= 1 && P <= 4) {
            nb = hop<P - 1>(g, x, +1);
            load_link<P - 1>(thin, x.s, w);
        } else if constexpr (P >= 5 && P <= 8) {
            nb = hop<P - 5>(g, x, -1);
            load_link<P - 5>(thin, nb, w);
        }
        u2v v[6];
        load_act_half(in, nb, h, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cx<float> vb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) vb[c] = {half_chan(v[2 * c], q), half_chan(v[2 * c + 1], q)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cx<float> t = {0.f, 0.f};
                if constexpr (P == 0) {
                    t = vb[a];
                } else if constexpr (P <= 4) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) cmac(t, w[3 * a + c], vb[c]);
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) cmac(t, cconj(w[3 * c + a]), vb[c]);  // conj(U[c][a]) v[c]
                }
                tr[a][q] = t.re;
                ti[a][q] = t.im;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const b4v r = {(__bf16)tr[a][0], (__bf16)tr[a][1], (__bf16)tr[a][2], (__bf16)tr[a][3]};
        const b4v i = {(__bf16)ti[a][0], (__bf16)ti[a][1], (__bf16)ti[a][2], (__bf16)ti[a][3]};
        *(b4v *)(col + a * BT_LD + koff + 4 * h) = r;
        *(b4v *)(col + a * BT_LD + koff + 8 + 4 * h) = i;
    }
}

// Path P of the one-channel even-site input (FP32 public spinor) at site x;
// lane half h writes the re (h = 0) or im (h = 1) parts at K = 2P + h.
template <int P>
__device__ __forceinline__ void transport_even_path(const Lex &g, const void *thin, const float *in, const SiteGeo &x,
                                                    bool valid, int h, __bf16 *col) {
    cx<float> t[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
    // the input lives on even sites: path 0 needs x even, the hops x odd
    const bool live = valid && (P == 0 ? x.par == 0 : x.par == 1);
    if (live) {
        const int vh = g.V / 2;
        if constexpr (P == 0) {
            Spinor<F32>{const_cast<float *>(in), vh}.load(x.s >> 1, t);
        } else {
            cx<float> w[9], v[3];
            int nb;
            if constexpr (P <= 4) {
                nb = hop<P - 1>(g, x, +1);
                load_link<P - 1>(thin, x.s, w);
            } else {
                nb = hop<P - 5>(g, x, -1);
                load_link<P - 5>(thin, nb, w);
            }
            Spinor<F32>{const_cast<float *>(in), vh}.load(nb >> 1, v);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (P <= 4) {
                        cmac(t[a], w[3 * a + c], v[c]);
                    } else {
                        cmac(t[a], cconj(w[3 * c + a]), v[c]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) col[a * BT_LD + 2 * P + h] = (__bf16)(h ? t[a].im : t[a].re);
}

// All nine paths of the even-site input, zeros in the padding K = 18..31.
__device__ __forceinline__ void transport_even(const Lex &g, const void *thin, const float *in, const SiteGeo &x,
                                               bool valid, int h, __bf16 *col) {
    transport_even_path<0>(g, thin, in, x, valid, h, col);
    transport_even_path<1>(g, thin, in, x, valid, h, col);
    transport_even_path<2>(g, thin, in, x, valid, h, col);
    transport_even_path<3>(g, thin, in, x, valid, h, col);
    transport_even_path<4>(g, thin, in, x, valid, h, col);
    transport_even_path<5>(g, thin, in, x, valid, h, col);
    transport_even_path<6>(g, thin, in, x, valid, h, col);
    transport_even_path<7>(g, thin, in, x, valid, h, col);
    transport_even_path<8>(g, thin, in, x, valid, h, col);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 7; ++j) col[a * BT_LD + 18 + 2 * j + h] = (__bf16)0.f;
}

// Transported input chunk q (K rows 32 q .. 32 q + 31) of the lane pair's site.
template <int INM>
__device__ __forceinline__ void transport_chunk(int q, const Lex &g, const void *thin, const void *in,
                                                const SiteGeo &x, bool valid, int h, __bf16 *col) {
    if constexpr (INM == IO_EVEN) {
        transport_even(g, thin, (const float *)in, x, valid, h, col);
    } else {
        switch (q) {
            case 0:
                transport_hidden<0>(g, thin, in, x, valid, h, col, 0);
                transport_hidden<1>(g, thin, in, x, valid, h, col, 16);
                break;
            case 1:
                transport_hidden<2>(g, thin, in, x, valid, h, col, 0);
                transport_hidden<3>(g, thin, in, x, valid, h, col, 16);
                break;
            case 2:
                transport_hidden<4>(g, thin, in, x, valid, h, col, 0);
                transport_hidden<5>(g, thin, in, x, valid, h, col, 16);
                break;
            case 3:
                transport_hidden<6>(g, thin, in, x, valid, h, col, 0);
                transport_hidden<7>(g, thin, in, x, valid, h, col, 16);
                break;
            default:
                transport_hidden<8>(g, thin, in, x, valid, h, col, 0);
                transport_hidden<9>(g, thin, in, x, valid, h, col, 16);
                break;
        }
    }
}

// ------------------------------------------------------------------ layer kernel
// amat: bf16 [16][kp_of(INM)], rows 0..7 Re and 8..15 Im of the output
// channels.  OUTM == IO_FULL: all V sites, output BF16 hidden units;
// IO_EVEN: even sites in checkerboard order, output channel 0 as an FP32
// public spinor.
template <int INM, int OUTM>
__global__ __launch_bounds__(64 * NN_WAVES) void k_nn_layer(Lex g, const void *thin, const void *__restrict__ in,
                                                            void *__restrict__ out, const __bf16 *__restrict__ amat) {
    constexpr int KP = kp_of(INM);
    __shared__ __attribute__((aligned(16))) __bf16 Bt[NN_WAVES][NW_COLS][BT_LD];
    __shared__ float Of[NN_WAVES][NW_SITES][6];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, j = l >> 4;
    const int nsites = OUTM == IO_FULL ? g.V : g.V / 2;
    const int base = (blockIdx.x * NN_WAVES + w) * NW_SITES;
    const int sl = l >> 1, h = l & 1;  // lane pair (site, half)
    const int idx = base + sl;
    const bool valid = idx < nsites;
    const SiteGeo x = site_geo(g, valid ? site_of<OUTM>(g, idx) : 0);
    __bf16 *col = &Bt[w][sl * 3][0];

    f4v acc[6];
#pragma unroll
    for (int cb = 0; cb < 6; ++cb) acc[cb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < KP / 32; ++q) {
        transport_chunk<INM>(q, g, thin, in, x, valid, h, col);
        __syncthreads();
        const b8v a = *(const b8v *)(amat + i * KP + q * 32 + j * 8);
#pragma unroll
        for (int cb = 0; cb < 6; ++cb) {
            const b8v b = *(const b8v *)(&Bt[w][cb * 16 + i][j * 8]);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
        }
        __syncthreads();
    }

    // lane (i, j) holds rows 4j .. 4j + 3 of column cb * 16 + i
    if constexpr (OUTM == IO_FULL) {
        __bf16 *Ot = &Bt[w][0][0];  // staging [32 sites][48] (unit u = 2 colour + ri, channel)
#pragma unroll
        for (int cb = 0; cb < 6; ++cb) {
            const int cl = cb * 16 + i, s = cl / 3, c = cl % 3;
            const b4v v = {(__bf16)acc[cb][0], (__bf16)acc[cb][1], (__bf16)acc[cb][2], (__bf16)acc[cb][3]};
            *(b4v *)(Ot + s * 48 + (2 * c + (j >> 1)) * 8 + (j & 1) * 4) = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = t * 64 + l, s = e & 31, u = e >> 5;
            const int S = base + s;
            if (S < nsites) {
                const u4v val = *(const u4v *)(Ot + s * 48 + u * 8);
                ((u4v *)out)[((size_t)(S >> 6) * 6 + u) * 64 + (S & 63)] = val;
            }
        }
    } else {
#pragma unroll
        for (int cb = 0; cb < 6; ++cb) {
            const int cl = cb * 16 + i, s = cl / 3, c = cl % 3;
            if (j == 0) Of[w][s][2 * c] = acc[cb][0];      // row 0: Re of channel 0
            if (j == 2) Of[w][s][2 * c + 1] = acc[cb][0];  // row 8: Im of channel 0
        }
        __syncthreads();
        if (l < NW_SITES && base + l < nsites) {
            cx<float> v[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = {Of[w][l][2 * c], Of[w][l][2 * c + 1]};
            Spinor<F32>{(float *)out, g.V / 2}.store(base + l, v);
        }
    }
}

// ------------------------------------------------------------------ weight gradient
// Per block: partial[blk][16][KC], KC = 80 (hidden input: column 8 p + b) or
// 16 (even input: column p), C[r][n] = sum over the block's (site, colour) of
// r < 8: Re(g_r conj t_n), r >= 8: Im(g_{r-8} conj t_n).  The upstream gradient
// g has mode GM (IO_FULL: BF16 hidden units on all sites; IO_EVEN: channel 0
// as an FP32 public spinor on even sites); sites are enumerated like the
// layer kernel with OUTM = GM.
template <int INM, int GM>
__global__ __launch_bounds__(64 * NN_WAVES) void k_nn_wgrad(Lex g, const void *thin, const void *__restrict__ in,
                                                            const void *__restrict__ grad, float *__restrict__ partial) {
    constexpr int KP = kp_of(INM);
    constexpr int NQ = KP / 32;  // chunks
    constexpr int KC = INM == IO_EVEN ? 16 : 80;
    __shared__ __attribute__((aligned(16))) __bf16 Bt[NN_WAVES][NW_COLS][BT_LD];
    __shared__ __attribute__((aligned(16))) __bf16 Gt[NN_WAVES][16][GT_LD];
    __shared__ float Red[NN_WAVES][16][KC];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, j = l >> 4;
    const int nsites = GM == IO_FULL ? g.V : g.V / 2;
    const int base = (blockIdx.x * NN_WAVES + w) * NW_SITES;
    const int sl = l >> 1, h = l & 1;
    const int idx = base + sl;
    const bool valid = idx < nsites;
    const SiteGeo x = site_geo(g, valid ? site_of<GM>(g, idx) : 0);
    __bf16 *col = &Bt[w][sl * 3][0];

    // A2 = [[Gr, Gi], [Gi, -Gr]] over m = (site, colour): re block m < 96, im block m >= 96
    for (int e = l; e < 16 * GT_LD; e += 64) (&Gt[w][0][0])[e] = (__bf16)0.f;
    __syncthreads();
    if constexpr (GM == IO_FULL) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int e = t * 64 + l, s = e & 31, u = e >> 5, c = u >> 1, ri = u & 1;
            const int S = base + s, m = s * 3 + c;
            u4v val = {0u, 0u, 0u, 0u};
            if (S < nsites) val = ((const u4v *)grad)[((size_t)(S >> 6) * 6 + u) * 64 + (S & 63)];
            const unsigned wd[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const float v = (a & 1) ? bf_hi(wd[a >> 1]) : bf_lo(wd[a >> 1]);
                if (ri == 0) {
                    Gt[w][a][m] = (__bf16)v;
                    Gt[w][8 + a][NW_COLS + m] = (__bf16)(-v);
                } else {
                    Gt[w][a][NW_COLS + m] = (__bf16)v;
                    Gt[w][8 + a][m] = (__bf16)v;
                }
            }
        }
    } else {
        if (l < NW_SITES) {
            cx<float> v[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
            if (base + l < nsites) Spinor<F32>{(float *)grad, g.V / 2}.load(base + l, v);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int m = l * 3 + c;
                Gt[w][0][m] = (__bf16)v[c].re;
                Gt[w][8][NW_COLS + m] = (__bf16)(-v[c].re);
                Gt[w][0][NW_COLS + m] = (__bf16)v[c].im;
                Gt[w][8][m] = (__bf16)v[c].im;
            }
        }
    }

    f4v acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        transport_chunk<INM>(q, g, thin, in, x, valid, h, col);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < (2 * NW_COLS) / 32; ++ks) {
            const b8v a = *(const b8v *)(&Gt[w][i][ks * 32 + j * 8]);
            const int ri = ks >= 3 ? 1 : 0;
            b8v b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int m = (ks % 3) * 32 + j * 8 + e;  // column of the transported tile
                __bf16 v;
                if constexpr (INM == IO_EVEN) v = i < 9 ? Bt[w][m][2 * i + ri] : (__bf16)0.f;
                else v = Bt[w][m][(i >> 3) * 16 + ri * 8 + (i & 7)];
                b[e] = v;
            }
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) Red[w][j * 4 + r][q * 16 + i] = acc[q][r];
    __syncthreads();
    // sum the block's waves in a fixed order, write the block partial
    for (int e = threadIdx.x; e < 16 * KC; e += blockDim.x) {
        const int r = e / KC, k = e % KC;
        float s = 0.f;
        for (int ww = 0; ww < NN_WAVES; ++ww) s += Red[ww][r][k];
        partial[(size_t)blockIdx.x * 16 * KC + e] = s;
    }
}

// Two-stage fixed-order sum of the block partials.  Stage 1: segment sg of
// the blocks, every entry e of the 16 x KC partial: fold[sg][e].
constexpr int NN_FOLD = 64;  // segments

__global__ __launch_bounds__(256) void k_nn_wgrad_fold(const float *__restrict__ partial, int nblk, int nent,
                                                      float *__restrict__ fold) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x, sg = blockIdx.y;
    if (e >= nent) return;
    const int per = (nblk + NN_FOLD - 1) / NN_FOLD;
    const int b0 = sg * per, b1 = min(nblk, b0 + per);
    float s = 0.f;
    for (int b = b0; b < b1; ++b) s += partial[(size_t)b * nent + e];
    fold[(size_t)sg * nent + e] = s;
}

// Stage 2: grad[p][a][b] (complex double) += sum over the segments (fixed order).
__global__ void k_nn_wgrad_reduce(const float *__restrict__ fold, int inm, int cin, int cout, double *grad) {
    const int KC = inm == IO_EVEN ? 16 : 80;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (a, p, b)
    if (e >= cout * 9 * cin) return;
    const int a = e / (9 * cin), pb = e % (9 * cin), p = pb / cin, b = pb % cin;
    const int n = inm == IO_EVEN ? p : 8 * p + b;
    double re = 0.0, im = 0.0;
    for (int sg = 0; sg < NN_FOLD; ++sg) {
        const float *P = fold + (size_t)sg * 16 * KC;
        re += P[a * KC + n];
        im += P[(8 + a) * KC + n];
    }
    double *gp = grad + 2 * (((size_t)p * cout + a) * cin + b);
    gp[0] += re;
    gp[1] += im;
}

// Real-block bf16 matrix of a layer (transposed = the adjoint layer), in the
// K order of the input mode: hidden k = 16 p + 8 ri + b, even k = 2 p + ri.
__global__ void k_nn_build_amat(const double *__restrict__ W, int cin, int cout, int transposed, int inm,
                                __bf16 *amat) {
    // forward: out channels cout, in channels cin; transposed: out = cin, in = cout
    const int ci = transposed ? cout : cin, co = transposed ? cin : cout;
    const int KP = kp_of(inm);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 16 * KP) return;
    const int r = e / KP, k = e % KP;
    int p, ri, b;
    if (inm == IO_EVEN) {
        p = k >> 1;
        ri = k & 1;
        b = 0;
    } else {
        p = k >> 4;
        ri = (k >> 3) & 1;
        b = k & 7;
    }
    double val = 0.0;
    const int a = r & 7;
    if (p < 9 && a < co && b < ci) {
        double wr, wi;
        if (!transposed) {  // y_a += W_p[a][b] t_{p,b}
            const double *src = W + 2 * (((size_t)p * cout + a) * cin + b);
            wr = src[0];
            wi = src[1];
        } else {  // W'_{p'}[a][b] = conj(W_p[b][a]), p' adjoint of p
            const int pf = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
            const double *src = W + 2 * (((size_t)pf * cout + b) * cin + a);
            wr = src[0];
            wi = -src[1];
        }
        const bool im_row = r >= 8, im_col = ri == 1;
        // [[Wr, -Wi], [Wi, Wr]]
        val = !im_row ? (!im_col ? wr : -wi) : (!im_col ? wi : wr);
    }
    amat[e] = (__bf16)(float)val;
}

// loss pieces on even sites, one sample: partial |out - v|^2 and G(out) = scale (out - v)
__global__ __launch_bounds__(256) void k_nn_loss_grad(Spinor<F32> out, Spinor<F32> v, const double *__restrict__ scale,
                                                      Spinor<F32> gout, double *__restrict__ part) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double dd = 0.0;
    if (h < v.vh) {
        cx<float> o[3], t[3], gg[3];
        out.load(h, o);
        v.load(h, t);
        const float sc = (float)scale[0];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float dr = o[c].re - t[c].re, di = o[c].im - t[c].im;
            dd += (double)dr * dr + (double)di * di;
            gg[c] = {sc * dr, sc * di};
        }
        gout.store(h, gg);
    }
    __shared__ double red[4];
    for (int off = 32; off >= 1; off >>= 1) dd += __shfl_xor(dd, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dd;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_nn_norm2(Spinor<F32> v, double *__restrict__ part) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double dd = 0.0;
    if (h < v.vh) {
        cx<float> t[3];
        v.load(h, t);
#pragma unroll
        for (int c = 0; c < 3; ++c) dd += (double)t[c].re * t[c].re + (double)t[c].im * t[c].im;
    }
    __shared__ double red[4];
    for (int off = 32; off >= 1; off >>= 1) dd += __shfl_xor(dd, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dd;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// s[0] = sum of partials (fixed order); mode 0: scale = 2 / (B |v|^2) into s[1], keep |v|^2 in s[2]
// mode 1: loss += sum / (|v|^2 B)
__global__ void k_nn_scalar(const double *__restrict__ part, int n, double *s, int mode, int batch) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        if (mode == 0) {
            s[2] = t;
            s[1] = t > 0.0 ? 2.0 / ((double)batch * t) : 0.0;
        } else {
            s[3] += s[2] > 0.0 ? t / (s[2] * (double)batch) : 0.0;
        }
    }
}

// Adam on the real and imaginary parts of every weight (FP64 master copy).
__global__ void k_nn_adam(double *w, double *m, double *v, const double *g, int n, double lr, double b1, double b2,
                          double eps, int step) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    m[i] = b1 * m[i] + (1.0 - b1) * gi;
    v[i] = b2 * v[i] + (1.0 - b2) * gi * gi;
    const double mh = m[i] / (1.0 - pow(b1, (double)step));
    const double vh = v[i] / (1.0 - pow(b2, (double)step));
    w[i] -= lr * mh / (sqrt(vh) + eps);
}

// ------------------------------------------------------------------ dispatch
static Lex lex_of(const NnGeom &G) { return Lex{{G.L[0], G.L[1], G.L[2], G.L[3]}, G.V}; }

static int grid_blocks(int nsites) { return (nsites + NB_SITES - 1) / NB_SITES; }

bool nn_channels_supported(int c) { return c >= 1 && c <= 8; }

size_t nn_act_bytes(const NnGeom &G) { return (size_t)((G.V + 63) / 64) * 6 * 1024; }

size_t nn_amat_elems(int inm) { return (size_t)16 * kp_of(inm); }

size_t nn_wgrad_partial_floats(const NnGeom &G) { return ((size_t)grid_blocks(G.V) + NN_FOLD) * 16 * 80; }

size_t nn_thin_bytes(const NnGeom &G) { return (size_t)((G.V + 63) / 64) * 9 * 1024 + 256; }

int nn_layer(const NnGeom &G, const void *thin, int inm, int outm, const void *in, void *out, const void *amat,
             hipStream_t s) {
    const Lex L = lex_of(G);
    const dim3 grid(grid_blocks(outm == IO_FULL ? G.V : G.V / 2)), block(64 * NN_WAVES);
    const __bf16 *A = (const __bf16 *)amat;
    if (inm == IO_FULL && outm == IO_FULL)
        hipLaunchKernelGGL((k_nn_layer<IO_FULL, IO_FULL>), grid, block, 0, s, L, thin, in, out, A);
    else if (inm == IO_EVEN && outm == IO_FULL)
        hipLaunchKernelGGL((k_nn_layer<IO_EVEN, IO_FULL>), grid, block, 0, s, L, thin, in, out, A);
    else if (inm == IO_FULL && outm == IO_EVEN)
        hipLaunchKernelGGL((k_nn_layer<IO_FULL, IO_EVEN>), grid, block, 0, s, L, thin, in, out, A);
    else
        hipLaunchKernelGGL((k_nn_layer<IO_EVEN, IO_EVEN>), grid, block, 0, s, L, thin, in, out, A);
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

int nn_wgrad(const NnGeom &G, const void *thin, int cin, int cout, int inm, int gm, const void *in, const void *grad,
             float *partial, double *gacc, hipStream_t s) {
    const Lex L = lex_of(G);
    const int nblk = grid_blocks(gm == IO_FULL ? G.V : G.V / 2);
    const dim3 grid(nblk), block(64 * NN_WAVES);
    if (inm == IO_FULL && gm == IO_FULL)
        hipLaunchKernelGGL((k_nn_wgrad<IO_FULL, IO_FULL>), grid, block, 0, s, L, thin, in, grad, partial);
    else if (inm == IO_EVEN && gm == IO_FULL)
        hipLaunchKernelGGL((k_nn_wgrad<IO_EVEN, IO_FULL>), grid, block, 0, s, L, thin, in, grad, partial);
    else if (inm == IO_FULL && gm == IO_EVEN)
        hipLaunchKernelGGL((k_nn_wgrad<IO_FULL, IO_EVEN>), grid, block, 0, s, L, thin, in, grad, partial);
    else
        hipLaunchKernelGGL((k_nn_wgrad<IO_EVEN, IO_EVEN>), grid, block, 0, s, L, thin, in, grad, partial);
    const int nent = 16 * (inm == IO_EVEN ? 16 : 80);
    float *fold = partial + (size_t)grid_blocks(G.V) * 16 * 80;
    hipLaunchKernelGGL(k_nn_wgrad_fold, dim3((nent + 255) / 256, NN_FOLD), dim3(256), 0, s, partial, nblk, nent, fold);
    const int n = cout * 9 * cin;
    hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3((n + 127) / 128), dim3(128), 0, s, fold, inm, cin, cout, gacc);
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

void nn_build_amat(const double *W, int cin, int cout, bool transposed, int inm, void *amat, hipStream_t s) {
    const int n = (int)nn_amat_elems(inm);
    hipLaunchKernelGGL(k_nn_build_amat, dim3((n + 255) / 256), dim3(256), 0, s, W, cin, cout, (int)transposed, inm,
                       (__bf16 *)amat);
}

int nn_pack_thin(const NnGeom &G, const double *U, void *dst, hipStream_t s) {
    const Lex L = lex_of(G);
    unsigned *bad = (unsigned *)((char *)dst + nn_thin_bytes(G) - 256);
    HISQ_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_pack_thin, dim3((G.V + 255) / 256, 4), dim3(256), 0, s, L, U, dst, bad);
    HISQ_HIP_CHECK(hipGetLastError());
    unsigned hb = 0;
    HISQ_HIP_CHECK(hipMemcpyAsync(&hb, bad, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    if (hb) {
        set_error("thin links: an entry is not finite or exceeds the FP16 range (|x| >= 32768)");
        return HISQ_ERR_INVALID;
    }
    return HISQ_OK;
}

void nn_loss_grad(int vh, const float *out, const float *v, float *gout, double *part, double *scal, int batch,
                  hipStream_t s) {
    const int nb = (vh + 255) / 256;
    Spinor<F32> O{const_cast<float *>(out), vh}, T{const_cast<float *>(v), vh}, Gg{gout, vh};
    hipLaunchKernelGGL(k_nn_norm2, dim3(nb), dim3(256), 0, s, T, part);
    hipLaunchKernelGGL(k_nn_scalar, dim3(1), dim3(256), 0, s, part, nb, scal, 0, batch);
    hipLaunchKernelGGL(k_nn_loss_grad, dim3(nb), dim3(256), 0, s, O, T, scal + 1, Gg, part);
    hipLaunchKernelGGL(k_nn_scalar, dim3(1), dim3(256), 0, s, part, nb, scal, 1, batch);
}

void nn_adam(double *w, double *m, double *v, const double *g, int n, double lr, int step, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, m, v, g, n, lr, 0.9, 0.999, 1e-8, step);
}

}  // namespace hisq
