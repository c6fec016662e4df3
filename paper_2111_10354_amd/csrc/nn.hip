// Gauge-covariant preconditioner network: forward, backward and Adam kernels.
//
// Layer with CIN -> COUT complex channels on the full lattice:
//   y_a(x) = sum_b [ W0_ab psi_b(x) + sum_mu ( Wf_mu,ab U_mu(x) psi_b(x+mu)
//                                            + Wb_mu,ab U_mu(x-mu)^+ psi_b(x-mu) ) ]
// (linear, gauge covariant; the L-CNN construction of Favoni et al. 2022 used
// as a solver preconditioner as in Lehner and Wettig 2023).
//
// One wavefront handles 16 sites = 48 (site, colour) columns:
//  1. its four lane groups compute the 9 transported inputs T_p psi_b of every
//     input channel in FP32 (lane group j owns the paths p = j, j+4, j+8) and
//     write them to LDS as BF16;
//  2. the channel mixing is a real GEMM  [Re y; Im y] (16 x 48) =
//     [[Wr, -Wi], [Wi, Wr]] (16 x 2K) x [Re T; Im T] (2K x 48), K = 9 CIN, run
//     on v_mfma_f32_16x16x32_bf16 with FP32 accumulation;
//  3. the 16 x 48 result is staged in LDS and written as FP32 activations.
// The transposed layer needed by back-propagation is the same kernel with
// weights W'_{p'} = W_p^H, p' the adjoint hop (forward and backward swap).
// Weight gradients G(W_p[a][b]) = sum_{x,c} g_a(x)_c conj((T_p psi_b)(x)_c) use
// the same MFMA with the (site, colour) dimension as the reduction, per-block
// partials and a fixed-order final sum (deterministic).

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nn_internal.h"

namespace hisq {

typedef __bf16 b8v __attribute__((ext_vector_type(8)));

constexpr int NN_SITES = 16;             // sites per wavefront
constexpr int NN_COLS = NN_SITES * 3;    // 48 MFMA columns
constexpr int NN_WAVES = 2;              // wavefronts per block

__host__ __device__ constexpr int kpad(int cin) { return ((2 * 9 * cin + 31) / 32) * 32; }

// ------------------------------------------------------------------ geometry (full lattice)
struct Lex {
    int L[4];
    int V;
    __device__ __forceinline__ void coords(int s, int c[4]) const {
        c[0] = s % L[0];
        s /= L[0];
        c[1] = s % L[1];
        s /= L[1];
        c[2] = s % L[2];
        c[3] = s / L[2];
    }
    __device__ __forceinline__ int lex(const int c[4]) const { return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3])); }
    __device__ __forceinline__ int hop(int s, int mu, int d) const {
        int c[4];
        coords(s, c);
        c[mu] = wrap(c[mu] + d, L[mu]);
        return lex(c);
    }
    __device__ __forceinline__ int parity(int s) const {
        int c[4];
        coords(s, c);
        return (c[0] + c[1] + c[2] + c[3]) & 1;
    }
};

// Thin links (FP32): per site 4 links = 2 groups of 2 links, tiled like the
// Dslash links: unit e of group gi of site s at u4v index ((s/64)*2 + gi)*9*64 + e*64 + s%64.
__device__ __forceinline__ void load_thin(const void *base, int s, int mu, cx<float> w[9]) {
    const u4v *b = (const u4v *)base + ((size_t)((s >> 6) * 2 + (mu >> 1)) * 9) * 64 + (s & 63);
    const int sl = mu & 1;
    // complex entries 9 sl .. 9 sl + 8 of the 18 in the group record
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int idx = 9 * sl + c;  // complex index in the 144-byte record
        const u4v raw = b[(idx >> 1) * 64];
        const f4v u = __builtin_bit_cast(f4v, raw);
        w[c] = (idx & 1) ? cx<float>{u.z, u.w} : cx<float>{u.x, u.y};
    }
}

__global__ __launch_bounds__(256) void k_pack_thin(Lex g, const double *__restrict__ U, void *dst) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= g.V) return;
    char *rec = (char *)dst + ((size_t)((s >> 6) * 2 + (mu >> 1)) * 9) * 1024 + (size_t)(s & 63) * 16;
    const double *src = U + ((size_t)s * 4 + mu) * 18;
    for (int c = 0; c < 9; ++c) {
        const int off = ((mu & 1) * 9 + c) * 8;
        *(f2v *)(rec + (size_t)(off >> 4) * 1024 + (off & 15)) = f2v{(float)src[2 * c], (float)src[2 * c + 1]};
    }
}

// ------------------------------------------------------------------ activations
// Input / output modes of a layer:
//   IO_FULL: C channels on all V sites, channel b = FP32 spinor buffer b of a
//            stack with vh = V (lexicographic site order);
//   IO_EVEN: one channel on even sites only, an FP32 spinor of the public
//            layout (checkerboard order); odd sites read as zero.
enum { IO_FULL = 0, IO_EVEN = 1 };

template <int MODE>
__device__ __forceinline__ void load_act(const Lex &g, const float *buf, int b, int s, cx<float> v[3]) {
    if constexpr (MODE == IO_FULL) {
        Spinor<F32>{const_cast<float *>(buf), g.V}.rhs(b).load(s, v);
    } else {
        if (g.parity(s) == 0) {
            Spinor<F32>{const_cast<float *>(buf), g.V / 2}.load(s >> 1, v);
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = {0.f, 0.f};
        }
    }
}

// Transported inputs of 16 sites into LDS: Bt[col][k], col = site*3 + colour,
// k = p*CIN + b (real part) and K + p*CIN + b (imaginary part).
template <int CIN, int INM>
__device__ __forceinline__ void transport_tile(const Lex &g, const void *thin, const float *in, int site, bool valid,
                                               int j, __bf16 (*Bt)[kpad(CIN) + 8]) {
    constexpr int K = 9 * CIN;
    const int s = threadIdx.x & 15;
    for (int p = j; p < 9; p += 4) {
        cx<float> w[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) w[c] = {0.f, 0.f};  // tail sites multiply zeros, never garbage
        int nb = site;
        bool adj = false;
        if (valid && p != 0) {
            const int mu = (p - 1) & 3;
            if (p <= 4) {
                nb = g.hop(site, mu, +1);
                load_thin(thin, site, mu, w);
            } else {
                nb = g.hop(site, mu, -1);
                load_thin(thin, nb, mu, w);
                adj = true;
            }
        }
        for (int b = 0; b < CIN; ++b) {
            cx<float> v[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}}, t[3];
            if (valid) load_act<INM>(g, in, b, nb, v);
            if (p == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) t[c] = v[c];
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    t[a] = {0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (adj) {  // conj(U[c][a]) v[c]
                            const cx<float> u = w[3 * c + a];
                            t[a].re += u.re * v[c].re + u.im * v[c].im;
                            t[a].im += u.re * v[c].im - u.im * v[c].re;
                        } else {
                            cmac(t[a], w[3 * a + c], v[c]);
                        }
                    }
                }
            }
            const int k = p * CIN + b;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                Bt[s * 3 + c][k] = (__bf16)t[c].re;
                Bt[s * 3 + c][K + k] = (__bf16)t[c].im;
            }
        }
    }
}

// ------------------------------------------------------------------ layer kernel
// amat: bf16 [16][kpad(CIN)] real-block weight matrix (rows 0..7 Re, 8..15 Im of
// the output channels).  Sites: OUTM == IO_FULL -> all V sites in lex order;
// IO_EVEN -> even sites in checkerboard order (output to a public FP32 spinor).
template <int CIN, int COUT, int INM, int OUTM>
__global__ __launch_bounds__(64 * NN_WAVES) void k_nn_layer(Lex g, const void *thin, const float *__restrict__ in,
                                                            float *__restrict__ out, const __bf16 *__restrict__ amat) {
    constexpr int KP = kpad(CIN);
    __shared__ __attribute__((aligned(16))) __bf16 Bt[NN_WAVES][NN_COLS][KP + 8];
    __shared__ float Ct[NN_WAVES][16][NN_COLS + 4];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, j = l >> 4;
    const int nsites = OUTM == IO_FULL ? g.V : g.V / 2;
    const int idx = (blockIdx.x * NN_WAVES + w) * NN_SITES + i;
    const bool valid = idx < nsites;
    int site = idx;
    if (OUTM == IO_EVEN && valid) {  // checkerboard index of an even site -> lex
        const int lxh = g.L[0] >> 1;
        const int xh = idx % lxh, r = idx / lxh;
        const int y = r % g.L[1], z = (r / g.L[1]) % g.L[2], t = r / (g.L[1] * g.L[2]);
        site = 2 * xh + ((y + z + t) & 1) + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
    }
    // zero the K padding rows of this wave's tile
    for (int e = l; e < NN_COLS * (KP - 18 * CIN); e += 64) {
        const int col = e % NN_COLS, k = 18 * CIN + e / NN_COLS;
        Bt[w][col][k] = (__bf16)0.f;
    }
    transport_tile<CIN, INM>(g, thin, in, site, valid, j, Bt[w]);
    __syncthreads();

    f4v acc[3] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
        const b8v a = *(const b8v *)(amat + i * KP + ks * 32 + j * 8);
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
            const b8v b = *(const b8v *)(&Bt[w][cb * 16 + i][ks * 32 + j * 8]);
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) Ct[w][j * 4 + q][cb * 16 + i] = acc[cb][q];
    __syncthreads();

    // write: lane handles (channel a, site s) pairs
    for (int e = l; e < COUT * NN_SITES; e += 64) {
        const int a = e / NN_SITES, s = e % NN_SITES;
        const int oidx = (blockIdx.x * NN_WAVES + w) * NN_SITES + s;
        if (oidx >= nsites) continue;
        cx<float> v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = {Ct[w][a][s * 3 + c], Ct[w][8 + a][s * 3 + c]};
        if constexpr (OUTM == IO_FULL) Spinor<F32>{out, g.V}.rhs(a).store(oidx, v);
        else Spinor<F32>{out, g.V / 2}.store(oidx, v);
    }
}

// ------------------------------------------------------------------ weight gradient
// partial[blk][16][KC] (KC = 16 * ceil(9 CIN / 16)): C[r][k] = sum over this
// block's (site, colour) of  r < 8: Re(g_r conj t_k),  r >= 8: Im(g_{r-8} conj t_k).
// The upstream gradient uses mode GM (IO_FULL: COUT channels on all sites, or
// IO_EVEN: one channel on even sites); sites are enumerated like k_nn_layer with OUTM = GM.
template <int CIN, int COUT, int INM, int GM>
__global__ __launch_bounds__(64 * NN_WAVES) void k_nn_wgrad(Lex g, const void *thin, const float *__restrict__ in,
                                                            const float *__restrict__ grad, float *__restrict__ partial) {
    constexpr int K = 9 * CIN;
    constexpr int KP = kpad(CIN);
    constexpr int NCB = (K + 15) / 16;
    __shared__ __attribute__((aligned(16))) __bf16 Bt[NN_WAVES][NN_COLS][KP + 8];
    __shared__ __attribute__((aligned(16))) __bf16 Gt[NN_WAVES][16][2 * NN_COLS + 8];  // A2 rows, m = 0..95
    __shared__ float Red[NN_WAVES][16][16 * NCB];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, j = l >> 4;
    const int nsites = GM == IO_FULL ? g.V : g.V / 2;
    const int idx = (blockIdx.x * NN_WAVES + w) * NN_SITES + i;
    const bool valid = idx < nsites;
    int site = idx;
    if (GM == IO_EVEN && valid) {
        const int lxh = g.L[0] >> 1;
        const int xh = idx % lxh, r = idx / lxh;
        const int y = r % g.L[1], z = (r / g.L[1]) % g.L[2], t = r / (g.L[1] * g.L[2]);
        site = 2 * xh + ((y + z + t) & 1) + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
    }
    transport_tile<CIN, INM>(g, thin, in, site, valid, j, Bt[w]);
    // A2 = [[Gr, Gi], [Gi, -Gr]] over m = (site, colour) (Re block then Im block)
    for (int e = l; e < 8 * NN_SITES; e += 64) {
        const int a = e / NN_SITES, s = e % NN_SITES;
        const int gidx = (blockIdx.x * NN_WAVES + w) * NN_SITES + s;
        cx<float> v[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
        if (a < COUT && gidx < nsites) {
            if constexpr (GM == IO_FULL) Spinor<F32>{const_cast<float *>(grad), g.V}.rhs(a).load(gidx, v);
            else Spinor<F32>{const_cast<float *>(grad), g.V / 2}.load(gidx, v);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int m = s * 3 + c;
            Gt[w][a][m] = (__bf16)v[c].re;
            Gt[w][a][NN_COLS + m] = (__bf16)v[c].im;
            Gt[w][8 + a][m] = (__bf16)v[c].im;
            Gt[w][8 + a][NN_COLS + m] = (__bf16)(-v[c].re);
        }
    }
    __syncthreads();

    f4v acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = f4v{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < (2 * NN_COLS) / 32; ++ks) {
        const b8v a = *(const b8v *)(&Gt[w][i][ks * 32 + j * 8]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int k = cb * 16 + i;
            b8v b;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int m = ks * 32 + j * 8 + q;
                __bf16 v = (__bf16)0.f;
                if (k < K) v = m < NN_COLS ? Bt[w][m][k] : Bt[w][m - NN_COLS][K + k];
                b[q] = v;
            }
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) Red[w][j * 4 + q][cb * 16 + i] = acc[cb][q];
    __syncthreads();
    // sum the block's waves in a fixed order, write the block partial
    for (int e = threadIdx.x; e < 16 * 16 * NCB; e += blockDim.x) {
        const int r = e / (16 * NCB), k = e % (16 * NCB);
        float s = 0.f;
        for (int ww = 0; ww < NN_WAVES; ++ww) s += Red[ww][r][k];
        partial[(size_t)blockIdx.x * 16 * 16 * NCB + e] = s;
    }
}

// grad[p][a][b] (complex double) += sum over blocks (fixed order) of the partials
__global__ void k_nn_wgrad_reduce(const float *__restrict__ partial, int nblk, int cin, int cout, double *grad) {
    const int K = 9 * cin, KC = 16 * ((K + 15) / 16);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;  // (a, k)
    if (e >= cout * K) return;
    const int a = e / K, k = e % K;
    double re = 0.0, im = 0.0;
    for (int blk = 0; blk < nblk; ++blk) {
        const float *P = partial + (size_t)blk * 16 * KC;
        re += P[a * KC + k];
        im += P[(8 + a) * KC + k];
    }
    const int p = k / cin, b = k % cin;
    double *gp = grad + 2 * (((size_t)p * cout + a) * cin + b);
    gp[0] += re;
    gp[1] += im;
}

// real-block bf16 matrix of a layer (transposed = the adjoint layer)
__global__ void k_nn_build_amat(const double *__restrict__ W, int cin, int cout, int transposed, __bf16 *amat) {
    // forward: out channels cout, in channels cin; transposed: out = cin, in = cout
    const int ci = transposed ? cout : cin, co = transposed ? cin : cout;
    const int K = 9 * ci, KP = ((2 * K + 31) / 32) * 32;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 16 * KP) return;
    const int r = e / KP, k = e % KP;
    double val = 0.0;
    const int a = r & 7;
    if (a < co && k < 2 * K) {
        const int kk = k % K;
        const int p = kk / ci, b = kk % ci;  // y_a += W'_p[a][b] t_{p,b}
        double wr, wi;
        if (!transposed) {
            const double *src = W + 2 * (((size_t)p * cout + a) * cin + b);
            wr = src[0];
            wi = src[1];
        } else {  // W'_{p'}[a][b] = conj(W_p[b][a]), p' adjoint of p
            const int pf = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
            const double *src = W + 2 * (((size_t)pf * cout + b) * cin + a);
            wr = src[0];
            wi = -src[1];
        }
        const bool im_row = r >= 8, im_col = k >= K;
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
template <int CIN, int COUT>
static void layer_launch(const Lex &L, const void *thin, int inm, int outm, const float *in, float *out,
                         const __bf16 *amat, hipStream_t s) {
    const int nsites = outm == IO_FULL ? L.V : L.V / 2;
    const dim3 grid((nsites + NN_SITES * NN_WAVES - 1) / (NN_SITES * NN_WAVES)), block(64 * NN_WAVES);
    if (inm == IO_FULL && outm == IO_FULL)
        hipLaunchKernelGGL((k_nn_layer<CIN, COUT, IO_FULL, IO_FULL>), grid, block, 0, s, L, thin, in, out, amat);
    else if (inm == IO_EVEN && outm == IO_FULL)
        hipLaunchKernelGGL((k_nn_layer<CIN, COUT, IO_EVEN, IO_FULL>), grid, block, 0, s, L, thin, in, out, amat);
    else if (inm == IO_FULL && outm == IO_EVEN)
        hipLaunchKernelGGL((k_nn_layer<CIN, COUT, IO_FULL, IO_EVEN>), grid, block, 0, s, L, thin, in, out, amat);
    else
        hipLaunchKernelGGL((k_nn_layer<CIN, COUT, IO_EVEN, IO_EVEN>), grid, block, 0, s, L, thin, in, out, amat);
}

template <int CIN, int COUT>
static int wgrad_launch(const Lex &L, const void *thin, int inm, int gm, const float *in, const float *grad,
                        float *partial, hipStream_t s) {
    const int nsites = gm == IO_FULL ? L.V : L.V / 2;
    const int nblk = (nsites + NN_SITES * NN_WAVES - 1) / (NN_SITES * NN_WAVES);
    const dim3 grid(nblk), block(64 * NN_WAVES);
    if (inm == IO_FULL && gm == IO_FULL)
        hipLaunchKernelGGL((k_nn_wgrad<CIN, COUT, IO_FULL, IO_FULL>), grid, block, 0, s, L, thin, in, grad, partial);
    else if (inm == IO_EVEN && gm == IO_FULL)
        hipLaunchKernelGGL((k_nn_wgrad<CIN, COUT, IO_EVEN, IO_FULL>), grid, block, 0, s, L, thin, in, grad, partial);
    else if (inm == IO_FULL && gm == IO_EVEN)
        hipLaunchKernelGGL((k_nn_wgrad<CIN, COUT, IO_FULL, IO_EVEN>), grid, block, 0, s, L, thin, in, grad, partial);
    else
        hipLaunchKernelGGL((k_nn_wgrad<CIN, COUT, IO_EVEN, IO_EVEN>), grid, block, 0, s, L, thin, in, grad, partial);
    return nblk;
}

#define NN_CHANNEL_SWITCH(CI, CO, CALL)                                   \
    switch ((CI) * 100 + (CO)) {                                          \
        case 101: CALL(1, 1); break;                                      \
        case 102: CALL(1, 2); break;                                      \
        case 104: CALL(1, 4); break;                                      \
        case 108: CALL(1, 8); break;                                      \
        case 201: CALL(2, 1); break;                                      \
        case 202: CALL(2, 2); break;                                      \
        case 401: CALL(4, 1); break;                                      \
        case 404: CALL(4, 4); break;                                      \
        case 801: CALL(8, 1); break;                                      \
        case 808: CALL(8, 8); break;                                      \
        case 204: CALL(2, 4); break;                                      \
        case 402: CALL(4, 2); break;                                      \
        case 408: CALL(4, 8); break;                                      \
        case 804: CALL(8, 4); break;                                      \
        case 208: CALL(2, 8); break;                                      \
        case 802: CALL(8, 2); break;                                      \
        default: return HISQ_ERR_UNSUPPORTED;                            \
    }

bool nn_channels_supported(int c) { return c == 1 || c == 2 || c == 4 || c == 8; }

int nn_layer(const NnGeom &G, const void *thin, int cin, int cout, int inm, int outm, const float *in, float *out,
             const void *amat, hipStream_t s) {
    const Lex L{{G.L[0], G.L[1], G.L[2], G.L[3]}, G.V};
#define CALL_LAYER(A, B) layer_launch<A, B>(L, thin, inm, outm, in, out, (const __bf16 *)amat, s)
    NN_CHANNEL_SWITCH(cin, cout, CALL_LAYER)
#undef CALL_LAYER
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

int nn_wgrad(const NnGeom &G, const void *thin, int cin, int cout, int inm, int gm, const float *in,
             const float *grad, float *partial, double *gacc, hipStream_t s) {
    const Lex L{{G.L[0], G.L[1], G.L[2], G.L[3]}, G.V};
    int nblk = 0;
#define CALL_WG(A, B) nblk = wgrad_launch<A, B>(L, thin, inm, gm, in, grad, partial, s)
    NN_CHANNEL_SWITCH(cin, cout, CALL_WG)
#undef CALL_WG
    const int n = cout * 9 * cin;
    hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3((n + 127) / 128), dim3(128), 0, s, partial, nblk, cin, cout, gacc);
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

size_t nn_wgrad_partial_floats(const NnGeom &G, int cin) {
    const int nblk = (G.V + NN_SITES * NN_WAVES - 1) / (NN_SITES * NN_WAVES);
    return (size_t)nblk * 16 * 16 * ((9 * cin + 15) / 16);
}

size_t nn_amat_elems(int cin) { return (size_t)16 * kpad(cin); }

void nn_build_amat(const double *W, int cin, int cout, bool transposed, void *amat, hipStream_t s) {
    const int ci = transposed ? cout : cin;
    const int n = 16 * kpad(ci);
    hipLaunchKernelGGL(k_nn_build_amat, dim3((n + 255) / 256), dim3(256), 0, s, W, cin, cout, (int)transposed,
                       (__bf16 *)amat);
}

int nn_pack_thin(const NnGeom &G, const double *U, void *dst, hipStream_t s) {
    const Lex L{{G.L[0], G.L[1], G.L[2], G.L[3]}, G.V};
    hipLaunchKernelGGL(k_pack_thin, dim3((G.V + 255) / 256, 4), dim3(256), 0, s, L, U, dst);
    HISQ_HIP_CHECK(hipGetLastError());
    return HISQ_OK;
}

size_t nn_thin_bytes(const NnGeom &G) { return (size_t)((G.V + 63) / 64) * 2 * 9 * 1024; }

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
