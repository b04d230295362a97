// Learned gauge-equivariant preconditioner: forward and backward kernels.
//
// Network (8 channels; d = 0..3 forward hops +mu, d = 4..7 backward hops -mu):
//   T_{+mu} psi(x) = eta_mu(x) s_mu(x)    U_mu(x)        psi(x+mu)
//   T_{-mu} psi(x) = eta_mu(x) s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu)     (T_d^dag = T_{d xor 4})
//   layer 1 : phi1[c](y) = sum_d w1h[c][d] (T_d r)(y) on odd y;  phi1[c](x) = w1s[c] r(x) on even x
//   layer 2 : f_k(x), k < 72 (x even): f_c' = phi1[c'](x), f_{8+8d+c'} = (T_d phi1[c'])(x);
//             phi2[c](x) = sum_k W2[c][k] f_k(x)
//   output  : P(r)(x) = sum_c wout[c] phi2[c](x)
// No weight touches colour, so P commutes with gauge transformations.
//
// Layer 2 is the dense contraction: per even site and colour, 72 complex
// inputs against the 8 x 72 complex W2.  In BF16 mode each lane rounds the
// inputs it gathers to BF16 and feeds them, from registers, to the matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) against a real
// 16 x 160 form of W2; the FP32 mode runs the same contraction on the vector
// ALU.  The hop gathers (links times colour vectors) are bandwidth work on
// the vector ALU.  Feature fields are stored as 24 planes [channel][colour]
// of V/2 sites so that neighbouring lanes read neighbouring words.
// The backward pass runs in FP32 on the vector ALU in both modes; its
// weight gradients are reduced per block into partials that one workgroup
// per parameter sums in a fixed order.
//
// Parameters theta: 656 complex, [w1s(8) | w1h(8x8) | W2(8x72) | wout(8)].
// Gradients are of L = Re sum_x <g(x), P(r)(x)>, stored per parameter as
// dL/dRe + i dL/dIm.
#include <hip/hip_runtime.h>

#include "links.h"
#include "net.h"

namespace stag {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kNetBlock = 256;
constexpr int kL2Sites = 64;       // even sites per block of the forward layer 2
constexpr int kBwdSites = 32;      // even sites per block of the backward even pass
constexpr int kPartE = 8 + kNetC * kNetK + 8;   // w1s, W2, wout partials per block
constexpr int kPartO = kNetC * 8;               // w1h partials per block

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cmulcf(float2 a, float2 b) {  // conj(a) * b
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 caddf(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// out = s * U v (forward hop) or s * U^dag v (backward hop)
__device__ __forceinline__ void transport(const su3<float> &u, float s, bool fwd, const float2 v[3], float2 out[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float2 t = make_float2(0.f, 0.f);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const float2 ue = fwd ? make_float2(u.e[a][b].re, u.e[a][b].im) : make_float2(u.e[b][a].re, -u.e[b][a].im);
            t = caddf(t, cmulf(ue, v[b]));
        }
        out[a] = make_float2(s * t.x, s * t.y);
    }
}

// Link, sign and neighbour eo index of hop d taken at site i (coords x) of parity p
// (LT = float: packed single precision links; BF16Link: the bfloat16 copy).
template <int NROW, typename LT = float>
__device__ __forceinline__ int hop_setup(const Geom &g, const void *links, int p, int i, const int x[4], int d,
                                         su3<float> &u, float &s) {
    const int mu = d & 3;
    if (d < 4) {
        u = LinkLayout<LT, NROW>::load(links, g.Vh, p * 4 + mu, i);
        s = float(fwd_sign(g, x, mu));
        return site_nbr(g, i, x, mu, +1);
    }
    const int j = site_nbr(g, i, x, mu, -1);
    u = LinkLayout<LT, NROW>::load(links, g.Vh, (1 - p) * 4 + mu, j);
    s = float(bwd_sign(g, x, mu));
    return j;
}

// 24 complex (8 channels x 3 colours) of site j of a feature field stored as
// 24 planes [channel][colour][V/2]: lanes of consecutive sites touch
// consecutive 8-byte words of every plane.
__device__ __forceinline__ void load24(const float2 *f, int64_t vh, int j, float2 v[kNetC][3]) {
#pragma unroll
    for (int c = 0; c < kNetC; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) v[c][b] = f[(c * 3 + b) * vh + j];
}
__device__ __forceinline__ void store24(float2 *f, int64_t vh, int j, const float2 v[kNetC][3]) {
#pragma unroll
    for (int c = 0; c < kNetC; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) f[(c * 3 + b) * vh + j] = v[c][b];
}

// Position p (0..39) of the K values that lane group kq feeds the matrix
// cores, as an index kr into the real layer-2 input vector
// (kr = 2 k + {0: re, 1: im}; k < 8 self inputs, k = 8 + 8 d + c' hop inputs),
// or -1 for padding.  Group kq owns hops 2kq and 2kq+1 (positions 0..31) and
// the self inputs of channels 2kq and 2kq+1 (positions 32..35).
__device__ __forceinline__ int mfma_feature(int kq, int p) {
    if (p < 32) {
        const int d = 2 * kq + (p >> 4), cp = (p & 15) >> 1;
        return 2 * (8 + 8 * d + cp) + (p & 1);
    }
    if (p < 36) return 2 * (2 * kq + ((p - 32) >> 1)) + (p & 1);
    return -1;
}

// ---------------------------------------------------------------- weights
// The network is linear and the hops act on colour only, so channel mixing
// commutes with transport.  With v_k = sum_c wout[c] W2[c][k]:
//   P r (x) = s r(x) + sum_d (T_d psi_d)(x),  s = sum_c' v_c' w1s[c'],
//   psi_d(y) = sum_d' A[d][d'] (T_d' r)(y),   A[d][d'] = sum_c' v_{8+8d+c'} w1h[c'][d'],
// an exact rewrite that gathers one colour vector per hop in layer 2.
__global__ void __launch_bounds__(kNetBlock) k_net_prep(const float2 *theta, NetDev *w) {
    __shared__ double vr[kNetK], vi[kNetK];
    const int t = threadIdx.x;
    for (int k = t; k < kNetK; k += kNetBlock) {
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < kNetC; ++c) {
            const float2 wo = theta[kNetWout + c], W = theta[kNetW2 + c * kNetK + k];
            sr += double(wo.x) * W.x - double(wo.y) * W.y;
            si += double(wo.x) * W.y + double(wo.y) * W.x;
        }
        vr[k] = sr;
        vi[k] = si;
    }
    __syncthreads();
    if (t < 64) {
        const int d = t >> 3, dp = t & 7;
        double sr = 0.0, si = 0.0;
        for (int cp = 0; cp < kNetC; ++cp) {
            const float2 h = theta[kNetW1H + 8 * cp + dp];
            const int k = 8 + 8 * d + cp;
            sr += vr[k] * h.x - vi[k] * h.y;
            si += vr[k] * h.y + vi[k] * h.x;
        }
        w->fA[d][dp] = make_float2(float(sr), float(si));
    } else if (t == 64) {
        double sr = 0.0, si = 0.0;
        for (int cp = 0; cp < kNetC; ++cp) {
            const float2 h = theta[kNetW1S + cp];
            sr += vr[cp] * h.x - vi[cp] * h.y;
            si += vr[cp] * h.y + vi[cp] * h.x;
        }
        w->fsig = make_float2(float(sr), float(si));
    }
    for (int j = t; j < kNetC; j += kNetBlock) w->w1s[j] = theta[kNetW1S + j];
    for (int j = t; j < kNetC * 8; j += kNetBlock) w->w1h[j / 8][j % 8] = theta[kNetW1H + j];
    for (int j = t; j < kNetC * kNetK; j += kNetBlock) w->W2[j / kNetK][j % kNetK] = theta[kNetW2 + j];
    for (int j = t; j < kNetC; j += kNetBlock) w->wout[j] = theta[kNetWout + j];
    // real form of W2: out_{2c} = sum_k Re W Re f - Im W Im f,
    // out_{2c+1} = sum_k Im W Re f + Re W Im f; stored in the order the
    // matrix-core B operand is read: B[step c][group kq][column n][8 values]
    for (int j = t; j < 5 * 4 * 16 * 8; j += kNetBlock) {
        const int e = j & 7, n = (j >> 3) & 15, kq = (j >> 7) & 3, c = j >> 9;
        const int kr = mfma_feature(kq, 8 * c + e);
        float v = 0.f;
        if (kr >= 0) {
            const float2 W = theta[kNetW2 + (n >> 1) * kNetK + (kr >> 1)];
            if ((n & 1) == 0) v = (kr & 1) ? -W.y : W.x;
            else v = (kr & 1) ? W.x : W.y;
        }
        reinterpret_cast<__bf16 *>(w->B)[j] = static_cast<__bf16>(v);
    }
}

// ---------------------------------------------------------------- forward layer 1 (odd sites)
template <int NROW>
__global__ void __launch_bounds__(kNetBlock) k_net_l1(NetArgs a) {
    if (a.skip && *a.skip) return;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kNetBlock + threadIdx.x;
    const Geom &g = a.g;
    if (i >= g.Vh) return;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    float2 *phi1 = a.phi1 + so * (size_t)g.Vh * 24;
    int x[4];
    site_coords(g, 1, i, x);
    float2 acc[kNetC][3];
#pragma unroll
    for (int c = 0; c < kNetC; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[c][b] = make_float2(0.f, 0.f);
    for (int d = 0; d < 8; ++d) {
        su3<float> u;
        float s;
        const int j = hop_setup<NROW>(g, a.links, 1, i, x, d, u, s);
        float2 v[3], h[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] = r[(size_t)b * g.Vh + j];
        transport(u, s, d < 4, v, h);
#pragma unroll
        for (int c = 0; c < kNetC; ++c) {
            const float2 w = a.w->w1h[c][d];
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[c][b] = caddf(acc[c][b], cmulf(w, h[b]));
        }
    }
    store24(phi1, g.Vh, i, acc);
}

// ---------------------------------------------------------------- folded form
// odd sites: psi_d = sum_d' A[d][d'] T_d' r, stored as 24 planes [d][colour][V/2]
// (LOWP: links from the bfloat16 copy, psi stored as bfloat16 pairs, so the
// planes take 4 instead of 8 bytes per entry; arithmetic stays FP32).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <bool LOWP>
__device__ __forceinline__ void psi_store(float2 *base, size_t k, float2 v) {
    if constexpr (LOWP) {
        bf16x2 w;
        w[0] = static_cast<__bf16>(v.x);
        w[1] = static_cast<__bf16>(v.y);
        reinterpret_cast<bf16x2 *>(base)[k] = w;
    } else {
        base[k] = v;
    }
}
template <bool LOWP>
__device__ __forceinline__ float2 psi_load(const float2 *base, size_t k) {
    if constexpr (LOWP) {
        const bf16x2 w = reinterpret_cast<const bf16x2 *>(base)[k];
        return make_float2(float(w[0]), float(w[1]));
    } else {
        return base[k];
    }
}

template <int NROW, bool LOWP>
__global__ void __launch_bounds__(kNetBlock) k_net_f1(NetArgs a) {
    __shared__ float2 sA[64];   // the 8 x 8 mixing, read by every lane at the same address
    if (a.skip && *a.skip) return;
    if (threadIdx.x < 64) sA[threadIdx.x] = a.w->fA[threadIdx.x >> 3][threadIdx.x & 7];
    __syncthreads();
    const Geom &g = a.g;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kNetBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    float2 *psi = a.phi1 + so * (size_t)g.Vh * 24;
    int x[4];
    site_coords(g, 1, i, x);
    float2 h[8][3];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        su3<float> u;
        float sg;
        const int j = LOWP ? hop_setup<2, BF16Link>(g, a.links16, 1, i, x, d, u, sg)
                           : hop_setup<NROW>(g, a.links, 1, i, x, d, u, sg);
        float2 v[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] = r[(size_t)b * g.Vh + j];
        transport(u, sg, d < 4, v, h[d]);
    }
#pragma unroll
    for (int d = 0; d < 8; ++d)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int dp = 0; dp < 8; ++dp) acc = caddf(acc, cmulf(sA[8 * d + dp], h[dp][b]));
            psi_store<LOWP>(psi, (size_t)(d * 3 + b) * g.Vh + i, acc);
        }
}

// even sites: P r = s r + sum_d T_d psi_d (one colour vector per hop)
template <int NROW, bool LOWP>
__global__ void __launch_bounds__(kNetBlock) k_net_f2(NetArgs a) {
    if (a.skip && *a.skip) return;
    const Geom &g = a.g;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * kNetBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    const float2 *psi = a.phi1 + so * (size_t)g.Vh * 24;
    float2 *out = a.out + so * a.vstride;
    int x[4];
    site_coords(g, 0, i, x);
    const float2 sig = a.w->fsig;
    float2 acc[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[b] = cmulf(sig, r[(size_t)b * g.Vh + i]);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        su3<float> u;
        float sg;
        const int j = LOWP ? hop_setup<2, BF16Link>(g, a.links16, 0, i, x, d, u, sg)
                           : hop_setup<NROW>(g, a.links, 0, i, x, d, u, sg);
        float2 v[3], h[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] = psi_load<LOWP>(psi, (size_t)(d * 3 + b) * g.Vh + j);
        transport(u, sg, d < 4, v, h);
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[b] = caddf(acc[b], h[b]);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) out[(size_t)b * g.Vh + i] = acc[b];
}

// ---------------------------------------------------------------- forward layer 2 (even sites)
// Block: 4 waves x 16 even sites.  Lane (s16, kq) = (lane % 16, lane / 16)
// builds, for site s16 of its wave, the inputs of hops 2kq and 2kq+1 and the
// self inputs of channels 2kq and 2kq+1.  In BF16 mode these 36 (+4 zero)
// real values per colour are exactly the lane's share of the A operand of
// five v_mfma_f32_16x16x32_bf16 steps (16 sites x 160 K), so the
// contraction with W2 runs from registers; the FP32 mode accumulates the
// same products on the vector ALU and sums the four lane groups.
// Operand layout of v_mfma_f32_16x16x32_bf16: lane l supplies row (A) or
// column (B) l % 16 and the K values 8 (l / 16) .. 8 (l / 16) + 7 of each
// step; it receives D rows 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
template <int NROW, int MIX>
__global__ void __launch_bounds__(kNetBlock) k_net_l2(NetArgs a) {
    if (a.skip && *a.skip) return;
    const Geom &g = a.g;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    const float2 *phi1 = a.phi1 + so * (size_t)g.Vh * 24;
    float2 *out = a.out + so * a.vstride;
    float2 *phi2 = a.phi2 ? a.phi2 + so * (size_t)g.Vh * 24 : nullptr;
    const NetDev *w = a.w;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int s16 = lane & 15, kq = lane >> 4;
    const int site0 = xcd_tile(blockIdx.x, gridDim.x) * kL2Sites + 16 * wv;
    const int i = site0 + s16;
    const bool valid = i < g.Vh;
    int x[4] = {0, 0, 0, 0};
    if (valid) site_coords(g, 0, i, x);

    // self inputs of channels 2kq, 2kq+1
    float2 rv[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) rv[b] = valid ? r[(size_t)b * g.Vh + i] : make_float2(0.f, 0.f);
    float2 fs[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int b = 0; b < 3; ++b) fs[h][b] = cmulf(w->w1s[2 * kq + h], rv[b]);

    if (MIX == kMixBF16) {
        bf16x8 av[3][5];   // [colour][step]
#pragma unroll
        for (int b = 0; b < 3; ++b) {
#pragma unroll
            for (int e = 0; e < 8; ++e) av[b][4][e] = static_cast<__bf16>(0.f);
            av[b][4][0] = static_cast<__bf16>(fs[0][b].x);
            av[b][4][1] = static_cast<__bf16>(fs[0][b].y);
            av[b][4][2] = static_cast<__bf16>(fs[1][b].x);
            av[b][4][3] = static_cast<__bf16>(fs[1][b].y);
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {   // hop d = 2kq + hh fills steps 2hh, 2hh+1
            const int d = 2 * kq + hh;
            float2 v[kNetC][3];
            su3<float> u;
            float sg = 0.f;
            if (valid) {
                const int j = hop_setup<NROW>(g, a.links, 0, i, x, d, u, sg);
                load24(phi1, g.Vh, j, v);
            }
#pragma unroll
            for (int cp = 0; cp < kNetC; ++cp) {
                float2 h[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                if (valid) transport(u, sg, d < 4, v[cp], h);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    av[b][2 * hh + (cp >> 2)][2 * (cp & 3)] = static_cast<__bf16>(h[b].x);
                    av[b][2 * hh + (cp >> 2)][2 * (cp & 3) + 1] = static_cast<__bf16>(h[b].y);
                }
            }
        }
        const bf16x8 *Bw = reinterpret_cast<const bf16x8 *>(w->B);
        bf16x8 bv[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) bv[c] = Bw[(c * 4 + kq) * 16 + s16];
        const int ch = s16 >> 1;   // D column n = s16: channel n / 2, real (n even) or imaginary part
        const float2 wo = w->wout[ch];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            f32x4 d4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 5; ++c) d4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[b][c], bv[c], d4, 0, 0, 0);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const float v = d4[jj];
                float pre = (s16 & 1) ? -wo.y * v : wo.x * v;
                float pim = (s16 & 1) ? wo.x * v : wo.y * v;
#pragma unroll
                for (int off = 8; off >= 1; off >>= 1) {
                    pre += __shfl_xor(pre, off, 16);
                    pim += __shfl_xor(pim, off, 16);
                }
                const int site = site0 + 4 * kq + jj;
                if (site < g.Vh) {
                    if (s16 == 0) out[(size_t)b * g.Vh + site] = make_float2(pre, pim);
                    if (phi2) reinterpret_cast<float *>(&phi2[(size_t)(ch * 3 + b) * g.Vh + site])[s16 & 1] = v;
                }
            }
        }
    } else {
        float2 acc[kNetC][3];   // this lane's share of phi2
#pragma unroll
        for (int c = 0; c < kNetC; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                acc[c][b] = caddf(cmulf(w->W2[c][2 * kq], fs[0][b]), cmulf(w->W2[c][2 * kq + 1], fs[1][b]));
            }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int d = 2 * kq + hh;
            float2 v[kNetC][3];
            su3<float> u;
            float sg = 0.f;
            if (valid) {
                const int j = hop_setup<NROW>(g, a.links, 0, i, x, d, u, sg);
                load24(phi1, g.Vh, j, v);
            }
            for (int cp = 0; cp < kNetC; ++cp) {
                float2 h[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                if (valid) transport(u, sg, d < 4, v[cp], h);
                const int k = 8 + 8 * d + cp;
#pragma unroll
                for (int b = 0; b < 3; ++b)
#pragma unroll
                    for (int c = 0; c < kNetC; ++c) acc[c][b] = caddf(acc[c][b], cmulf(w->W2[c][k], h[b]));
            }
        }
        // sum the four lane groups of each site (lanes s16, s16+16, s16+32, s16+48)
#pragma unroll
        for (int c = 0; c < kNetC; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float2 v = acc[c][b];
                v.x += __shfl_xor(v.x, 16);
                v.y += __shfl_xor(v.y, 16);
                v.x += __shfl_xor(v.x, 32);
                v.y += __shfl_xor(v.y, 32);
                acc[c][b] = v;
            }
        if (valid && kq == 0) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                float2 pv = make_float2(0.f, 0.f);
#pragma unroll
                for (int c = 0; c < kNetC; ++c) pv = caddf(pv, cmulf(w->wout[c], acc[c][b]));
                out[(size_t)b * g.Vh + i] = pv;
            }
            if (phi2) store24(phi2, g.Vh, i, acc);
        }
    }
}

// ---------------------------------------------------------------- loss
// Per sample: e = P - x, g = 2 e / (n_samples ||x||^2), partial of ||e||^2 / (n_samples ||x||^2).
__global__ void __launch_bounds__(kNetBlock) k_net_loss(NetArgs a, const float2 *xs, const double *xnorm2, int n_samples,
                                                     float2 *gout, double *loss_part) {
    __shared__ double red[kNetBlock / kWave];
    const size_t so = blockIdx.y;
    const int64_t n = 3 * (int64_t)a.g.Vh;
    const double nx = xnorm2[so] > 0.0 ? xnorm2[so] : 1.0;
    const float scale = float(2.0 / (n_samples * nx));
    double part = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kNetBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kNetBlock) {
        const float2 p = a.out[so * a.vstride + j];
        const float2 xv = xs[so * a.vstride + j];
        const float2 e = make_float2(p.x - xv.x, p.y - xv.y);
        part += double(e.x) * e.x + double(e.y) * e.y;
        gout[so * a.vstride + j] = make_float2(scale * e.x, scale * e.y);
    }
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) loss_part[so * gridDim.x + blockIdx.x] = s / (n_samples * nx);
}

// ||x_k||^2 per sample: partials [sample][block]
__global__ void __launch_bounds__(kNetBlock) k_net_norm(const float2 *xs, int64_t vstride, double *part) {
    __shared__ double red[kNetBlock / kWave];
    const size_t so = blockIdx.y;
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kNetBlock + threadIdx.x; j < vstride; j += (int64_t)gridDim.x * kNetBlock) {
        const float2 v = xs[so * vstride + j];
        acc += double(v.x) * v.x + double(v.y) * v.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[so * gridDim.x + blockIdx.x] = s;
}

// out[row] = sum of part[row][0 .. ncol), one workgroup per row, fixed order
__global__ void __launch_bounds__(kNetBlock) k_net_rowsum(const double *part, int ncol, double *out) {
    __shared__ double red[kNetBlock / kWave];
    double acc = 0.0;
    for (int k = threadIdx.x; k < ncol; k += kNetBlock) acc += part[(size_t)blockIdx.x * ncol + k];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ---------------------------------------------------------------- backward, even sites
// Block: 32 even sites x 8 threads; thread (sl, q) rebuilds the inputs of hop
// d = q of its site; q = 0 also handles the self inputs, g2 = conj(wout) g,
// and the per-site gradients of wout and w1s.  Then the block reduces the
// W2 gradient sum_{sites, colours} g2[c] conj(f_k) from LDS.
template <int NROW>
__global__ void __launch_bounds__(kNetBlock) k_net_bwd_even(NetArgs a, const float2 *gin, float2 *g2out, float2 *partE) {
    constexpr int S = kBwdSites;
    __shared__ float2 Fs[S * 3 * kNetK];          // f[site][colour][k]
    __shared__ float2 G2s[S * 3 * kNetC];         // g2[site][colour][c]
    __shared__ float2 red_wout[S][kNetC], red_w1s[S][kNetC];
    const Geom &g = a.g;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    const float2 *phi1 = a.phi1 + so * (size_t)g.Vh * 24;
    const float2 *phi2 = a.phi2 + so * (size_t)g.Vh * 24;
    const float2 *gg = gin + so * a.vstride;
    float2 *g2o = g2out + so * (size_t)g.Vh * 24;
    const NetDev *w = a.w;
    const int t = threadIdx.x, sl = t >> 3, q = t & 7;
    const int i = blockIdx.x * S + sl;
    const bool valid = i < g.Vh;
    int x[4] = {0, 0, 0, 0};
    if (valid) site_coords(g, 0, i, x);

    {   // hop inputs of hop d = q
        const int d = q;
        float2 v[kNetC][3];
        su3<float> u;
        float s = 0.f;
        if (valid) {
            const int j = hop_setup<NROW>(g, a.links, 0, i, x, d, u, s);
            load24(phi1, g.Vh, j, v);
        }
        for (int cp = 0; cp < kNetC; ++cp) {
            float2 h[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
            if (valid) transport(u, s, d < 4, v[cp], h);
            for (int b = 0; b < 3; ++b) Fs[(sl * 3 + b) * kNetK + 8 + 8 * d + cp] = h[b];
        }
    }
    if (q == 0) {
        float2 rv[3], gv[3], p2[kNetC][3], g2[kNetC][3];
        for (int b = 0; b < 3; ++b) {
            rv[b] = valid ? r[(size_t)b * g.Vh + i] : make_float2(0.f, 0.f);
            gv[b] = valid ? gg[(size_t)b * g.Vh + i] : make_float2(0.f, 0.f);
        }
        if (valid) load24(phi2, g.Vh, i, p2);
        for (int c = 0; c < kNetC; ++c) {
            float2 gw = make_float2(0.f, 0.f);
            for (int b = 0; b < 3; ++b) {
                if (!valid) p2[c][b] = make_float2(0.f, 0.f);
                g2[c][b] = cmulcf(w->wout[c], gv[b]);          // conj(wout) g
                gw = caddf(gw, cmulcf(p2[c][b], gv[b]));       // g conj(phi2)
                G2s[(sl * 3 + b) * kNetC + c] = g2[c][b];
            }
            red_wout[sl][c] = gw;
        }
        if (valid) store24(g2o, g.Vh, i, g2);
        for (int cp = 0; cp < kNetC; ++cp) {
            float2 gs = make_float2(0.f, 0.f);
            for (int b = 0; b < 3; ++b) {
                const float2 f = cmulf(w->w1s[cp], rv[b]);
                Fs[(sl * 3 + b) * kNetK + cp] = f;
                float2 gf = make_float2(0.f, 0.f);   // adjoint of the self input f_cp
                for (int c = 0; c < kNetC; ++c) gf = caddf(gf, cmulcf(w->W2[c][cp], g2[c][b]));
                gs = caddf(gs, cmulcf(rv[b], gf));   // gf conj(r)
            }
            red_w1s[sl][cp] = gs;
        }
    }
    __syncthreads();
    float2 *pb = partE + ((size_t)so * gridDim.x + blockIdx.x) * kPartE;
    if (t < 2 * kNetC) {
        const int c = t % kNetC;
        float2 sum = make_float2(0.f, 0.f);
        for (int k = 0; k < S; ++k) sum = caddf(sum, t < kNetC ? red_w1s[k][c] : red_wout[k][c]);
        pb[(t < kNetC ? 0 : 8 + kNetC * kNetK) + c] = sum;
    }
    // grad W2[c][k] = sum_{sites, colours} g2[c] conj(f_k)
    for (int e = t; e < kNetC * kNetK; e += kNetBlock) {
        const int c = e / kNetK, k = e % kNetK;
        float2 sum = make_float2(0.f, 0.f);
        for (int row = 0; row < S * 3; ++row) sum = caddf(sum, cmulcf(Fs[row * kNetK + k], G2s[row * kNetC + c]));
        pb[8 + e] = sum;
    }
}

// ---------------------------------------------------------------- backward, odd sites
// gphi1[c'](y) = sum_d T_{d xor 4} [ sum_c conj(W2[c][8+8d+c']) g2[c] ](y): the adjoint of the
// layer-2 hops, gathered at odd y from the 8 even neighbours; then the w1h
// gradient sum_y gphi1[c](y) conj((T_d r)(y)).
template <int NROW>
__global__ void __launch_bounds__(kNetBlock) k_net_bwd_odd(NetArgs a, const float2 *g2in, float2 *partO) {
    __shared__ double red[kNetBlock / kWave];
    const Geom &g = a.g;
    const size_t so = blockIdx.y;
    const float2 *r = a.r + so * a.vstride;
    const float2 *g2 = g2in + so * (size_t)g.Vh * 24;
    const NetDev *w = a.w;
    const int i = blockIdx.x * kNetBlock + threadIdx.x;
    const bool valid = i < g.Vh;
    int x[4] = {0, 0, 0, 0};
    if (valid) site_coords(g, 1, i, x);
    float2 gp[kNetC][3];
    for (int c = 0; c < kNetC; ++c)
        for (int b = 0; b < 3; ++b) gp[c][b] = make_float2(0.f, 0.f);
    if (valid) {
        for (int db = 0; db < 8; ++db) {   // hop db at y reads the even neighbour hit by hop d = db xor 4
            const int d = db ^ 4;
            su3<float> u;
            float s;
            const int j = hop_setup<NROW>(g, a.links, 1, i, x, db, u, s);
            float2 gv[kNetC][3];
            load24(g2, g.Vh, j, gv);
            for (int cp = 0; cp < kNetC; ++cp) {
                float2 gf[3];
                for (int b = 0; b < 3; ++b) {
                    float2 acc = make_float2(0.f, 0.f);
                    for (int c = 0; c < kNetC; ++c) acc = caddf(acc, cmulcf(w->W2[c][8 + 8 * d + cp], gv[c][b]));
                    gf[b] = acc;
                }
                float2 h[3];
                transport(u, s, db < 4, gf, h);
                for (int b = 0; b < 3; ++b) gp[cp][b] = caddf(gp[cp][b], h[b]);
            }
        }
    }
    // w1h gradient of this site, reduced over the block (double, fixed order)
    float2 *pb = partO + ((size_t)so * gridDim.x + blockIdx.x) * kPartO;
    for (int d = 0; d < 8; ++d) {
        float2 hr[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        if (valid) {
            su3<float> u;
            float s;
            const int j = hop_setup<NROW>(g, a.links, 1, i, x, d, u, s);
            float2 v[3];
            for (int b = 0; b < 3; ++b) v[b] = r[(size_t)b * g.Vh + j];
            transport(u, s, d < 4, v, hr);
        }
        for (int c = 0; c < kNetC; ++c) {
            float2 gw = make_float2(0.f, 0.f);
            for (int b = 0; b < 3; ++b) gw = caddf(gw, cmulcf(hr[b], gp[c][b]));   // gphi1 conj(T_d r)
            const double sr = block_sum(double(gw.x), red);
            const double si = block_sum(double(gw.y), red);
            if (threadIdx.x == 0) pb[c * 8 + d] = make_float2(float(sr), float(si));
        }
    }
}

// ---------------------------------------------------------------- gradient reduction and Adam
// grad[j] = sum over samples and blocks of the partials, one workgroup per parameter.
__global__ void __launch_bounds__(kNetBlock) k_net_reduce(const float2 *partE, int rowsE, const float2 *partO, int rowsO,
                                                       double2 *grad) {
    __shared__ double red[kNetBlock / kWave];
    const int j = blockIdx.x;
    const float2 *src;
    int stride, off, rows;
    if (j >= kNetW1H && j < kNetW2) {
        src = partO; stride = kPartO; off = j - kNetW1H; rows = rowsO;
    } else {
        src = partE; stride = kPartE; rows = rowsE;
        off = j < kNetW1H ? j : (j < kNetWout ? 8 + (j - kNetW2) : 8 + kNetC * kNetK + (j - kNetWout));
    }
    double sr = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < rows; k += kNetBlock) {
        const float2 v = src[(size_t)k * stride + off];
        sr += v.x;
        si += v.y;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    if (threadIdx.x == 0) grad[j] = make_double2(sr, si);
}

// Adam on the 1312 real parameters (FP32 master weights).
__global__ void __launch_bounds__(kNetBlock) k_net_adam(float2 *theta, float2 *m, float2 *v, const double2 *grad, int t,
                                                     float lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, float(t)), c2 = 1.f - powf(b2, float(t));
    for (int j = threadIdx.x; j < kNetNParam; j += kNetBlock) {
        const float gr = float(grad[j].x), gi = float(grad[j].y);
        float2 mm = m[j], vv = v[j], th = theta[j];
        mm.x = b1 * mm.x + (1.f - b1) * gr;
        mm.y = b1 * mm.y + (1.f - b1) * gi;
        vv.x = b2 * vv.x + (1.f - b2) * gr * gr;
        vv.y = b2 * vv.y + (1.f - b2) * gi * gi;
        th.x -= lr * (mm.x / c1) / (sqrtf(vv.x / c2) + eps);
        th.y -= lr * (mm.y / c1) / (sqrtf(vv.y / c2) + eps);
        m[j] = mm;
        v[j] = vv;
        theta[j] = th;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t net_launch_prep(const float2 *theta, NetDev *w, hipStream_t s) {
    hipLaunchKernelGGL(k_net_prep, dim3(1), dim3(kNetBlock), 0, s, theta, w);
    return hipGetLastError();
}

hipError_t net_launch_forward(const NetArgs &a, int n_samples, int mix, hipStream_t s) {
    const dim3 g1((a.g.Vh + kNetBlock - 1) / kNetBlock, n_samples), g2((a.g.Vh + kL2Sites - 1) / kL2Sites, n_samples);
    if (mix == kMixFoldedBF16) {
        if (!a.links16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_net_f1<2, true>), g1, dim3(kNetBlock), 0, s, a);
        hipLaunchKernelGGL((k_net_f2<2, true>), g1, dim3(kNetBlock), 0, s, a);
        return hipGetLastError();
    }
    if (mix == kMixFolded) {
        if (a.nrow == 1) {
            hipLaunchKernelGGL((k_net_f1<1, false>), g1, dim3(kNetBlock), 0, s, a);
            hipLaunchKernelGGL((k_net_f2<1, false>), g1, dim3(kNetBlock), 0, s, a);
        } else if (a.nrow == 2) {
            hipLaunchKernelGGL((k_net_f1<2, false>), g1, dim3(kNetBlock), 0, s, a);
            hipLaunchKernelGGL((k_net_f2<2, false>), g1, dim3(kNetBlock), 0, s, a);
        } else {
            hipLaunchKernelGGL((k_net_f1<3, false>), g1, dim3(kNetBlock), 0, s, a);
            hipLaunchKernelGGL((k_net_f2<3, false>), g1, dim3(kNetBlock), 0, s, a);
        }
        return hipGetLastError();
    }
    if (a.nrow == 1) {
        hipLaunchKernelGGL(k_net_l1<1>, g1, dim3(kNetBlock), 0, s, a);
        if (mix == kMixBF16) hipLaunchKernelGGL((k_net_l2<1, kMixBF16>), g2, dim3(kNetBlock), 0, s, a);
        else hipLaunchKernelGGL((k_net_l2<1, kMixFP32>), g2, dim3(kNetBlock), 0, s, a);
    } else if (a.nrow == 2) {
        hipLaunchKernelGGL(k_net_l1<2>, g1, dim3(kNetBlock), 0, s, a);
        if (mix == kMixBF16) hipLaunchKernelGGL((k_net_l2<2, kMixBF16>), g2, dim3(kNetBlock), 0, s, a);
        else hipLaunchKernelGGL((k_net_l2<2, kMixFP32>), g2, dim3(kNetBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_net_l1<3>, g1, dim3(kNetBlock), 0, s, a);
        if (mix == kMixBF16) hipLaunchKernelGGL((k_net_l2<3, kMixBF16>), g2, dim3(kNetBlock), 0, s, a);
        else hipLaunchKernelGGL((k_net_l2<3, kMixFP32>), g2, dim3(kNetBlock), 0, s, a);
    }
    return hipGetLastError();
}

int net_blocks_even_bwd(const Geom &g) { return (g.Vh + kBwdSites - 1) / kBwdSites; }
int net_blocks_odd_bwd(const Geom &g) { return (g.Vh + kNetBlock - 1) / kNetBlock; }
int net_part_e() { return kPartE; }
int net_part_o() { return kPartO; }

hipError_t net_launch_backward(const NetArgs &a, int n_samples, const float2 *gin, float2 *g2, float2 *partE,
                               float2 *partO, double2 *grad, hipStream_t s) {
    const dim3 ge(net_blocks_even_bwd(a.g), n_samples), go(net_blocks_odd_bwd(a.g), n_samples);
    if (a.nrow == 1) {
        hipLaunchKernelGGL(k_net_bwd_even<1>, ge, dim3(kNetBlock), 0, s, a, gin, g2, partE);
        hipLaunchKernelGGL(k_net_bwd_odd<1>, go, dim3(kNetBlock), 0, s, a, (const float2 *)g2, partO);
    } else if (a.nrow == 2) {
        hipLaunchKernelGGL(k_net_bwd_even<2>, ge, dim3(kNetBlock), 0, s, a, gin, g2, partE);
        hipLaunchKernelGGL(k_net_bwd_odd<2>, go, dim3(kNetBlock), 0, s, a, (const float2 *)g2, partO);
    } else {
        hipLaunchKernelGGL(k_net_bwd_even<3>, ge, dim3(kNetBlock), 0, s, a, gin, g2, partE);
        hipLaunchKernelGGL(k_net_bwd_odd<3>, go, dim3(kNetBlock), 0, s, a, (const float2 *)g2, partO);
    }
    hipLaunchKernelGGL(k_net_reduce, dim3(kNetNParam), dim3(kNetBlock), 0, s, (const float2 *)partE,
                       int(ge.x * ge.y), (const float2 *)partO, int(go.x * go.y), grad);
    return hipGetLastError();
}

int net_loss_blocks(const Geom &g) {
    const int64_t n = 3 * (int64_t)g.Vh;
    int64_t b = (n + kNetBlock - 1) / kNetBlock;
    return (int)(b > 1024 ? 1024 : b);
}

hipError_t net_launch_loss(const NetArgs &a, int n_samples, const float2 *xs, double *xnorm2, double *norm_part,
                           float2 *gout, double *loss_part, double *loss_rows, hipStream_t s) {
    const int nb = net_loss_blocks(a.g);
    hipLaunchKernelGGL(k_net_norm, dim3(nb, n_samples), dim3(kNetBlock), 0, s, xs, a.vstride, norm_part);
    hipLaunchKernelGGL(k_net_rowsum, dim3(n_samples), dim3(kNetBlock), 0, s, (const double *)norm_part, nb, xnorm2);
    hipLaunchKernelGGL(k_net_loss, dim3(nb, n_samples), dim3(kNetBlock), 0, s, a, xs, (const double *)xnorm2, n_samples,
                       gout, loss_part);
    hipLaunchKernelGGL(k_net_rowsum, dim3(1), dim3(kNetBlock), 0, s, (const double *)loss_part, nb * n_samples,
                       loss_rows);
    return hipGetLastError();
}

hipError_t net_launch_adam(float2 *theta, float2 *m, float2 *v, const double2 *grad, int t, float lr, hipStream_t s) {
    hipLaunchKernelGGL(k_net_adam, dim3(1), dim3(kNetBlock), 0, s, theta, m, v, grad, t, lr);
    return hipGetLastError();
}

}  // namespace stag
