// Packed gauge-link storage: even/odd structure of arrays, element-major
// with the site index fastest, so that 64 consecutive sites of a wave read
// one contiguous 1 KiB (or 512 B) segment per load instruction.  This is the
// coalescing idea of the paper's storage model (Section 5, Figure 2) laid
// out for 16-byte-per-lane loads on CDNA.
//
// Links are grouped by (parity, mu): block (p*4 + mu) holds the links
// U_mu(x) of the V/2 sites x of parity p.  Inside a block:
//   double, 18 reals : 9 planes of double2 (one complex entry e = 3*row+col)
//   double, 12 reals : 6 planes of double2 (rows 0 and 1)
//   float,  18 reals : 4 planes of float4 (entries {0,1},{2,3},{4,5},{6,7})
//                      then 1 plane of float2 (entry 8)
//   float,  12 reals : 3 planes of float4 (entries {0,1},{2,3},{4,5})
// Staggered phases and boundary signs are never folded into the links: a
// sign flip would leave det = -1 and break the third-row rebuild.
//
// Double precision links are read with nontemporal loads: a 32^4 field
// (403-604 MB) cannot stay in the 256 MB Infinity Cache anyway, and keeping
// the streamed links out of the L2 leaves room for the neighbour vectors
// (measured 122 -> 115 us per 18-real half-Dslash at 32^4).  Single
// precision fields (201-302 MB) partly live in the Infinity Cache, and
// nontemporal loads measured slower there, so they use ordinary loads.
#pragma once

#include "common.h"

namespace stag {

template <typename R, int NROW> struct LinkLayout;

template <int NROW> struct LinkLayout<double, NROW> {
    static constexpr int64_t kBytesPerLink = 16 * 3 * NROW;
    __device__ static __forceinline__ su3<double> load(const void *base, int64_t vh, int blk, int64_t i) {
        const double2 *b = static_cast<const double2 *>(base) + (int64_t)blk * (3 * NROW) * vh;
        su3<double> u;
#pragma unroll
        for (int r = 0; r < NROW; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 v = ld_nt(&b[(r * 3 + c) * vh + i]);
                u.e[r][c] = {v.x, v.y};
            }
        if (NROW == 2) su3_rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<double> &u) {
        double2 *b = static_cast<double2 *>(base) + (int64_t)blk * (3 * NROW) * vh;
#pragma unroll
        for (int r = 0; r < NROW; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) b[(r * 3 + c) * vh + i] = make_double2(u.e[r][c].re, u.e[r][c].im);
    }
};

template <> struct LinkLayout<float, 3> {
    static constexpr int64_t kBytesPerLink = 72;
    __device__ static __forceinline__ su3<float> load(const void *base, int64_t vh, int blk, int64_t i) {
        const char *b = static_cast<const char *>(base) + (int64_t)blk * kBytesPerLink * vh;
        const float4 *q = reinterpret_cast<const float4 *>(b);
        const float2 *t = reinterpret_cast<const float2 *>(b + 64 * vh);
        su3<float> u;
        float4 v;
        v = q[0 * vh + i]; u.e[0][0] = {v.x, v.y}; u.e[0][1] = {v.z, v.w};
        v = q[1 * vh + i]; u.e[0][2] = {v.x, v.y}; u.e[1][0] = {v.z, v.w};
        v = q[2 * vh + i]; u.e[1][1] = {v.x, v.y}; u.e[1][2] = {v.z, v.w};
        v = q[3 * vh + i]; u.e[2][0] = {v.x, v.y}; u.e[2][1] = {v.z, v.w};
        const float2 w = t[i];
        u.e[2][2] = {w.x, w.y};
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<float> &u) {
        char *b = static_cast<char *>(base) + (int64_t)blk * kBytesPerLink * vh;
        float4 *q = reinterpret_cast<float4 *>(b);
        float2 *t = reinterpret_cast<float2 *>(b + 64 * vh);
        q[0 * vh + i] = make_float4(u.e[0][0].re, u.e[0][0].im, u.e[0][1].re, u.e[0][1].im);
        q[1 * vh + i] = make_float4(u.e[0][2].re, u.e[0][2].im, u.e[1][0].re, u.e[1][0].im);
        q[2 * vh + i] = make_float4(u.e[1][1].re, u.e[1][1].im, u.e[1][2].re, u.e[1][2].im);
        q[3 * vh + i] = make_float4(u.e[2][0].re, u.e[2][0].im, u.e[2][1].re, u.e[2][1].im);
        t[i] = make_float2(u.e[2][2].re, u.e[2][2].im);
    }
};

template <> struct LinkLayout<float, 2> {
    static constexpr int64_t kBytesPerLink = 48;
    __device__ static __forceinline__ su3<float> load(const void *base, int64_t vh, int blk, int64_t i) {
        const float4 *q = reinterpret_cast<const float4 *>(static_cast<const char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        su3<float> u;
        float4 v;
        v = q[0 * vh + i]; u.e[0][0] = {v.x, v.y}; u.e[0][1] = {v.z, v.w};
        v = q[1 * vh + i]; u.e[0][2] = {v.x, v.y}; u.e[1][0] = {v.z, v.w};
        v = q[2 * vh + i]; u.e[1][1] = {v.x, v.y}; u.e[1][2] = {v.z, v.w};
        su3_rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<float> &u) {
        float4 *q = reinterpret_cast<float4 *>(static_cast<char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        q[0 * vh + i] = make_float4(u.e[0][0].re, u.e[0][0].im, u.e[0][1].re, u.e[0][1].im);
        q[1 * vh + i] = make_float4(u.e[0][2].re, u.e[0][2].im, u.e[1][0].re, u.e[1][0].im);
        q[2 * vh + i] = make_float4(u.e[1][1].re, u.e[1][1].im, u.e[1][2].re, u.e[1][2].im);
    }
};

// Bytes of one packed link field (both parities, 4 directions).
inline int64_t link_field_bytes(bool dbl, int nrow, int64_t vh) {
    const int64_t per = dbl ? 16 * 3 * nrow : (nrow == 3 ? 72 : 48);
    return per * 8 * vh;
}

}  // namespace stag
