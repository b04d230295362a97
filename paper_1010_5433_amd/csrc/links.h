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
//   double,  8 reals : 4 planes of double2 (u01, u02, c, {arg u00, t})
//   float,   8 reals : 2 planes of float4 ({u01, u02}, {c, arg u00, t})
// The 8-real form (NROW = 1) keeps the first row except u00, the smaller in
// modulus of u10 and u20 (c), the phase of u00 and the phase of the other
// one (t, plus 8 when c is u20); the rest follows from unitarity and
// det U = 1 (see rebuild8).  It needs u01, u02 not both zero.
// Staggered phases and boundary signs are never folded into the links: a
// sign flip would leave det = -1 and break the third-row rebuild.
//
// Double precision links are read with nontemporal loads by default: a 32^4
// field (268-604 MB) cannot stay whole in the 256 MB Infinity Cache, and
// keeping the streamed links out of the L2 leaves room for the neighbour
// vectors (measured 122 -> 115 us per 18-real half-Dslash at 32^4).  For the
// 8-real form the Dslash reads a chosen set of link blocks with ordinary
// loads instead (`cached`): that part of the field, sized to fit the cache
// next to the vectors, is then served from the Infinity Cache from one
// launch to the next (see link_cache_mask).  Single precision fields
// (201-302 MB) partly live in the Infinity Cache, and nontemporal loads
// measured slower there, so they use ordinary loads.
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

// sin and cos of a phase |a| <= pi (as atan2 returns): quadrant k = rint(2a/pi),
// r = a - k pi/2 with pi/2 split in two parts (Cody and Waite), |r| <= pi/4,
// then the Taylor series of sin r and cos r in r^2, evaluated by Horner's
// rule, to the term that falls below the unit roundoff (r^17/17! and
// r^16/16! for double, r^9/9! and r^8/8! for float).
template <typename R> struct PhaseSeries;
template <> struct PhaseSeries<double> {
    static constexpr int kTerms = 8;
    static constexpr double kPio2Hi = 1.57079632679489655800e+00, kPio2Lo = 6.12323399573676603587e-17;
};
template <> struct PhaseSeries<float> {
    static constexpr int kTerms = 4;
    static constexpr float kPio2Hi = 1.57079625129699707031e+00f, kPio2Lo = 7.54978995489188216e-08f;
};
// (-1)^n / (2n+1)! and (-1)^n / (2n)!
__host__ __device__ constexpr double taylor_sin(int n) {
    double f = 1.0;
    for (int k = 2; k <= 2 * n + 1; ++k) f *= k;
    return (n & 1 ? -1.0 : 1.0) / f;
}
__host__ __device__ constexpr double taylor_cos(int n) {
    double f = 1.0;
    for (int k = 2; k <= 2 * n; ++k) f *= k;
    return (n & 1 ? -1.0 : 1.0) / f;
}
template <typename R> __device__ __forceinline__ void sin_cos(R a, R *sn, R *cs) {
    using P = PhaseSeries<R>;
    const R k = rint(a * R(0.63661977236758134308));
    const R r = (a - k * P::kPio2Hi) - k * P::kPio2Lo;
    const R r2 = r * r;
    R ps = R(taylor_sin(P::kTerms)), pc = R(taylor_cos(P::kTerms));
#pragma unroll
    for (int n = P::kTerms - 1; n >= 0; --n) {
        ps = fma(ps, r2, R(taylor_sin(n)));
        pc = fma(pc, r2, R(taylor_cos(n)));
    }
    const R s0 = r * ps, c0 = pc;
    const int q = int(k) & 3;
    *sn = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
    *cs = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
}

// 8-real form.  With u = row 0, v = row 1, w = row 2 and N = |u1|^2 + |u2|^2:
//   |u0| = sqrt(1 - N), |v0|^2 + |w0|^2 = N                 (unit row 0 and column 0)
// of v0 and w0 the smaller in modulus is stored and the other's modulus is
// sqrt(N - |stored|^2), which has no cancellation.  From u . conj(v) = 0 and
// w0 = conj(u1 v2 - u2 v1) (w = conj(u x v)), and the same two relations for
// w (v = conj(w x u)), a 2 x 2 system each with determinant N:
//   v1 = -(conj(u0) u1 v0 + conj(u2) conj(w0)) / N,  v2 = (conj(u1) conj(w0) - conj(u0) u2 v0) / N
//   w1 = (conj(u2) conj(v0) - conj(u0) u1 w0) / N,   w2 = -(conj(u1) conj(v0) + conj(u0) u2 w0) / N
// (largest entry error of a rebuilt double field: 1.4e-15 on smoothed 32^4
// fields, 2.4e-14 on Haar fields).
__device__ __forceinline__ double rcp_approx(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R>
__device__ __forceinline__ void rebuild8(su3<R> &u, cplx<R> c, R arg_u0, R t) {
    const cplx<R> u1 = u.e[0][1], u2 = u.e[0][2];
    const R n = u1.re * u1.re + u1.im * u1.im + u2.re * u2.re + u2.im * u2.im;
    const bool c_is_w0 = t > R(4);
    const R arg_other = c_is_w0 ? t - R(8) : t;
    const R m_u0 = sqrt(fmax(R(1) - n, R(0)));
    const R m_other = sqrt(fmax(n - (c.re * c.re + c.im * c.im), R(0)));
    R s, co;
    sin_cos(arg_u0, &s, &co);
    const cplx<R> u0 = {m_u0 * co, m_u0 * s};
    sin_cos(arg_other, &s, &co);
    const cplx<R> other = {m_other * co, m_other * s};
    const cplx<R> v0 = c_is_w0 ? other : c, w0 = c_is_w0 ? c : other;
    // 1/n from the hardware reciprocal and one Newton step (n is in (0, 1])
    R inv = rcp_approx(n);
    inv = inv * fma(-n, inv, R(2));
    const cplx<R> cu0v0 = cmul(conj(u0), v0), cu0w0 = cmul(conj(u0), w0);
    u.e[0][0] = u0;
    u.e[1][0] = v0;
    u.e[2][0] = w0;
    u.e[1][1] = (-inv) * (cmul(cu0v0, u1) + cmul(conj(u2), conj(w0)));
    u.e[1][2] = inv * (cmul(conj(u1), conj(w0)) - cmul(cu0v0, u2));
    u.e[2][1] = inv * (cmul(conj(u2), conj(v0)) - cmul(cu0w0, u1));
    u.e[2][2] = (-inv) * (cmul(conj(u1), conj(v0)) + cmul(cu0w0, u2));
}

// The stored column-0 entry and the phase word t of a link (8-real form).
template <typename R>
__device__ __forceinline__ void pack8_column(const su3<R> &u, cplx<R> &c, R &t) {
    const cplx<R> v0 = u.e[1][0], w0 = u.e[2][0];
    const bool c_is_w0 = (w0.re * w0.re + w0.im * w0.im) < (v0.re * v0.re + v0.im * v0.im);
    c = c_is_w0 ? w0 : v0;
    const cplx<R> o = c_is_w0 ? v0 : w0;
    t = atan2(o.im, o.re) + (c_is_w0 ? R(8) : R(0));
}

template <> struct LinkLayout<double, 1> {
    static constexpr int64_t kBytesPerLink = 64;
    // the stored words of one link; load_raw issues the loads, build rebuilds
    // (split so that a kernel can issue the next link's loads first)
    struct Raw { double2 a, d, c, t; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int blk, int64_t i,
                                                   bool cached = false) {
        const double2 *b = static_cast<const double2 *>(base) + (int64_t)blk * 4 * vh;
        // `cached` is uniform over a launch: a branch, not a select of two loads
        if (cached) return {b[0 * vh + i], b[1 * vh + i], b[2 * vh + i], b[3 * vh + i]};
        return {ld_nt(&b[0 * vh + i]), ld_nt(&b[1 * vh + i]), ld_nt(&b[2 * vh + i]), ld_nt(&b[3 * vh + i])};
    }
    __device__ static __forceinline__ su3<double> build(const Raw &w) {
        su3<double> u;
        u.e[0][1] = {w.a.x, w.a.y};
        u.e[0][2] = {w.d.x, w.d.y};
        rebuild8(u, cplx<double>{w.c.x, w.c.y}, w.t.x, w.t.y);
        return u;
    }
    __device__ static __forceinline__ su3<double> load(const void *base, int64_t vh, int blk, int64_t i,
                                                      bool cached = false) {
        return build(load_raw(base, vh, blk, i, cached));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<double> &u) {
        double2 *b = static_cast<double2 *>(base) + (int64_t)blk * 4 * vh;
        cplx<double> c;
        double t;
        pack8_column(u, c, t);
        b[0 * vh + i] = make_double2(u.e[0][1].re, u.e[0][1].im);
        b[1 * vh + i] = make_double2(u.e[0][2].re, u.e[0][2].im);
        b[2 * vh + i] = make_double2(c.re, c.im);
        b[3 * vh + i] = make_double2(atan2(u.e[0][0].im, u.e[0][0].re), t);
    }
};
template <> struct LinkLayout<float, 1> {
    static constexpr int64_t kBytesPerLink = 32;
    struct Raw { float4 a, t; };
    __device__ static __forceinline__ Raw load_raw(const void *base, int64_t vh, int blk, int64_t i) {
        const float4 *q = reinterpret_cast<const float4 *>(static_cast<const char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        return {q[0 * vh + i], q[1 * vh + i]};
    }
    __device__ static __forceinline__ su3<float> build(const Raw &w) {
        su3<float> u;
        u.e[0][1] = {w.a.x, w.a.y};
        u.e[0][2] = {w.a.z, w.a.w};
        rebuild8(u, cplx<float>{w.t.x, w.t.y}, w.t.z, w.t.w);
        return u;
    }
    __device__ static __forceinline__ su3<float> load(const void *base, int64_t vh, int blk, int64_t i) {
        return build(load_raw(base, vh, blk, i));
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<float> &u) {
        float4 *q = reinterpret_cast<float4 *>(static_cast<char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        cplx<float> c;
        float t;
        pack8_column(u, c, t);
        q[0 * vh + i] = make_float4(u.e[0][1].re, u.e[0][1].im, u.e[0][2].re, u.e[0][2].im);
        q[1 * vh + i] = make_float4(c.re, c.im, atan2f(u.e[0][0].im, u.e[0][0].re), t);
    }
};

// Double precision links stored as pairs of floats (Section 5 of the paper:
// a double a kept as b = RN_float(a) and c = RN_float(a - b), a = b + c to
// about 2^-48 |a|), as the one device copy of the field: the 8 link blocks
// of the single precision form (hi) come first, the 8 blocks of the
// remainders (lo) after them, both in the LinkLayout<float, NROW> form.
// Single precision kernels read the first half as an ordinary single
// precision field; double precision kernels read both halves and add them
// in double.  Coded as NROW = kHiLo + 2 (12 reals) or kHiLo + 3 (18 reals).
constexpr int kHiLo = 10;

__device__ __forceinline__ cplx<double> hilo_pair(float hre, float him, float lre, float lim) {
    return {double(hre) + double(lre), double(him) + double(lim)};
}
__device__ __forceinline__ void hilo_split(const cplx<double> &a, float &hre, float &him, float &lre, float &lim) {
    hre = float(a.re);
    him = float(a.im);
    lre = float(a.re - double(hre));
    lim = float(a.im - double(him));
}

template <> struct LinkLayout<double, kHiLo + 2> {
    static constexpr int64_t kHalf = 48;               // bytes per link of each half
    static constexpr int64_t kBytesPerLink = 2 * kHalf;
    __device__ static __forceinline__ su3<double> load(const void *base, int64_t vh, int blk, int64_t i) {
        const float4 *h = reinterpret_cast<const float4 *>(static_cast<const char *>(base) + (int64_t)blk * kHalf * vh);
        const float4 *l = reinterpret_cast<const float4 *>(static_cast<const char *>(base) + (int64_t)(8 + blk) * kHalf * vh);
        su3<double> u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float4 a = ld_nt(&h[k * vh + i]), b = ld_nt(&l[k * vh + i]);
            const int e0 = 2 * k, e1 = 2 * k + 1;   // entries {u00,u01}, {u02,u10}, {u11,u12}
            u.e[e0 / 3][e0 % 3] = hilo_pair(a.x, a.y, b.x, b.y);
            u.e[e1 / 3][e1 % 3] = hilo_pair(a.z, a.w, b.z, b.w);
        }
        su3_rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<double> &u) {
        float4 *h = reinterpret_cast<float4 *>(static_cast<char *>(base) + (int64_t)blk * kHalf * vh);
        float4 *l = reinterpret_cast<float4 *>(static_cast<char *>(base) + (int64_t)(8 + blk) * kHalf * vh);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e0 = 2 * k, e1 = 2 * k + 1;
            float4 a, b;
            hilo_split(u.e[e0 / 3][e0 % 3], a.x, a.y, b.x, b.y);
            hilo_split(u.e[e1 / 3][e1 % 3], a.z, a.w, b.z, b.w);
            h[k * vh + i] = a;
            l[k * vh + i] = b;
        }
    }
};

template <> struct LinkLayout<double, kHiLo + 3> {
    static constexpr int64_t kHalf = 72;
    static constexpr int64_t kBytesPerLink = 2 * kHalf;
    __device__ static __forceinline__ su3<double> load(const void *base, int64_t vh, int blk, int64_t i) {
        const char *hb = static_cast<const char *>(base) + (int64_t)blk * kHalf * vh;
        const char *lb = static_cast<const char *>(base) + (int64_t)(8 + blk) * kHalf * vh;
        const float4 *h = reinterpret_cast<const float4 *>(hb), *l = reinterpret_cast<const float4 *>(lb);
        su3<double> u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {   // entries 2k and 2k + 1 in row-major order
            const float4 a = ld_nt(&h[k * vh + i]), b = ld_nt(&l[k * vh + i]);
            const int e0 = 2 * k, e1 = 2 * k + 1;
            u.e[e0 / 3][e0 % 3] = hilo_pair(a.x, a.y, b.x, b.y);
            u.e[e1 / 3][e1 % 3] = hilo_pair(a.z, a.w, b.z, b.w);
        }
        const float2 a = ld_nt(reinterpret_cast<const float2 *>(hb + 64 * vh) + i);
        const float2 b = ld_nt(reinterpret_cast<const float2 *>(lb + 64 * vh) + i);
        u.e[2][2] = hilo_pair(a.x, a.y, b.x, b.y);
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<double> &u) {
        char *hb = static_cast<char *>(base) + (int64_t)blk * kHalf * vh;
        char *lb = static_cast<char *>(base) + (int64_t)(8 + blk) * kHalf * vh;
        float4 *h = reinterpret_cast<float4 *>(hb), *l = reinterpret_cast<float4 *>(lb);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e0 = 2 * k, e1 = 2 * k + 1;
            float4 a, b;
            hilo_split(u.e[e0 / 3][e0 % 3], a.x, a.y, b.x, b.y);
            hilo_split(u.e[e1 / 3][e1 % 3], a.z, a.w, b.z, b.w);
            h[k * vh + i] = a;
            l[k * vh + i] = b;
        }
        float2 a, b;
        hilo_split(u.e[2][2], a.x, a.y, b.x, b.y);
        reinterpret_cast<float2 *>(hb + 64 * vh)[i] = a;
        reinterpret_cast<float2 *>(lb + 64 * vh)[i] = b;
    }
};

// Single precision form of a stored format (the hi half of a float-pair field).
inline int nrow_single(int nrow) { return nrow > kHiLo ? nrow - kHiLo : nrow; }

// Low-precision copy for the learned preconditioner: 12 reals in bfloat16,
// 3 planes of 4 bf16 (8 bytes) per site: {u00, u01}, {u02, u10}, {u11, u12};
// the third row is rebuilt in single precision.
struct BF16Link {};
template <> struct LinkLayout<BF16Link, 2> {
    static constexpr int64_t kBytesPerLink = 24;
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    __device__ static __forceinline__ su3<float> load(const void *base, int64_t vh, int blk, int64_t i) {
        const bf16x4 *q = reinterpret_cast<const bf16x4 *>(static_cast<const char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        su3<float> u;
        bf16x4 v = q[0 * vh + i];
        u.e[0][0] = {float(v[0]), float(v[1])};
        u.e[0][1] = {float(v[2]), float(v[3])};
        v = q[1 * vh + i];
        u.e[0][2] = {float(v[0]), float(v[1])};
        u.e[1][0] = {float(v[2]), float(v[3])};
        v = q[2 * vh + i];
        u.e[1][1] = {float(v[0]), float(v[1])};
        u.e[1][2] = {float(v[2]), float(v[3])};
        su3_rebuild_row2(u);
        return u;
    }
    __device__ static __forceinline__ void store(void *base, int64_t vh, int blk, int64_t i, const su3<float> &u) {
        bf16x4 *q = reinterpret_cast<bf16x4 *>(static_cast<char *>(base) + (int64_t)blk * kBytesPerLink * vh);
        auto pk = [](cplx<float> a, cplx<float> b) {
            bf16x4 v;
            v[0] = static_cast<__bf16>(a.re);
            v[1] = static_cast<__bf16>(a.im);
            v[2] = static_cast<__bf16>(b.re);
            v[3] = static_cast<__bf16>(b.im);
            return v;
        };
        q[0 * vh + i] = pk(u.e[0][0], u.e[0][1]);
        q[1 * vh + i] = pk(u.e[0][2], u.e[1][0]);
        q[2 * vh + i] = pk(u.e[1][1], u.e[1][2]);
    }
};

// Bytes of one packed link field (both parities, 4 directions).
inline int64_t link_field_bytes(bool dbl, int nrow, int64_t vh) {
    int64_t per;
    if (nrow > kHiLo) per = 2 * (nrow - kHiLo == 3 ? 72 : 48);   // one field for both precisions
    else if (nrow == 1) per = dbl ? 64 : 32;
    else per = dbl ? 16 * 3 * nrow : (nrow == 3 ? 72 : 48);
    return per * 8 * vh;
}

}  // namespace stag
