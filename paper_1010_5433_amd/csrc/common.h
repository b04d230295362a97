// Shared device-side building blocks: complex arithmetic, SU(3) x colour
// vector products, deterministic wave64/block FP64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stag {

constexpr int kWave = 64;

// ---------------------------------------------------------------- complex
template <typename R> struct cplx { R re, im; };

template <typename R> __device__ __forceinline__ cplx<R> cmake(R a, R b) { return {a, b}; }
template <typename R> __device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }

template <typename R> struct vec3 { cplx<R> c[3]; };
template <typename R> struct su3 { cplx<R> e[3][3]; };

// Third row of an SU(3) matrix from the first two: conj(row0 x row1).
template <typename R> __device__ __forceinline__ void su3_rebuild_row2(su3<R> &u) {
    u.e[2][0] = conj(cmul(u.e[0][1], u.e[1][2]) - cmul(u.e[0][2], u.e[1][1]));
    u.e[2][1] = conj(cmul(u.e[0][2], u.e[1][0]) - cmul(u.e[0][0], u.e[1][2]));
    u.e[2][2] = conj(cmul(u.e[0][0], u.e[1][1]) - cmul(u.e[0][1], u.e[1][0]));
}

// acc += s * U v
template <typename R> __device__ __forceinline__ void acc_mul(vec3<R> &acc, R s, const su3<R> &u, const vec3<R> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cplx<R> t = cmul(u.e[a][0], v.c[0]);
        t = t + cmul(u.e[a][1], v.c[1]);
        t = t + cmul(u.e[a][2], v.c[2]);
        acc.c[a] = acc.c[a] + s * t;
    }
}

// acc += s * U^dag v
template <typename R> __device__ __forceinline__ void acc_mul_dag(vec3<R> &acc, R s, const su3<R> &u, const vec3<R> &v) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cplx<R> t = cmulc(u.e[0][a], v.c[0]);
        t = t + cmulc(u.e[1][a], v.c[1]);
        t = t + cmulc(u.e[2][a], v.c[2]);
        acc.c[a] = acc.c[a] + s * t;
    }
}

// ---------------------------------------------------------------- streaming loads
// Nontemporal loads: data that is read once (the gauge links) should not
// push reusable data (neighbour colour vectors) out of the XCD's L2.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld_nt(const float2 *p) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v) {
    __builtin_nontemporal_store(d2v{v.x, v.y}, reinterpret_cast<d2v *>(p));
}
__device__ __forceinline__ void st_nt(float2 *p, float2 v) {
    __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v *>(p));
}

// ---------------------------------------------------------------- storage types
// Library vectors: [colour][site] planes of {re,im}.
template <typename R> struct vtype;
template <> struct vtype<double> { using t2 = double2; };
template <> struct vtype<float> { using t2 = float2; };

template <typename R> __device__ __forceinline__ cplx<R> ld2(const typename vtype<R>::t2 *p, int64_t i) {
    typename vtype<R>::t2 v = p[i];
    return {v.x, v.y};
}
template <typename R> __device__ __forceinline__ void st2(typename vtype<R>::t2 *p, int64_t i, cplx<R> c) {
    typename vtype<R>::t2 v;
    v.x = c.re;
    v.y = c.im;
    p[i] = v;
}

template <typename R> __device__ __forceinline__ vec3<R> load_vec(const void *base, int64_t vh, int64_t i) {
    const typename vtype<R>::t2 *p = static_cast<const typename vtype<R>::t2 *>(base);
    vec3<R> v;
#pragma unroll
    for (int c = 0; c < 3; ++c) v.c[c] = ld2<R>(p + c * vh, i);
    return v;
}
// Nontemporal store of a colour vector: for an output that the next kernel
// reads through its neighbour gathers, not through this kernel's caches.
template <typename R> __device__ __forceinline__ void store_vec_nt(void *base, int64_t vh, int64_t i, const vec3<R> &v) {
    using T2 = typename vtype<R>::t2;
    T2 *b = static_cast<T2 *>(base);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T2 w;
        w.x = v.c[c].re;
        w.y = v.c[c].im;
        st_nt(&b[c * vh + i], w);
    }
}
template <typename R> __device__ __forceinline__ void store_vec(void *base, int64_t vh, int64_t i, const vec3<R> &v) {
    typename vtype<R>::t2 *p = static_cast<typename vtype<R>::t2 *>(base);
#pragma unroll
    for (int c = 0; c < 3; ++c) st2<R>(p + c * vh, i, v.c[c]);
}

// ---------------------------------------------------------------- reductions
// Every lane of a 16-lane row ends with the row sum, bitwise identical across
// the row: two quad permutations (xor 1, xor 2), then the half-row and row
// mirrors.  All 64 lanes must be active.
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    int2 b = *reinterpret_cast<int2 *>(&v);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xF, 0xF, false);
    return *reinterpret_cast<double *>(&r);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    int2 b = *reinterpret_cast<int2 *>(&v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(b.x, lane);
    r.y = __builtin_amdgcn_readlane(b.y, lane);
    return *reinterpret_cast<double *>(&r);
}

// Wave64 sum, returned uniformly (same value in every lane).  Fixed order.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x141>(v);  // row_half_mirror
    v += dpp_d<0x140>(v);  // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Block sum (blockDim.x a multiple of 64, <= 1024).  Result valid in every
// thread.  lds must hold blockDim.x/64 doubles.  Fixed order.
__device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int nw = blockDim.x / kWave;
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += lds[k];
    __syncthreads();
    return s;
}

// Per-thread part of a fixed-order sum of reduction partials: t = part[k]
// for k = threadIdx.x, threadIdx.x + B, ... < n, added in that order (B =
// the threads that share the sum).  The loads go out in groups of
// kPartGroup, all of a group before its first addition: a loop that adds
// each partial as it arrives waits for the loads one after another.  The
// index is clamped instead of branched on, so that no branch ties an
// addition to its load.
constexpr int kPartGroup = 8;

template <int B>
__device__ __forceinline__ void part_load_group(const double *part, int n, int k0, double (&v)[kPartGroup]) {
    if (n < 1) return;
#pragma unroll
    for (int u = 0; u < kPartGroup; ++u) {
        const int k = k0 + u * B;
        v[u] = part[k < n ? k : n - 1];
    }
}
template <int B>
__device__ __forceinline__ double part_add_group(double t, int n, int k0, const double (&v)[kPartGroup]) {
#pragma unroll
    for (int u = 0; u < kPartGroup; ++u)
        if (k0 + u * B < n) t += v[u];
    return t;
}
// the sum from k0 on, its earlier terms already in t
template <int B> __device__ __forceinline__ double part_sum_from(double t, const double *part, int n, int k0) {
    for (; k0 < n; k0 += kPartGroup * B) {
        double v[kPartGroup];
        part_load_group<B>(part, n, k0, v);
        t = part_add_group<B>(t, n, k0, v);
    }
    return t;
}
template <int B> __device__ __forceinline__ double part_sum(const double *part, int n) {
    return part_sum_from<B>(0.0, part, n, threadIdx.x);
}

}  // namespace stag
