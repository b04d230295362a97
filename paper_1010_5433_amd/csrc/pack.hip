// Layout conversion (set-up, not in the solver loop) and the geometry-table
// export used to check the device index functions.
#include "internal.h"
#include "links.h"

namespace stag {

constexpr int kPackBlock = 256;

// Canonical complex128 (4,V,3,3) [mu][lex][row][col] -> packed even/odd SoA.
template <typename R, int NROW>
__global__ void __launch_bounds__(kPackBlock) k_pack_links(Geom g, const double2 *canon, void *dst) {
    const int64_t vol = 2 * (int64_t)g.Vh;
    const int64_t k = (int64_t)blockIdx.x * kPackBlock + threadIdx.x;
    if (k >= 4 * vol) return;
    const int mu = (int)(k / vol);
    const int64_t lex = k - mu * vol;
    int64_t r = lex;
    int x[4];
    for (int nu = 0; nu < 4; ++nu) {
        x[nu] = (int)(r % g.L[nu]);
        r /= g.L[nu];
    }
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    su3<R> u;
    const double2 *src = canon + k * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double2 v = src[e];
        u.e[e / 3][e % 3] = {R(v.x), R(v.y)};
    }
    LinkLayout<R, NROW>::store(dst, g.Vh, p * 4 + mu, lex >> 1, u);
}

// Packed double precision field (any format) -> canonical complex128
// (4,V,3,3), rebuilding the rows a compressed format does not store.
template <int NROW>
__global__ void __launch_bounds__(kPackBlock) k_unpack_links(Geom g, const void *packed, double2 *canon) {
    const int64_t vol = 2 * (int64_t)g.Vh;
    const int64_t k = (int64_t)blockIdx.x * kPackBlock + threadIdx.x;
    if (k >= 4 * vol) return;
    const int mu = (int)(k / vol);
    const int64_t lex = k - mu * vol;
    int64_t r = lex;
    int x[4];
    for (int nu = 0; nu < 4; ++nu) {
        x[nu] = (int)(r % g.L[nu]);
        r /= g.L[nu];
    }
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const su3<double> u = LinkLayout<double, NROW>::load(packed, g.Vh, p * 4 + mu, lex >> 1);
    double2 *dst = canon + k * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) dst[e] = make_double2(u.e[e / 3][e % 3].re, u.e[e / 3][e % 3].im);
}

// Largest entry-wise difference between the canonical links and the links
// rebuilt from a packed double precision field (one partial per block).
template <int NROW>
__global__ void __launch_bounds__(kPackBlock) k_check_links(Geom g, const double2 *canon, const void *packed,
                                                          double *partial) {
    const int64_t vol = 2 * (int64_t)g.Vh;
    const int64_t k = (int64_t)blockIdx.x * kPackBlock + threadIdx.x;
    double err = 0.0;
    if (k < 4 * vol) {
        const int mu = (int)(k / vol);
        const int64_t lex = k - mu * vol;
        int64_t r = lex;
        int x[4];
        for (int nu = 0; nu < 4; ++nu) {
            x[nu] = (int)(r % g.L[nu]);
            r /= g.L[nu];
        }
        const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
        const su3<double> u = LinkLayout<double, NROW>::load(packed, g.Vh, p * 4 + mu, lex >> 1);
        const double2 *src = canon + k * 9;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const double2 v = src[e];
            const double d = fmax(fabs(u.e[e / 3][e % 3].re - v.x), fabs(u.e[e / 3][e % 3].im - v.y));
            err = (d > err || d != d) ? d : err;   // a NaN wins
        }
    }
    // block maximum, NaN-propagating, in a fixed order
    __shared__ double mx[kPackBlock];
    mx[threadIdx.x] = err;
    __syncthreads();
    for (int h = kPackBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double a = mx[threadIdx.x], b = mx[threadIdx.x + h];
            mx[threadIdx.x] = (b > a || b != b) ? b : a;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = mx[0];
}

// bfloat16 12-real copy of a packed single precision field (any format).
template <int NROW>
__global__ void __launch_bounds__(kPackBlock) k_pack_links16(int vh, const void *src, void *dst) {
    const int64_t k = (int64_t)blockIdx.x * kPackBlock + threadIdx.x;
    if (k >= 8 * (int64_t)vh) return;
    const int blk = (int)(k / vh);
    const int64_t i = k - (int64_t)blk * vh;
    const su3<float> u = LinkLayout<float, NROW>::load(src, vh, blk, i);
    LinkLayout<BF16Link, 2>::store(dst, vh, blk, i, u);
}

template <typename R>
__global__ void __launch_bounds__(kPackBlock) k_pack_vec(int vh, const double2 *canon, void *dst) {
    const int i = blockIdx.x * kPackBlock + threadIdx.x;
    if (i >= vh) return;
    vec3<R> v;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double2 z = canon[(int64_t)i * 3 + c];
        v.c[c] = {R(z.x), R(z.y)};
    }
    store_vec<R>(dst, vh, i, v);
}

template <typename R>
__global__ void __launch_bounds__(kPackBlock) k_unpack_vec(int vh, const void *src, double2 *canon) {
    const int i = blockIdx.x * kPackBlock + threadIdx.x;
    if (i >= vh) return;
    const vec3<R> v = load_vec<R>(src, vh, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) canon[(int64_t)i * 3 + c] = make_double2(double(v.c[c].re), double(v.c[c].im));
}

__global__ void __launch_bounds__(kPackBlock) k_tables(Geom g, int32_t *nbr, int32_t *coord, int32_t *sign) {
    const int k = blockIdx.x * kPackBlock + threadIdx.x;
    if (k >= 2 * g.Vh) return;
    const int p = k / g.Vh, i = k - p * g.Vh;
    int x[4];
    site_coords(g, p, i, x);
    for (int mu = 0; mu < 4; ++mu) {
        if (nbr) {
            nbr[(int64_t)(p * 8 + mu) * g.Vh + i] = site_nbr(g, i, x, mu, +1);
            nbr[(int64_t)(p * 8 + 4 + mu) * g.Vh + i] = site_nbr(g, i, x, mu, -1);
        }
        if (sign) {
            sign[(int64_t)(p * 8 + mu) * g.Vh + i] = fwd_sign(g, x, mu);
            sign[(int64_t)(p * 8 + 4 + mu) * g.Vh + i] = bwd_sign(g, x, mu);
        }
        if (coord) coord[((int64_t)p * g.Vh + i) * 4 + mu] = x[mu];
    }
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kPackBlock - 1) / kPackBlock); }

hipError_t launch_pack_links(const Geom &g, const void *canon, void *dst, bool dbl, int nrow, hipStream_t s) {
    const int64_t n = 8 * (int64_t)g.Vh;
    const double2 *c = static_cast<const double2 *>(canon);
    if (dbl) {
        if (nrow == kHiLo + 2) hipLaunchKernelGGL((k_pack_links<double, kHiLo + 2>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else if (nrow == kHiLo + 3) hipLaunchKernelGGL((k_pack_links<double, kHiLo + 3>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else if (nrow == 1) hipLaunchKernelGGL((k_pack_links<double, 1>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else if (nrow == 2) hipLaunchKernelGGL((k_pack_links<double, 2>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else hipLaunchKernelGGL((k_pack_links<double, 3>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
    } else {
        if (nrow > kHiLo) return hipErrorInvalidValue;   // float pairs are packed in one double pass
        if (nrow == 1) hipLaunchKernelGGL((k_pack_links<float, 1>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else if (nrow == 2) hipLaunchKernelGGL((k_pack_links<float, 2>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
        else hipLaunchKernelGGL((k_pack_links<float, 3>), dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, dst);
    }
    return hipGetLastError();
}

hipError_t launch_pack_links16(const Geom &g, const void *links32, int nrow, void *dst, hipStream_t s) {
    const int64_t n = 8 * (int64_t)g.Vh;
    nrow = nrow_single(nrow);
    if (nrow == 1) hipLaunchKernelGGL(k_pack_links16<1>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g.Vh, links32, dst);
    else if (nrow == 2) hipLaunchKernelGGL(k_pack_links16<2>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g.Vh, links32, dst);
    else hipLaunchKernelGGL(k_pack_links16<3>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g.Vh, links32, dst);
    return hipGetLastError();
}

int check_links_blocks(const Geom &g) { return (int)blocks_for(8 * (int64_t)g.Vh); }

hipError_t launch_check_links(const Geom &g, const void *canon, const void *packed64, int nrow, double *partial,
                              hipStream_t s) {
    const int64_t n = 8 * (int64_t)g.Vh;
    const double2 *c = static_cast<const double2 *>(canon);
    if (nrow == 1) hipLaunchKernelGGL(k_check_links<1>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, packed64, partial);
    else if (nrow == 2) hipLaunchKernelGGL(k_check_links<2>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, packed64, partial);
    else hipLaunchKernelGGL(k_check_links<3>, dim3(blocks_for(n)), dim3(kPackBlock), 0, s, g, c, packed64, partial);
    return hipGetLastError();
}

hipError_t launch_unpack_links(const Geom &g, const void *packed64, int nrow, void *canon, hipStream_t s) {
    const int64_t n = 8 * (int64_t)g.Vh;
    double2 *c = static_cast<double2 *>(canon);
    const dim3 grid(blocks_for(n)), block(kPackBlock);
    switch (nrow) {
        case 1: hipLaunchKernelGGL(k_unpack_links<1>, grid, block, 0, s, g, packed64, c); break;
        case 2: hipLaunchKernelGGL(k_unpack_links<2>, grid, block, 0, s, g, packed64, c); break;
        case 3: hipLaunchKernelGGL(k_unpack_links<3>, grid, block, 0, s, g, packed64, c); break;
        case kHiLo + 2: hipLaunchKernelGGL(k_unpack_links<kHiLo + 2>, grid, block, 0, s, g, packed64, c); break;
        case kHiLo + 3: hipLaunchKernelGGL(k_unpack_links<kHiLo + 3>, grid, block, 0, s, g, packed64, c); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_vec(const Geom &g, const void *canon, void *dst, bool dbl, hipStream_t s) {
    const double2 *c = static_cast<const double2 *>(canon);
    if (dbl) hipLaunchKernelGGL((k_pack_vec<double>), dim3(blocks_for(g.Vh)), dim3(kPackBlock), 0, s, g.Vh, c, dst);
    else hipLaunchKernelGGL((k_pack_vec<float>), dim3(blocks_for(g.Vh)), dim3(kPackBlock), 0, s, g.Vh, c, dst);
    return hipGetLastError();
}

hipError_t launch_unpack_vec(const Geom &g, const void *src, void *canon, bool dbl, hipStream_t s) {
    double2 *c = static_cast<double2 *>(canon);
    if (dbl) hipLaunchKernelGGL((k_unpack_vec<double>), dim3(blocks_for(g.Vh)), dim3(kPackBlock), 0, s, g.Vh, src, c);
    else hipLaunchKernelGGL((k_unpack_vec<float>), dim3(blocks_for(g.Vh)), dim3(kPackBlock), 0, s, g.Vh, src, c);
    return hipGetLastError();
}

hipError_t launch_tables(const Geom &g, int32_t *nbr, int32_t *coord, int32_t *sign, hipStream_t s) {
    hipLaunchKernelGGL(k_tables, dim3(blocks_for(2 * (int64_t)g.Vh)), dim3(kPackBlock), 0, s, g, nbr, coord, sign);
    return hipGetLastError();
}

}  // namespace stag
