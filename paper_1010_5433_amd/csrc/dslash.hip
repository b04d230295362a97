// Half hopping term of the even/odd staggered operator and its fused
// normal-operator epilogues.
//
// One lane per output site (the paper's Dirac kernel also gives every even
// site its own thread, Section 3).  Per site: 8 SU(3) x colour-vector
// products, 4 with the forward links U_mu(x) stored at the output parity and
// 4 with U_mu(x-mu)^dag stored at the input parity.  The kernel is bound by
// HBM bandwidth (0.46 flop/byte in double precision with 18-real links), so
// it uses no matrix cores: the work is to stream links and vectors with
// 16-byte coalesced loads and keep enough loads in flight.
#include "internal.h"
#include "links.h"

namespace stag {

template <typename R, int NROW, int MODE>
__global__ void __launch_bounds__(kDslashBlock) k_dslash(DslashArgs a) {
    if (a.skip && *a.skip) return;
    __shared__ double red[kDslashBlock / kWave];
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int i = tile * kDslashBlock + threadIdx.x;
    const int vh = a.g.Vh;
    const int p = a.out_parity;
    double part = 0.0;
    if (i < vh) {
        int x[4];
        site_coords(a.g, p, i, x);
        vec3<R> acc;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.c[c] = {R(0), R(0)};
        auto hop = [&](int mu) {
            const int jf = site_nbr(a.g, i, x, mu, +1);
            const int jb = site_nbr(a.g, i, x, mu, -1);
            const su3<R> uf = LinkLayout<R, NROW>::load(a.links, vh, p * 4 + mu, i);
            const vec3<R> vf = load_vec<R>(a.in, vh, jf);
            const su3<R> ub = LinkLayout<R, NROW>::load(a.links, vh, (1 - p) * 4 + mu, jb);
            const vec3<R> vb = load_vec<R>(a.in, vh, jb);
            acc_mul(acc, R(fwd_sign(a.g, x, mu)), uf, vf);
            acc_mul_dag(acc, R(-bwd_sign(a.g, x, mu)), ub, vb);
        };
        if constexpr (NROW == 1 && sizeof(R) == sizeof(double)) {
            // The 8-real double precision rebuild is long (two phases, two
            // square roots, a reciprocal): one hop per loop trip, with the next
            // hop's stored words and neighbour vector loaded before the
            // current link is rebuilt, so that the rebuild runs while the
            // next loads are in flight (144 VGPRs, three waves per SIMD).
            using L8 = LinkLayout<double, 1>;
            L8::Raw rw;
            vec3<R> vw;
            auto fetch = [&](int h) {
                const int mu = h >> 1;
                if (h & 1) {
                    const int jb = site_nbr(a.g, i, x, mu, -1), bb = (1 - p) * 4 + mu;
                    rw = L8::load_raw(a.links, vh, bb, jb, (a.link_cache >> bb) & 1);
                    vw = load_vec<R>(a.in, vh, jb);
                } else {
                    const int bf = p * 4 + mu;
                    rw = L8::load_raw(a.links, vh, bf, i, (a.link_cache >> bf) & 1);
                    vw = load_vec<R>(a.in, vh, site_nbr(a.g, i, x, mu, +1));
                }
            };
            fetch(0);
#pragma unroll 1
            for (int h = 0; h < 8; ++h) {
                const L8::Raw cw = rw;
                const vec3<R> cv = vw;
                if (h < 7) fetch(h + 1);
                const int mu = h >> 1;
                if (h & 1) acc_mul_dag(acc, R(-bwd_sign(a.g, x, mu)), L8::build(cw), cv);
                else acc_mul(acc, R(fwd_sign(a.g, x, mu)), L8::build(cw), cv);
            }
        } else if constexpr (NROW == 1) {
            // single precision: one direction at a time (the prefetching
            // form measured slower here)
#pragma unroll 1
            for (int mu = 0; mu < 4; ++mu) hop(mu);
        } else {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) hop(mu);
        }
        const R half = R(0.5);
        if (MODE == DS_PLAIN) {
            vec3<R> o;
#pragma unroll
            for (int c = 0; c < 3; ++c) o.c[c] = half * acc.c[c];
            store_vec_nt<R>(a.out, vh, i, o);   // measured: -2 to -4 % time per launch
        } else if (MODE == DS_NORMAL || MODE == DS_NORMAL_DOT) {
            const vec3<R> pv = load_vec<R>(a.aux, vh, i);
            const R c = R(a.c);
            vec3<R> o;
#pragma unroll
            for (int k = 0; k < 3; ++k) o.c[k] = c * pv.c[k] - half * acc.c[k];
            store_vec<R>(a.out, vh, i, o);
            if (MODE == DS_NORMAL_DOT) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    part += double(pv.c[k].re) * double(o.c[k].re) + double(pv.c[k].im) * double(o.c[k].im);
            }
        } else {  // DS_RESID, double precision only
            const vec3<R> xv = load_vec<R>(a.aux, vh, i);
            const vec3<R> bv = load_vec<R>(a.rhs, vh, i);
            const R c = R(a.c);
            vec3<R> r;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                r.c[k] = bv.c[k] - (c * xv.c[k] - half * acc.c[k]);
                part += double(r.c[k].re) * double(r.c[k].re) + double(r.c[k].im) * double(r.c[k].im);
            }
            if (a.out) store_vec<R>(a.out, vh, i, r);
        }
    }
    if (MODE == DS_NORMAL_DOT || MODE == DS_RESID) {
        const double s = block_sum(part, red);
        if (threadIdx.x == 0) a.partial[tile] = s;
    }
}

int dslash_grid(const Geom &g, int block) { return (g.Vh + block - 1) / block; }

template <typename R, int NROW>
static hipError_t launch_mode(int mode, const DslashArgs &a, hipStream_t s) {
    const dim3 grid(dslash_grid(a.g, kDslashBlock)), block(kDslashBlock);
    switch (mode) {
        case DS_PLAIN: hipLaunchKernelGGL((k_dslash<R, NROW, DS_PLAIN>), grid, block, 0, s, a); break;
        case DS_NORMAL: hipLaunchKernelGGL((k_dslash<R, NROW, DS_NORMAL>), grid, block, 0, s, a); break;
        case DS_NORMAL_DOT: hipLaunchKernelGGL((k_dslash<R, NROW, DS_NORMAL_DOT>), grid, block, 0, s, a); break;
        case DS_RESID:
            if (sizeof(R) != sizeof(double)) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_dslash<double, NROW, DS_RESID>), grid, block, 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dslash(bool dbl, int nrow, int mode, const DslashArgs &a, hipStream_t s) {
    if (dbl) {
        if (nrow == kHiLo + 2) return launch_mode<double, kHiLo + 2>(mode, a, s);
        if (nrow == kHiLo + 3) return launch_mode<double, kHiLo + 3>(mode, a, s);
        if (nrow == 1) return launch_mode<double, 1>(mode, a, s);
        return nrow == 2 ? launch_mode<double, 2>(mode, a, s) : launch_mode<double, 3>(mode, a, s);
    }
    nrow = nrow_single(nrow);   // a float-pair field: its hi half
    if (nrow == 1) return launch_mode<float, 1>(mode, a, s);
    return nrow == 2 ? launch_mode<float, 2>(mode, a, s) : launch_mode<float, 3>(mode, a, s);
}

}  // namespace stag
