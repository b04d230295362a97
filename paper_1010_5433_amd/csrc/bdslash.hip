// Multi-RHS batched half-Dslash.
//
// A launch walks a tile table.  A tile is (lattice, 64..256 consecutive
// output sites, up to RPT systems on that lattice).  Each lane handles one
// site: it loads the 4 forward and 4 backward links once and applies them
// to the neighbour vectors of every live system of the tile, so the link
// traffic -- 92% of a single-RHS Dslash in double precision -- is divided by
// the number of right-hand sides.  Tiles of different lattices (different
// extents) share the launch: every tile reads its own geometry.
#include "batch.h"
#include "links.h"

namespace stag {

template <typename R, int NROW, int RPT, int ROLE>
__global__ void __launch_bounds__(256) kb_dslash(BView v, int sel, int skip_done, int write) {
    const BTile tile = v.tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BLat lat = v.lats[tile.lat];
    const int vh = lat.g.Vh;
    const BSys *sp[RPT];
    const void *in[RPT];
    int sh[RPT];
    bool live[RPT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        live[r] = false;
        sp[r] = nullptr;
        in[r] = nullptr;
        sh[r] = 0;
        if (r < tile.nsys) {
            const BSys *s = v.sys + tile.sys[r];
            const int k = sel < 0 ? s->base : sel;
            // skip_done 1: systems whose solve ended; 2: systems with no reliable update due
            bool l = !(skip_done == 1 ? s->st->done : skip_done == 2 ? s->st->rel_skip : 0);
            if (ROLE == BR_OE_X || ROLE == BR_EO_RESID) l = l && k < s->n;
            if (l) {
                live[r] = true;
                sp[r] = s;
                sh[r] = k;
                in[r] = ROLE == BR_OE_P ? s->p[s->base] : ROLE == BR_EO_AP ? s->t
                      : ROLE == BR_OE_X ? (const void *)s->xhi[k] : (const void *)s->t64;
                any = true;
            }
        }
    }
    if (!any) return;

    const int p = (ROLE == BR_OE_P || ROLE == BR_OE_X) ? 1 : 0;
    const void *links = (ROLE == BR_OE_X || ROLE == BR_EO_RESID) ? lat.links64 : lat.links;
    const int i = tile.site0 + threadIdx.x;
    vec3<R> acc[RPT];
    double part[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        part[r] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r].c[c] = {R(0), R(0)};
    }
    if (i < vh) {
        int x[4];
        site_coords(lat.g, p, i, x);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int jf = site_nbr(lat.g, i, x, mu, +1);
            const int jb = site_nbr(lat.g, i, x, mu, -1);
            const su3<R> uf = LinkLayout<R, NROW>::load(links, vh, p * 4 + mu, i);
            const R sf = R(fwd_sign(lat.g, x, mu));
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (live[r]) acc_mul(acc[r], sf, uf, load_vec<R>(in[r], vh, jf));
            const su3<R> ub = LinkLayout<R, NROW>::load(links, vh, (1 - p) * 4 + mu, jb);
            const R sb = R(-bwd_sign(lat.g, x, mu));
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (live[r]) acc_mul_dag(acc[r], sb, ub, load_vec<R>(in[r], vh, jb));
        }
        const R half = R(0.5);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!live[r]) continue;
            const BSys *s = sp[r];
            if (ROLE == BR_OE_P || ROLE == BR_OE_X) {
                vec3<R> o;
#pragma unroll
                for (int c = 0; c < 3; ++c) o.c[c] = half * acc[r].c[c];
                store_vec<R>(ROLE == BR_OE_P ? s->t : (void *)s->t64, vh, i, o);
            } else if (ROLE == BR_EO_AP) {
                const vec3<R> pv = load_vec<R>(s->p[s->base], vh, i);
                const R c = R(s->m2 + s->shifts[s->base]);
                vec3<R> o;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    o.c[k] = c * pv.c[k] - half * acc[r].c[k];
                    part[r] += double(pv.c[k].re) * double(o.c[k].re) + double(pv.c[k].im) * double(o.c[k].im);
                }
                store_vec<R>(s->ap, vh, i, o);
            } else {  // BR_EO_RESID (double)
                const vec3<R> xv = load_vec<R>(s->xhi[sh[r]], vh, i);
                const vec3<R> bv = load_vec<R>(s->src, vh, i);
                const R c = R(s->m2 + s->shifts[sh[r]]);
                vec3<R> o;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    o.c[k] = bv.c[k] - (c * xv.c[k] - half * acc[r].c[k]);
                    part[r] += double(o.c[k].re) * double(o.c[k].re) + double(o.c[k].im) * double(o.c[k].im);
                }
                if (write) store_vec<R>(s->rhi, vh, i, o);
            }
        }
    }
    if (ROLE == BR_EO_AP || ROLE == BR_EO_RESID) {
        // one partial per 64 consecutive sites, independent of the block size
        const int chunk = (tile.site0 >> 6) + (int)(threadIdx.x >> 6);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!live[r]) continue;
            const double w = wave_sum(part[r]);
            if ((threadIdx.x & 63) == 0 && chunk < sp[r]->nchunk_ds) sp[r]->part_ds[chunk] = w;
        }
    }
}

template <typename R, int NROW, int RPT>
static hipError_t launch_role(int role, int block, BView v, int sel, int skip, int write, hipStream_t s) {
    const dim3 grid(v.ntiles), blk(block);
    switch (role) {
        case BR_OE_P: hipLaunchKernelGGL((kb_dslash<R, NROW, RPT, BR_OE_P>), grid, blk, 0, s, v, sel, skip, write); break;
        case BR_EO_AP: hipLaunchKernelGGL((kb_dslash<R, NROW, RPT, BR_EO_AP>), grid, blk, 0, s, v, sel, skip, write); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NROW, int RPT>
static hipError_t launch_role64(int role, int block, BView v, int sel, int skip, int write, hipStream_t s) {
    const dim3 grid(v.ntiles), blk(block);
    switch (role) {
        case BR_OE_P: hipLaunchKernelGGL((kb_dslash<double, NROW, RPT, BR_OE_P>), grid, blk, 0, s, v, sel, skip, write); break;
        case BR_EO_AP: hipLaunchKernelGGL((kb_dslash<double, NROW, RPT, BR_EO_AP>), grid, blk, 0, s, v, sel, skip, write); break;
        case BR_OE_X: hipLaunchKernelGGL((kb_dslash<double, NROW, RPT, BR_OE_X>), grid, blk, 0, s, v, sel, skip, write); break;
        case BR_EO_RESID: hipLaunchKernelGGL((kb_dslash<double, NROW, RPT, BR_EO_RESID>), grid, blk, 0, s, v, sel, skip, write); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NROW>
static hipError_t launch_nrow(bool dbl, BDslashCfg cfg, BView v, int role, int sel, int skip, int write, hipStream_t s) {
    // the double precision residual roles always run on the double links
    if (dbl || role == BR_OE_X || role == BR_EO_RESID) {
        switch (cfg.rpt) {
            case 1: return launch_role64<NROW, 1>(role, cfg.block, v, sel, skip, write, s);
            case 2: return launch_role64<NROW, 2>(role, cfg.block, v, sel, skip, write, s);
            case 4: return launch_role64<NROW, 4>(role, cfg.block, v, sel, skip, write, s);
            case 8: return launch_role64<NROW, 8>(role, cfg.block, v, sel, skip, write, s);
        }
    } else {
        switch (cfg.rpt) {
            case 1: return launch_role<float, NROW, 1>(role, cfg.block, v, sel, skip, write, s);
            case 2: return launch_role<float, NROW, 2>(role, cfg.block, v, sel, skip, write, s);
            case 4: return launch_role<float, NROW, 4>(role, cfg.block, v, sel, skip, write, s);
            case 8: return launch_role<float, NROW, 8>(role, cfg.block, v, sel, skip, write, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_bdslash(bool dbl, int nrow, BDslashCfg cfg, BView v, int role, int sel, int skip_done, int write,
                          hipStream_t s) {
    if (v.ntiles <= 0) return hipSuccess;
    if (cfg.block != 64 && cfg.block != 128 && cfg.block != 256) return hipErrorInvalidValue;
    return nrow == 2 ? launch_nrow<2>(dbl, cfg, v, role, sel, skip_done, write, s)
                     : launch_nrow<3>(dbl, cfg, v, role, sel, skip_done, write, s);
}

}  // namespace stag
