// Batched shifted CG: the multi-RHS half-Dslash and the iteration driver.
//
// Many systems (pseudo-fermions x shifts, and lattices of different sizes)
// advance together.  Per iteration:
//  * the two half-Dslash launches run per lattice, one lane per site, each
//    lane loading its 8 links once for up to 8 right-hand sides (the systems
//    of that lattice); the per-system pointers and scalars travel in the
//    kernel arguments;
//  * the vector updates and the scalar recursions run once for all systems
//    (grid.y = system, or one workgroup per system), whatever their lattice;
//  * the double precision residual work (reliable updates, true residuals,
//    warm starts) is rare and uses the single-system kernels.
// Everything is enqueued on the caller's stream in chunks of iterations; a
// 4-byte "all systems done" flag is read one chunk behind.  The launch shape
// of the multi-RHS Dslash (sites per block, right-hand sides per launch) is
// timed on the first batch of each layout and cached.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "batch.h"
#include "links.h"
#include "ms_device.h"

namespace stag {

// Arguments of one multi-RHS half-Dslash launch on one lattice.
struct BDArgs {
    Geom g;
    const void *links;
    int nrhs;
    unsigned link_cache;         // 8-real double precision links: blocks read with ordinary loads
    const void *in[kMaxRpt];     // OE: p_base; EO: t
    void *out[kMaxRpt];          // OE: t; EO: ap
    const void *aux[kMaxRpt];    // EO: p_base; RESID: x
    const void *rhs[kMaxRpt];    // RESID: b
    double c[kMaxRpt];           // EO: m^2 + sigma_base; RESID: m^2 + sigma
    double *part[kMaxRpt];       // EO: one partial of <p, ap> per 64 consecutive sites
    int nchunk[kMaxRpt];         // partials of each system (ceil(V/2 / 64))
    const int *done[kMaxRpt];    // a system whose solve ended is skipped (null: never)
};

// OE: t = D_oe p; EO: q = c p - D_eo t with <p, q> partials; RESID: r = b - (c x - D_eo t)
// with |r|^2 partials (double precision; r stored only where out is non-null)
enum BDRole { BD_OE = 0, BD_EO = 1, BD_RESID = 2 };

// Link `blk` of site i: the 8-real double precision field honours the
// lattice's Infinity Cache blocks (link_cache_mask), the other layouts stream
// or cache as their loads do.
template <typename R, int NROW>
__device__ __forceinline__ su3<R> bd_link(const BDArgs &a, int vh, int blk, int i) {
    if constexpr (NROW == 1 && sizeof(R) == sizeof(double))
        return LinkLayout<double, 1>::load(a.links, vh, blk, i, (a.link_cache >> blk) & 1);
    else
        return LinkLayout<R, NROW>::load(a.links, vh, blk, i);
}

// The multi-RHS half-Dslash of one workgroup: `tile` numbers the group of
// blockDim.x consecutive output sites it covers.
template <typename R, int NROW, int RPT, int ROLE>
__device__ __forceinline__ void bd_tile(const BDArgs &a, int tile) {
    const int vh = a.g.Vh;
    bool live[RPT];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        live[r] = r < a.nrhs && !(a.done[r] && *a.done[r]);
        any = any || live[r];
    }
    if (!any) return;
    const int p = ROLE == BD_OE ? 1 : 0;
    const int i = tile * blockDim.x + threadIdx.x;
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
        site_coords(a.g, p, i, x);
        auto hop = [&](int mu) {
            const int jf = site_nbr(a.g, i, x, mu, +1);
            const int jb = site_nbr(a.g, i, x, mu, -1);
            const su3<R> uf = bd_link<R, NROW>(a, vh, p * 4 + mu, i);
            const R sf = R(fwd_sign(a.g, x, mu));
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (live[r]) acc_mul(acc[r], sf, uf, load_vec<R>(a.in[r], vh, jf));
            const su3<R> ub = bd_link<R, NROW>(a, vh, (1 - p) * 4 + mu, jb);
            const R sb = R(-bwd_sign(a.g, x, mu));
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (live[r]) acc_mul_dag(acc[r], sb, ub, load_vec<R>(a.in[r], vh, jb));
        };
        if (NROW == 1) {   // 8-real links: one direction at a time (registers)
#pragma unroll 1
            for (int mu = 0; mu < 4; ++mu) hop(mu);
        } else {
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) hop(mu);
        }
        const R half = R(0.5);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!live[r]) continue;
            vec3<R> o;
            if (ROLE == BD_OE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) o.c[c] = half * acc[r].c[c];
            } else if (ROLE == BD_RESID) {
                const vec3<R> xv = load_vec<R>(a.aux[r], vh, i);
                const vec3<R> bv = load_vec<R>(a.rhs[r], vh, i);
                const R cc = R(a.c[r]);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    o.c[k] = bv.c[k] - (cc * xv.c[k] - half * acc[r].c[k]);
                    part[r] += double(o.c[k].re) * double(o.c[k].re) + double(o.c[k].im) * double(o.c[k].im);
                }
                if (a.out[r]) store_vec<R>(a.out[r], vh, i, o);
                continue;
            } else {
                const vec3<R> pv = load_vec<R>(a.aux[r], vh, i);
                const R cc = R(a.c[r]);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    o.c[k] = cc * pv.c[k] - half * acc[r].c[k];
                    part[r] += double(pv.c[k].re) * double(o.c[k].re) + double(pv.c[k].im) * double(o.c[k].im);
                }
            }
            store_vec<R>(a.out[r], vh, i, o);
        }
    }
    if (ROLE == BD_EO || ROLE == BD_RESID) {
        // one partial per 64 consecutive sites, whatever the block size
        const int chunk = (i - (threadIdx.x & (kWave - 1))) >> 6;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!live[r]) continue;
            const double w = wave_sum(part[r]);
            if ((threadIdx.x & (kWave - 1)) == 0 && chunk < a.nchunk[r]) a.part[r][chunk] = w;
        }
    }
}

template <typename R, int NROW, int RPT, int ROLE>
__global__ void __launch_bounds__(256) kb_dslash(BDArgs a) {
    bd_tile<R, NROW, RPT, ROLE>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Every lattice of a batch in one launch: group g (a lattice and up to RPT
// of its systems) owns workgroups [blk0[g], blk0[g+1]); each group's range
// starts at a multiple of 8, so the XCD-aware tile order holds inside it.
// The groups' arguments are read from device memory (written once per solve).
struct BDGroups {
    int ngroups;
    int blk0[kMaxBatch + 1];
};

template <typename R, int NROW, int RPT, int ROLE>
__global__ void __launch_bounds__(256) kb_dslash_multi(const BDArgs *groups, BDGroups m) {
    int g = 0;
    while (g + 1 < m.ngroups && (int)blockIdx.x >= m.blk0[g + 1]) ++g;
    const int local = (int)blockIdx.x - m.blk0[g];
    bd_tile<R, NROW, RPT, ROLE>(groups[g], xcd_tile(local, m.blk0[g + 1] - m.blk0[g]));
}

template <typename R, int NROW, int RPT>
static hipError_t bd_launch_rpt(int role, int block, const BDArgs &a, hipStream_t s) {
    const dim3 grid((a.g.Vh + block - 1) / block), blk(block);
    if (role == BD_OE) hipLaunchKernelGGL((kb_dslash<R, NROW, RPT, BD_OE>), grid, blk, 0, s, a);
    else if (role == BD_EO) hipLaunchKernelGGL((kb_dslash<R, NROW, RPT, BD_EO>), grid, blk, 0, s, a);
    else if (sizeof(R) == sizeof(double)) hipLaunchKernelGGL((kb_dslash<double, NROW, RPT, BD_RESID>), grid, blk, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename R, int NROW>
static hipError_t bd_launch_nrow(int role, BDslashCfg cfg, const BDArgs &a, hipStream_t s) {
    switch (cfg.rpt) {
        case 1: return bd_launch_rpt<R, NROW, 1>(role, cfg.block, a, s);
        case 2: return bd_launch_rpt<R, NROW, 2>(role, cfg.block, a, s);
        case 4: return bd_launch_rpt<R, NROW, 4>(role, cfg.block, a, s);
        case 8: return bd_launch_rpt<R, NROW, 8>(role, cfg.block, a, s);
    }
    return hipErrorInvalidValue;
}

static hipError_t bd_launch(bool dbl, int nrow, int role, BDslashCfg cfg, const BDArgs &a, hipStream_t s) {
    if (a.nrhs < 1 || a.nrhs > cfg.rpt || a.nrhs > kMaxRpt) return hipErrorInvalidValue;
    if (cfg.block != 64 && cfg.block != 128 && cfg.block != 256) return hipErrorInvalidValue;
    if (dbl) {
        if (nrow == kHiLo + 2) return bd_launch_nrow<double, kHiLo + 2>(role, cfg, a, s);
        if (nrow == kHiLo + 3) return bd_launch_nrow<double, kHiLo + 3>(role, cfg, a, s);
        if (nrow == 1) return bd_launch_nrow<double, 1>(role, cfg, a, s);
        return nrow == 2 ? bd_launch_nrow<double, 2>(role, cfg, a, s) : bd_launch_nrow<double, 3>(role, cfg, a, s);
    }
    nrow = nrow_single(nrow);   // a float-pair field: its hi half
    if (nrow == 1) return bd_launch_nrow<float, 1>(role, cfg, a, s);
    return nrow == 2 ? bd_launch_nrow<float, 2>(role, cfg, a, s) : bd_launch_nrow<float, 3>(role, cfg, a, s);
}

template <typename R, int NROW, int RPT>
static hipError_t bdm_launch_rpt(int role, int block, const BDArgs *groups, const BDGroups &m, hipStream_t s) {
    const dim3 grid(m.blk0[m.ngroups]), blk(block);
    if (role == BD_OE) hipLaunchKernelGGL((kb_dslash_multi<R, NROW, RPT, BD_OE>), grid, blk, 0, s, groups, m);
    else hipLaunchKernelGGL((kb_dslash_multi<R, NROW, RPT, BD_EO>), grid, blk, 0, s, groups, m);
    return hipGetLastError();
}

template <typename R, int NROW>
static hipError_t bdm_launch_nrow(int role, BDslashCfg cfg, const BDArgs *groups, const BDGroups &m, hipStream_t s) {
    switch (cfg.rpt) {
        case 1: return bdm_launch_rpt<R, NROW, 1>(role, cfg.block, groups, m, s);
        case 2: return bdm_launch_rpt<R, NROW, 2>(role, cfg.block, groups, m, s);
        case 4: return bdm_launch_rpt<R, NROW, 4>(role, cfg.block, groups, m, s);
        case 8: return bdm_launch_rpt<R, NROW, 8>(role, cfg.block, groups, m, s);
    }
    return hipErrorInvalidValue;
}

// One launch for every group of the batch (roles OE and EO).
static hipError_t bdm_launch(bool dbl, int nrow, int role, BDslashCfg cfg, const BDArgs *groups, const BDGroups &m,
                             hipStream_t s) {
    if (m.ngroups < 1 || m.ngroups > kMaxBatch || role == BD_RESID) return hipErrorInvalidValue;
    if (cfg.block != 64 && cfg.block != 128 && cfg.block != 256) return hipErrorInvalidValue;
    if (dbl) {
        if (nrow == kHiLo + 2) return bdm_launch_nrow<double, kHiLo + 2>(role, cfg, groups, m, s);
        if (nrow == kHiLo + 3) return bdm_launch_nrow<double, kHiLo + 3>(role, cfg, groups, m, s);
        if (nrow == 1) return bdm_launch_nrow<double, 1>(role, cfg, groups, m, s);
        return nrow == 2 ? bdm_launch_nrow<double, 2>(role, cfg, groups, m, s)
                         : bdm_launch_nrow<double, 3>(role, cfg, groups, m, s);
    }
    nrow = nrow_single(nrow);
    if (nrow == 1) return bdm_launch_nrow<float, 1>(role, cfg, groups, m, s);
    return nrow == 2 ? bdm_launch_nrow<float, 2>(role, cfg, groups, m, s)
                     : bdm_launch_nrow<float, 3>(role, cfg, groups, m, s);
}

// D_oe of n double precision even-site vectors of one lattice, rpt (1, 2,
// 4 or 8) per launch (the links read once for all of them).
hipError_t launch_dslash_oe_multi(const stag_lattice *lat, int n, const void *const *in, void *const *out, int block,
                                  int rpt, hipStream_t s) {
    if (rpt != 1 && rpt != 2 && rpt != 4 && rpt != 8) return hipErrorInvalidValue;
    for (int k0 = 0; k0 < n; k0 += rpt) {
        BDArgs a;
        std::memset(&a, 0, sizeof(a));
        a.g = lat->g;
        a.links = lat->links64;
        a.link_cache = lat->link_cache;
        a.nrhs = n - k0 < rpt ? n - k0 : rpt;
        for (int r = 0; r < a.nrhs; ++r) {
            a.in[r] = in[k0 + r];
            a.out[r] = out[k0 + r];
        }
        const BDslashCfg cfg = {block, a.nrhs > 4 ? 8 : a.nrhs > 2 ? 4 : a.nrhs > 1 ? 2 : 1};
        const hipError_t e = bd_launch(true, lat->nrow, BD_OE, cfg, a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_true_resid_multi(const stag_lattice *lat, int n, const void *const *x, const double *c,
                                   const void *b, void *const *t, double *const *part, int block, hipStream_t s) {
    const int nchunk = (int)((lat->Vh + kWave - 1) / kWave);
    for (int k0 = 0; k0 < n; k0 += kMaxRpt) {
        BDArgs oe;
        std::memset(&oe, 0, sizeof(oe));
        oe.g = lat->g;
        oe.links = lat->links64;
        oe.link_cache = lat->link_cache;
        oe.nrhs = n - k0 < kMaxRpt ? n - k0 : kMaxRpt;
        BDArgs rs = oe;
        for (int r = 0; r < oe.nrhs; ++r) {
            oe.in[r] = x[k0 + r];
            oe.out[r] = t[r];
            rs.in[r] = t[r];
            rs.aux[r] = x[k0 + r];
            rs.rhs[r] = b;
            rs.c[r] = c[k0 + r];
            rs.part[r] = part[k0 + r];
            rs.nchunk[r] = nchunk;
        }
        const BDslashCfg cfg = {block, oe.nrhs > 4 ? 8 : oe.nrhs > 2 ? 4 : oe.nrhs > 1 ? 2 : 1};
        hipError_t e = bd_launch(true, lat->nrow, BD_OE, cfg, oe, s);
        if (e == hipSuccess) e = bd_launch(true, lat->nrow, BD_RESID, cfg, rs, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------- launch-shape cache

static std::mutex g_tune_mu;
static std::map<std::string, BDslashCfg> g_tune;

// Launch shapes persist across processes when the environment variable
// STAG_AUTOTUNE_CACHE names a file: one line per layout,
// "<layout key>\t<sites per block>\t<right-hand sides per launch>".  A layout
// missing from the process cache is looked up there before it is timed; a
// newly timed one is appended.  Lines that do not parse, or name a shape the
// kernels do not have, are ignored.  (Callers hold g_tune_mu.)
static bool shape_ok(BDslashCfg c) {
    return (c.block == 64 || c.block == 128 || c.block == 256) && (c.rpt == 1 || c.rpt == 2 || c.rpt == 4 || c.rpt == 8);
}
static bool tune_file_lookup(const std::string &key, BDslashCfg *out) {
    const char *path = std::getenv("STAG_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char *t1 = std::strchr(line, '\t');
        if (!t1) continue;
        *t1 = 0;
        if (key != line) continue;
        BDslashCfg c = {0, 0};
        if (std::sscanf(t1 + 1, "%d\t%d", &c.block, &c.rpt) == 2 && shape_ok(c)) {
            *out = c;   // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}
static void tune_file_append(const std::string &key, BDslashCfg c) {
    const char *path = std::getenv("STAG_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s\t%d\t%d\n", key.c_str(), c.block, c.rpt);
    std::fclose(f);
}
static thread_local BDslashCfg g_last_cfg = {0, 0};

BDslashCfg last_batch_cfg() { return g_last_cfg; }

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

stag_status run_batched(const BSpec *spec, int nsys, const BOptions &opt, BOut *out, hipStream_t s) {
    if (nsys < 1 || nsys > kMaxBatch) return invalid("a batch holds 1..64 systems");
    const bool dbl = opt.dbl;
    const bool any_init = std::any_of(spec, spec + nsys, [](const BSpec &p) { return p.x_init; });
    const bool all_init = std::all_of(spec, spec + nsys, [](const BSpec &p) { return p.x_init; });
    if (any_init && !all_init) return invalid("a batch is either all zero-start or all warm-start");
    for (int k = 0; k < nsys; ++k) {
        if (spec[k].x_init && spec[k].n != 1) return invalid("a warm-started system has exactly one shift");
        if (spec[k].rat_out && (!opt.dbl || spec[k].x_init))
            return invalid("rational applications run in double precision from a zero start");
    }

    // ---- lattices and their systems
    std::vector<stag_lattice *> lats;
    std::vector<std::vector<int>> members;
    std::vector<int> sys_lat(nsys);
    for (int k = 0; k < nsys; ++k) {
        int li = -1;
        for (size_t l = 0; l < lats.size(); ++l)
            if (lats[l] == spec[k].lat) li = (int)l;
        if (li < 0) {
            lats.push_back(spec[k].lat);
            members.emplace_back();
            li = (int)lats.size() - 1;
        }
        members[li].push_back(k);
        sys_lat[k] = li;
    }
    const int nlat = (int)lats.size();
    const int nrow = lats[0]->nrow;
    for (int l = 1; l < nlat; ++l)
        if (lats[l]->nrow != nrow) return invalid("all lattices of a batch must use the same link format");

    // ---- deferred shift updates for multi-shift systems from a zero start
    // (blocks of kDefer iterations; in single precision the reliable-update
    // checks fall on the block ends)
    const int dlen_all = kDefer;
    if (!dbl && opt.reliable_every > 0 && opt.reliable_every % dlen_all != 0)
        return invalid("reliable updates must fall on deferred passes");
    auto dlen_of = [&](int k) {
        return ((spec[k].n >= 2 && !spec[k].x_init) || spec[k].rat_out) ? dlen_all : 0;
    };

    // ---- work arena (carved from the first lattice's handle)
    int max_ds = 1;   // partials of the single-system residual and dot kernels
    for (int l = 0; l < nlat; ++l)
        max_ds = std::max(max_ds, std::max(dslash_grid(lats[l]->g, kDslashBlock), blas_grid(3 * (int64_t)lats[l]->Vh)));
    size_t bytes = al256(sizeof(BLat) * nlat) + al256(sizeof(BSys) * nsys) + al256(sizeof(MsState) * nsys) + 256 +
                   al256(sizeof(BDArgs) * 2 * kMaxBatch);
    for (int k = 0; k < nsys; ++k) {
        const int64_t vh = spec[k].lat->Vh;
        const size_t vb = (size_t)(dbl ? 48 : 24) * vh, v64 = (size_t)48 * vh;
        const int nds = (int)((vh + 63) / 64), nbl = (int)((3 * vh + kBChunk - 1) / kBChunk);
        size_t b = al256(sizeof(double) * nds) + al256(sizeof(double) * nbl) + al256(sizeof(double) * max_ds);
        b += 3 * al256(vb) + 2 * al256(v64) + spec[k].n * al256(vb);
        if (!dbl) b += spec[k].n * al256(vb);
        if (dlen_of(k)) b += dlen_of(k) * al256(vb) + al256(vb) + al256(sizeof(DeferHist));
        bytes += b;
    }
    void *arena = nullptr;
    STAG_TRY(ws_get(lats[0], WS_BATCH, bytes, &arena));
    char *cur = static_cast<char *>(arena);
    auto take = [&](size_t n) {
        char *p = cur;
        cur += al256(n);
        return p;
    };
    BLat *d_lat = reinterpret_cast<BLat *>(take(sizeof(BLat) * nlat));
    BSys *d_sys = reinterpret_cast<BSys *>(take(sizeof(BSys) * nsys));
    MsState *d_st = reinterpret_cast<MsState *>(take(sizeof(MsState) * nsys));
    int *d_flag = reinterpret_cast<int *>(take(256));
    BDArgs *d_groups = reinterpret_cast<BDArgs *>(take(sizeof(BDArgs) * 2 * kMaxBatch));

    std::vector<BLat> h_lat(nlat);
    for (int l = 0; l < nlat; ++l) {
        std::memset(&h_lat[l], 0, sizeof(BLat));
        h_lat[l].g = lats[l]->g;
        h_lat[l].nrow = nrow;
        h_lat[l].links = dbl ? lats[l]->links64 : lats[l]->links32;
        h_lat[l].links64 = lats[l]->links64;
    }
    std::vector<BSys> h_sys(nsys);
    std::vector<MsState> h_st(nsys);
    std::vector<double *> pres(nsys);   // per-system partials of the single-system residual kernels
    int max_n = 0, max_blocks = 1;
    for (int k = 0; k < nsys; ++k) {
        const BSpec &sp = spec[k];
        BSys &y = h_sys[k];
        std::memset(&y, 0, sizeof(BSys));
        const int64_t vh = sp.lat->Vh;
        const size_t vb = (size_t)(dbl ? 48 : 24) * vh, v64 = (size_t)48 * vh;
        y.lat = sys_lat[k];
        y.n = sp.n;
        y.base = 0;
        for (int i = 1; i < sp.n; ++i)
            if (sp.shifts[i] < sp.shifts[y.base]) y.base = i;
        y.nchunk_ds = (int)((vh + 63) / 64);
        y.nchunk_bl = (int)((3 * vh + kBChunk - 1) / kBChunk);
        y.x_init = sp.x_init ? 1 : 0;
        y.dlen = dlen_of(k);
        y.m2 = sp.mass * sp.mass;
        for (int i = 0; i < sp.n; ++i) y.shifts[i] = sp.shifts[i];
        y.st = d_st + k;
        y.part_ds = reinterpret_cast<double *>(take(sizeof(double) * y.nchunk_ds));
        y.part_bl = reinterpret_cast<double *>(take(sizeof(double) * y.nchunk_bl));
        pres[k] = reinterpret_cast<double *>(take(sizeof(double) * max_ds));
        y.src = static_cast<const double2 *>(sp.src);
        y.r = take(vb);
        y.ap = take(vb);
        y.t = take(vb);
        y.t64 = reinterpret_cast<double2 *>(take(v64));
        y.rhi = reinterpret_cast<double2 *>(take(v64));
        for (int i = 0; i < sp.n; ++i) {
            y.p[i] = take(vb);
            if (sp.rat_out) continue;   // no solution vectors
            y.xhi[i] = static_cast<double2 *>(sp.sols[i]);
            y.x[i] = dbl ? sp.sols[i] : take(vb);
        }
        y.rat = sp.rat_out ? 1 : 0;
        y.out = static_cast<double2 *>(sp.rat_out);
        y.w0 = sp.rat_w0;
        if (y.dlen) {
            y.ring = take((size_t)y.dlen * al256(vb));
            y.pd = take(vb);
            y.hist = reinterpret_cast<DeferHist *>(take(sizeof(DeferHist)));
        }
        MsState &st = h_st[k];
        std::memset(&st, 0, sizeof(MsState));
        st.n = sp.n;
        st.base = y.base;
        st.tol = opt.tol;
        st.max_iter = opt.max_iter;
        st.rel_delta2 = (!dbl && opt.reliable_every > 0) ? 0.01 : 0.0;
        st.hist = y.hist;   // emptied by the start step
        st.rat = y.rat;
        if (y.rat)
            for (int i = 0; i < sp.n; ++i) st.wgt[i] = sp.rat_w[i];
        for (int i = 0; i < sp.n; ++i) st.shift_rel[i] = sp.shifts[i] - sp.shifts[y.base];
        max_n = std::max(max_n, sp.n);
        max_blocks = std::max(max_blocks, (y.nchunk_bl + kBBlock / kWave - 1) / (kBBlock / kWave));
    }
    STAG_HIP(hipMemcpyAsync(d_lat, h_lat.data(), sizeof(BLat) * nlat, hipMemcpyHostToDevice, s));
    STAG_HIP(hipMemcpyAsync(d_sys, h_sys.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, s));
    STAG_HIP(hipMemcpyAsync(d_st, h_st.data(), sizeof(MsState) * nsys, hipMemcpyHostToDevice, s));
    // the host copies must stay valid until the copies ran
    STAG_HIP(hipStreamSynchronize(s));

    BView v;
    std::memset(&v, 0, sizeof(v));
    v.lats = d_lat;
    v.sys = d_sys;
    v.nsys = nsys;

    // b - (M + shift_i) x_i of system k in double precision, single-system kernels
    auto residual = [&](int k, int i, void *rout, const int *skip, hipStream_t s) -> hipError_t {
        stag_lattice *lat = spec[k].lat;
        DslashArgs d;
        std::memset(&d, 0, sizeof(d));
        d.g = lat->g;
        d.links = lat->links64;
        d.link_cache = lat->link_cache;
        d.skip = skip;
        d.out_parity = 1;
        d.in = h_sys[k].xhi[i];
        d.out = h_sys[k].t64;
        hipError_t e = launch_dslash(true, nrow, DS_PLAIN, d, s);
        if (e != hipSuccess) return e;
        d.out_parity = 0;
        d.in = h_sys[k].t64;
        d.out = rout;
        d.aux = h_sys[k].xhi[i];
        d.rhs = spec[k].src;
        d.c = h_sys[k].m2 + spec[k].shifts[i];
        d.partial = pres[k];
        return launch_dslash(true, nrow, DS_RESID, d, s);
    };

    // ---- start
    if (all_init) {
        for (int k = 0; k < nsys; ++k) STAG_HIP(residual(k, 0, h_sys[k].rhi, nullptr, s));
        STAG_HIP(launch_bvec(dbl, v, BV_RESTART, max_blocks, s));
        STAG_HIP(launch_bvec(dbl, v, BV_NORM_SRC, max_blocks, s));
        for (int k = 0; k < nsys; ++k)
            STAG_HIP(launch_scalar_init(d_st + k, pres[k], dslash_grid(spec[k].lat->g, kDslashBlock),
                                        h_sys[k].part_bl, h_sys[k].nchunk_bl, s));
    } else {
        STAG_HIP(launch_bvec(dbl, v, BV_START, max_blocks, s));
        STAG_HIP(launch_bvec(dbl, v, BV_NORM_SRC, max_blocks, s));
        STAG_HIP(launch_btail(v, BT_INIT, s));
    }

    // ---- multi-RHS Dslash arguments: per lattice, groups of at most 8 systems
    auto make_args = [&](int l, const std::vector<int> &grp, int role) {
        BDArgs a;
        std::memset(&a, 0, sizeof(a));
        a.g = lats[l]->g;
        a.links = h_lat[l].links;
        a.link_cache = dbl ? lats[l]->link_cache : 0u;
        a.nrhs = (int)grp.size();
        for (size_t r = 0; r < grp.size(); ++r) {
            const int k = grp[r];
            const BSys &y = h_sys[k];
            a.done[r] = &d_st[k].done;
            a.nchunk[r] = y.nchunk_ds;
            void *dir = y.dlen ? y.pd : y.p[y.base];   // the base direction
            if (role == BD_OE) {
                a.in[r] = dir;
                a.out[r] = y.t;
            } else {
                a.in[r] = y.t;
                a.out[r] = y.ap;
                a.aux[r] = dir;
                a.c[r] = y.m2 + y.shifts[y.base];
                a.part[r] = y.part_ds;
            }
        }
        return a;
    };
    auto groups_of = [&](int l, int rpt) {
        std::vector<std::vector<int>> gs;
        const std::vector<int> &m = members[l];
        for (size_t k0 = 0; k0 < m.size(); k0 += rpt)
            gs.emplace_back(m.begin() + k0, m.begin() + std::min(m.size(), k0 + (size_t)rpt));
        return gs;
    };

    // ---- launch shape per lattice: cached, else timed on this batch (t = D_oe p)
    std::vector<BDslashCfg> cfg(nlat);
    for (int l = 0; l < nlat; ++l) {
        const stag_lattice *lat = lats[l];
        std::ostringstream key;
        key << (dbl ? "f64" : "f32") << " nrow" << nrow << " " << lat->dims[0] << "x" << lat->dims[1] << "x"
            << lat->dims[2] << "x" << lat->dims[3] << ":" << members[l].size();
        BDslashCfg c = {0, 0};
        if (opt.force_block && opt.force_rpt) {
            c = {opt.force_block, opt.force_rpt};
        } else {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key.str());
            if (it != g_tune.end()) c = it->second;
            else if (tune_file_lookup(key.str(), &c)) g_tune[key.str()] = c;
        }
        if (!c.block) {
            hipEvent_t e0, e1;
            STAG_HIP(hipEventCreate(&e0));
            STAG_HIP(hipEventCreate(&e1));
            float best = 1e30f;
            const size_t ns = members[l].size();
            for (int rpt : {1, 2, 4, 8}) {
                if (rpt > 1 && (size_t)rpt / 2 >= ns) continue;
                for (int blk : {64, 128, 256}) {
                    const BDslashCfg cc = {blk, rpt};
                    const auto gs = groups_of(l, rpt);
                    for (int w = 0; w < 7; ++w) {
                        if (w == 2) STAG_HIP(hipEventRecord(e0, s));
                        for (const auto &grp : gs) STAG_HIP(bd_launch(dbl, nrow, BD_OE, cc, make_args(l, grp, BD_OE), s));
                    }
                    STAG_HIP(hipEventRecord(e1, s));
                    STAG_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    STAG_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best) {
                        best = ms;
                        c = cc;
                    }
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key.str()] = c;
            tune_file_append(key.str(), c);
            stag_log(1, "batched: launch shape of %s timed: %d sites per block, %d right-hand sides", key.str().c_str(),
                     c.block, c.rpt);
        }
        cfg[l] = c;
    }
    g_last_cfg = cfg[0];
    std::vector<std::vector<std::pair<BDArgs, BDArgs>>> args(nlat);
    int ngroups = 0;
    for (int l = 0; l < nlat; ++l)
        for (const auto &grp : groups_of(l, cfg[l].rpt)) {
            args[l].push_back({make_args(l, grp, BD_OE), make_args(l, grp, BD_EO)});
            ++ngroups;
        }

    // ---- one launch per phase for all lattices: every group gets its own
    // range of workgroups (a multiple of 8 each), the groups' arguments go
    // to device memory once; the right-hand sides per thread are the largest
    // of the lattices' tuned values, the block size is timed on this layout
    const bool merged = opt.merge_lattices && nlat > 1;
    BDGroups mg;
    std::memset(&mg, 0, sizeof(mg));
    BDslashCfg mcfg = {0, 0};
    std::vector<BDArgs> h_groups;
    if (merged) {
        if (ngroups > kMaxBatch) return invalid("too many multi-RHS groups");
        for (int l = 0; l < nlat; ++l) {
            mcfg.rpt = std::max(mcfg.rpt, cfg[l].rpt);
            for (const auto &pa : args[l]) h_groups.push_back(pa.first);
        }
        for (int l = 0; l < nlat; ++l)
            for (const auto &pa : args[l]) h_groups.push_back(pa.second);
        STAG_HIP(hipMemcpyAsync(d_groups, h_groups.data(), sizeof(BDArgs) * h_groups.size(), hipMemcpyHostToDevice,
                                s));
        STAG_HIP(hipStreamSynchronize(s));   // h_groups must outlive the copy
        mg.ngroups = ngroups;
        auto layout = [&](int block) {
            int g = 0;
            mg.blk0[0] = 0;
            for (int l = 0; l < nlat; ++l)
                for (size_t k = 0; k < args[l].size(); ++k, ++g) {
                    const int nb = (lats[l]->g.Vh + block - 1) / block;
                    mg.blk0[g + 1] = mg.blk0[g] + ((nb + 7) & ~7);
                }
        };
        std::ostringstream key;
        key << "multi " << (dbl ? "f64" : "f32") << " nrow" << nrow << " rpt" << mcfg.rpt;
        for (int l = 0; l < nlat; ++l)
            key << " " << lats[l]->dims[0] << "x" << lats[l]->dims[1] << "x" << lats[l]->dims[2] << "x"
                << lats[l]->dims[3] << ":" << members[l].size();
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key.str());
            if (it != g_tune.end()) mcfg = it->second;
            else if (tune_file_lookup(key.str(), &mcfg)) g_tune[key.str()] = mcfg;
        }
        if (opt.force_block) mcfg.block = opt.force_block;
        if (!mcfg.block) {
            hipEvent_t e0, e1;
            STAG_HIP(hipEventCreate(&e0));
            STAG_HIP(hipEventCreate(&e1));
            float best = 1e30f;
            for (int blk : {64, 128, 256}) {
                layout(blk);
                const BDslashCfg cc = {blk, mcfg.rpt};
                for (int w = 0; w < 7; ++w) {
                    if (w == 2) STAG_HIP(hipEventRecord(e0, s));
                    STAG_HIP(bdm_launch(dbl, nrow, BD_OE, cc, d_groups, mg, s));
                }
                STAG_HIP(hipEventRecord(e1, s));
                STAG_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                STAG_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    mcfg.block = blk;
                }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key.str()] = mcfg;
            tune_file_append(key.str(), mcfg);
            stag_log(1, "batched: launch shape of %s timed: %d sites per block", key.str().c_str(), mcfg.block);
        }
        layout(mcfg.block);
    }

    // ---- iterations
    bool any_defer = false, all_defer = true;
    for (int k = 0; k < nsys; ++k) {
        any_defer = any_defer || h_sys[k].dlen > 0;
        all_defer = all_defer && h_sys[k].dlen > 0;
    }
    const bool use_rel = !dbl && opt.reliable_every > 0;
    const int check = use_rel ? opt.reliable_every : 0;
    auto iteration = [&](int it, hipStream_t s) -> hipError_t {
        hipError_t e = hipSuccess;
        if (merged) {
            e = bdm_launch(dbl, nrow, BD_OE, mcfg, d_groups, mg, s);
            if (e == hipSuccess) e = bdm_launch(dbl, nrow, BD_EO, mcfg, d_groups + ngroups, mg, s);
            if (e != hipSuccess) return e;
        } else {
            for (int l = 0; l < nlat && e == hipSuccess; ++l)
                for (const auto &pa : args[l]) {
                    e = bd_launch(dbl, nrow, BD_OE, cfg[l], pa.first, s);
                    if (e != hipSuccess) return e;
                    e = bd_launch(dbl, nrow, BD_EO, cfg[l], pa.second, s);
                    if (e != hipSuccess) return e;
                }
        }
        if (all_defer) {
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_R_UPDATE_FUSED, max_blocks, s, it);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_DIR_FUSED, max_blocks, s, it);
        } else {
            if (e == hipSuccess) e = launch_btail(v, BT_ALPHA, s);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_R_UPDATE, max_blocks, s, it);
            if (e == hipSuccess) e = launch_btail(v, BT_BETA, s);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_SHIFT_UPDATE, max_blocks, s, it);
        }
        if (e == hipSuccess && any_defer && (it + 1) % dlen_all == 0) {
            e = launch_bdefer_coef(v, s);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_DEFER_APPLY, max_blocks, s, it);
        }
        if (e == hipSuccess && check > 0 && (it + 1) % check == 0) {
            // reliable update of every system whose residual fell tenfold since its last one
            e = launch_bvec(dbl, v, BV_FLUSH, max_blocks, s);
            for (int k = 0; k < nsys && e == hipSuccess; ++k) {
                e = residual(k, h_sys[k].base, h_sys[k].rhi, &d_st[k].rel_skip, s);
                if (e == hipSuccess)
                    e = launch_reduce_tail(d_st + k, pres[k], dslash_grid(spec[k].lat->g, kDslashBlock), TAIL_RELIABLE,
                                           0, s);
            }
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_DEMOTE, max_blocks, s, it);
        }
        return e;
    };
    // Every kernel of an iteration depends on the iteration index only
    // through it mod kDefer (ring slots, deferred passes, reliable-update
    // checks every kDefer iterations), so one block of kDefer iterations,
    // captured once as a graph, is replayed for every block of the solve.
    // The capture runs on a private stream (nothing executes there); the
    // replays run on the caller's stream, which is drained before the
    // executable is destroyed.
    const int period = kDefer;
    if (check > 0 && check != period) return invalid("reliable updates must come every kDefer iterations");
    struct GraphExec {
        hipGraphExec_t exec = nullptr;
        hipStream_t replay = nullptr;
        ~GraphExec() {
            if (exec) {
                (void)hipStreamSynchronize(replay);
                (void)hipGraphExecDestroy(exec);
            }
        }
    } graph;
    graph.replay = s;
    if (opt.use_graph) {
        hipStream_t cs = nullptr;
        STAG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int k = 0; k < period && e == hipSuccess; ++k) e = iteration(k, cs);
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            graph.exec = nullptr;
            set_error(std::string("capture of the batched iterations failed: ") + hipGetErrorString(e));
            return STAG_EHIP;
        }
    }
    volatile int *flags = lats[0]->host_flags;
    flags[0] = flags[1] = 0;
    hipEvent_t ev[2];
    STAG_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    STAG_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    const int K = graph.exec ? period : 8;
    stag_status rc = STAG_OK;
    for (int chunk = 0;; ++chunk) {
        hipError_t e = hipSuccess;
        if (graph.exec) e = hipGraphLaunch(graph.exec, s);
        else
            for (int k = 0; k < K && e == hipSuccess; ++k) e = iteration(chunk * K + k, s);
        if (e == hipSuccess) e = launch_ball_done(v, d_flag, s);
        const int slot = chunk & 1;
        if (e == hipSuccess)
            e = hipMemcpyAsync(const_cast<int *>(flags + slot), d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(ev[slot], s);
        if (e == hipSuccess && chunk > 0) {
            e = hipEventSynchronize(ev[slot ^ 1]);
            if (e == hipSuccess && flags[slot ^ 1]) break;
        }
        if (e != hipSuccess) {
            set_error(std::string("batched iteration failed: ") + hipGetErrorString(e));
            rc = STAG_EHIP;
            break;
        }
        if ((chunk + 1) * K > opt.max_iter + K) break;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc != STAG_OK) return rc;

    // ---- finish: the last deferred pass (the loop may end inside a block),
    // flush single precision accumulators, double precision true residuals
    if (any_defer) {
        STAG_HIP(launch_bdefer_coef(v, s));
        STAG_HIP(launch_bvec(dbl, v, BV_DEFER_APPLY, max_blocks, s));
    }
    if (!dbl) STAG_HIP(launch_bvec(dbl, v, BV_FLUSH_FINAL, max_blocks, s));
    for (int k = 0; k < nsys; ++k) {
        if (!spec[k].rat_out) continue;
        // no solutions are kept: Re <src, out> instead of true residuals
        const int64_t ne = 3 * spec[k].lat->Vh;
        const int g = blas_grid(ne);
        STAG_HIP(launch_dot_re(static_cast<const double2 *>(spec[k].src),
                               static_cast<const double2 *>(spec[k].rat_out), ne, pres[k], g, s));
        STAG_HIP(launch_reduce_tail(d_st + k, pres[k], g, TAIL_SCRATCH, 0, s));
    }
    // FP64 true residuals of every (system, shift): round i takes shift i of
    // every system that has one, through the multi-RHS kernels (links loaded
    // once for up to 8 systems of a lattice), then one tail for all systems
    for (int i = 0; i < max_n; ++i) {
        for (int l = 0; l < nlat; ++l) {
            std::vector<int> in_round;
            for (int k : members[l])
                if (!spec[k].rat_out && i < spec[k].n) in_round.push_back(k);
            const BDslashCfg rc8 = {cfg[l].block, 8};
            for (size_t k0 = 0; k0 < in_round.size(); k0 += 8) {
                BDArgs oe, eo;
                std::memset(&oe, 0, sizeof(oe));
                oe.g = lats[l]->g;
                oe.links = h_lat[l].links64;
                oe.link_cache = lats[l]->link_cache;
                oe.nrhs = (int)std::min<size_t>(8, in_round.size() - k0);
                eo = oe;
                for (int r = 0; r < oe.nrhs; ++r) {
                    const int k = in_round[k0 + r];
                    const BSys &y = h_sys[k];
                    oe.in[r] = y.xhi[i];
                    oe.out[r] = y.t64;
                    eo.in[r] = y.t64;
                    eo.out[r] = nullptr;
                    eo.aux[r] = y.xhi[i];
                    eo.rhs[r] = spec[k].src;
                    eo.c[r] = y.m2 + spec[k].shifts[i];
                    eo.part[r] = y.part_ds;
                    eo.nchunk[r] = y.nchunk_ds;
                }
                STAG_HIP(bd_launch(true, nrow, BD_OE, rc8, oe, s));
                STAG_HIP(bd_launch(true, nrow, BD_RESID, rc8, eo, s));
            }
        }
        STAG_HIP(launch_btail(v, BT_TRUE_RESID, s, i));
    }
    STAG_HIP(hipMemcpyAsync(h_st.data(), d_st, sizeof(MsState) * nsys, hipMemcpyDeviceToHost, s));
    STAG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nsys; ++k) {
        const MsState &st = h_st[k];
        BOut &o = out[k];
        o.status = st.status;
        o.dot = st.scratch[0];
        o.iters = st.iter;
        o.n_reliable = st.n_reliable;
        for (int i = 0; i < st.n; ++i) {
            o.iters_shift[i] = st.active[i] ? st.iter : st.iters_shift[i];
            o.resid_iter[i] = st.resid_iter[i];
            o.resid_true[i] = st.resid_true[i];
        }
    }
    return STAG_OK;
}

}  // namespace stag
