// Host driver of the batched shifted CG (pseudo-fermions x shifts and
// lattices of different sizes in one set of launches).
//
//  * Systems that share a lattice handle form a multi-RHS group; the Dslash
//    tile table gives each tile up to RPT systems of one group.
//  * The launch shape (sites per block, RHS per thread) is picked by timing
//    every candidate on the actual batch the first time a batch layout is
//    seen; the choice is cached per layout in the process and, when the
//    environment variable STAG_AUTOTUNE_CACHE names a file, on disk.
//  * Ten iterations (in mixed precision followed by a double precision
//    reliable update for every system whose residual fell tenfold since its
//    last one) are captured once in a hipGraph and replayed; after each replay a 4-byte "all systems done" flag is copied
//    to pinned host memory and read one replay behind, so the queue never
//    drains.  Kernels of systems that already finished return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "batch.h"
#include "links.h"

namespace stag {

static thread_local BDslashCfg g_last_cfg = {0, 0};
BDslashCfg last_batch_cfg() { return g_last_cfg; }

// ---------------------------------------------------------------- autotune cache
static std::mutex g_tune_mu;
static std::map<std::string, BDslashCfg> g_tune;
static bool g_tune_loaded = false;

static const char *tune_file() { return std::getenv("STAG_AUTOTUNE_CACHE"); }

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = tune_file();
    if (!f) return;
    std::ifstream in(f);
    std::string line;
    while (std::getline(in, line)) {
        const size_t a = line.find('\t');
        if (a == std::string::npos) continue;
        int b = 0, r = 0;
        if (std::sscanf(line.c_str() + a + 1, "%d %d", &b, &r) == 2) g_tune[line.substr(0, a)] = {b, r};
    }
}

static void tune_store_locked(const std::string &key, BDslashCfg c) {
    g_tune[key] = c;
    const char *f = tune_file();
    if (!f) return;
    std::ofstream out(f, std::ios::app);
    out << key << '\t' << c.block << ' ' << c.rpt << '\n';
}

// ---------------------------------------------------------------- layout

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Group {
    stag_lattice *lat;
    int lat_idx;
    std::vector<int> sys;
};

static std::vector<BTile> build_tiles(const std::vector<Group> &groups, BDslashCfg cfg) {
    std::vector<BTile> t;
    for (const Group &g : groups) {
        const int vh = (int)g.lat->Vh;
        const int nb = (vh + cfg.block - 1) / cfg.block;
        for (size_t s0 = 0; s0 < g.sys.size(); s0 += cfg.rpt) {
            for (int b = 0; b < nb; ++b) {
                BTile tile;
                std::memset(&tile, 0, sizeof(tile));
                tile.lat = g.lat_idx;
                tile.site0 = b * cfg.block;
                tile.nsys = (int)std::min<size_t>(cfg.rpt, g.sys.size() - s0);
                for (int r = 0; r < tile.nsys; ++r) tile.sys[r] = g.sys[s0 + r];
                t.push_back(tile);
            }
        }
    }
    return t;
}

static stag_status get_capture_stream(stag_lattice *lat, hipStream_t *cs) {
    if (!lat->capture_stream) STAG_HIP(hipStreamCreateWithFlags(&lat->capture_stream, hipStreamNonBlocking));
    *cs = lat->capture_stream;
    return STAG_OK;
}

stag_status run_batched(const BSpec *spec, int nsys, const BOptions &opt, BOut *out, hipStream_t user_stream) {
    if (nsys < 1 || nsys > kMaxBatch) return invalid("a batch holds 1..64 systems");
    const bool dbl = opt.dbl;
    stag_lattice *lat0 = spec[0].lat;

    // ---- groups of systems sharing a lattice
    std::vector<Group> groups;
    std::vector<int> sys_lat(nsys);
    for (int k = 0; k < nsys; ++k) {
        int gi = -1;
        for (size_t g = 0; g < groups.size(); ++g)
            if (groups[g].lat == spec[k].lat) gi = (int)g;
        if (gi < 0) {
            groups.push_back({spec[k].lat, (int)groups.size(), {}});
            gi = (int)groups.size() - 1;
        }
        groups[gi].sys.push_back(k);
        sys_lat[k] = gi;
    }
    const int nlat = (int)groups.size();
    size_t max_group = 0;
    for (const Group &g : groups) max_group = std::max(max_group, g.sys.size());

    // ---- work arena
    size_t max_tiles = 0;
    for (const Group &g : groups) max_tiles += (size_t)((g.lat->Vh + 63) / 64) * g.sys.size();
    size_t bytes = align256(sizeof(BLat) * nlat) + align256(sizeof(BSys) * nsys) + align256(sizeof(BTile) * max_tiles) +
                   align256(sizeof(MsState) * nsys) + 256;
    std::vector<size_t> sys_bytes(nsys);
    for (int k = 0; k < nsys; ++k) {
        const int64_t vh = spec[k].lat->Vh;
        const size_t vb = (size_t)(dbl ? 48 : 24) * vh, v64 = (size_t)48 * vh;
        const int nds = (int)((vh + 63) / 64), nbl = (int)((3 * vh + kBChunk - 1) / kBChunk);
        size_t b = align256(sizeof(double) * nds) + align256(sizeof(double) * nbl);
        b += 3 * align256(vb) + 2 * align256(v64) + spec[k].n * align256(vb);
        if (!dbl) b += spec[k].n * align256(vb);
        sys_bytes[k] = b;
        bytes += b;
    }
    void *arena = nullptr;
    STAG_TRY(ws_get(lat0, WS_BATCH, bytes, &arena));
    char *cur = static_cast<char *>(arena);
    auto take = [&](size_t n) {
        char *p = cur;
        cur += align256(n);
        return p;
    };
    BLat *d_lat = reinterpret_cast<BLat *>(take(sizeof(BLat) * nlat));
    BSys *d_sys = reinterpret_cast<BSys *>(take(sizeof(BSys) * nsys));
    BTile *d_tiles = reinterpret_cast<BTile *>(take(sizeof(BTile) * max_tiles));
    MsState *d_st = reinterpret_cast<MsState *>(take(sizeof(MsState) * nsys));
    int *d_flag = reinterpret_cast<int *>(take(256));

    std::vector<BLat> h_lat(nlat);
    for (int g = 0; g < nlat; ++g) {
        std::memset(&h_lat[g], 0, sizeof(BLat));
        h_lat[g].g = groups[g].lat->g;
        h_lat[g].nrow = groups[g].lat->nrow;
        h_lat[g].links = dbl ? groups[g].lat->links64 : groups[g].lat->links32;
        h_lat[g].links64 = groups[g].lat->links64;
    }
    const int nrow = h_lat[0].nrow;
    for (int g = 1; g < nlat; ++g)
        if (h_lat[g].nrow != nrow) return invalid("all lattices of a batch must use the same link format");

    std::vector<BSys> h_sys(nsys);
    std::vector<MsState> h_st(nsys);
    int max_n = 0, max_blocks = 1;
    for (int k = 0; k < nsys; ++k) {
        const BSpec &sp = spec[k];
        BSys &s = h_sys[k];
        std::memset(&s, 0, sizeof(BSys));
        const int64_t vh = sp.lat->Vh;
        const size_t vb = (size_t)(dbl ? 48 : 24) * vh, v64 = (size_t)48 * vh;
        s.lat = sys_lat[k];
        s.n = sp.n;
        s.base = 0;
        for (int i = 1; i < sp.n; ++i)
            if (sp.shifts[i] < sp.shifts[s.base]) s.base = i;
        s.nchunk_ds = (int)((vh + 63) / 64);
        s.nchunk_bl = (int)((3 * vh + kBChunk - 1) / kBChunk);
        s.x_init = sp.x_init ? 1 : 0;
        s.m2 = sp.mass * sp.mass;
        for (int i = 0; i < sp.n; ++i) s.shifts[i] = sp.shifts[i];
        s.st = d_st + k;
        s.part_ds = reinterpret_cast<double *>(take(sizeof(double) * s.nchunk_ds));
        s.part_bl = reinterpret_cast<double *>(take(sizeof(double) * s.nchunk_bl));
        s.src = static_cast<const double2 *>(sp.src);
        s.r = take(vb);
        s.ap = take(vb);
        s.t = take(vb);
        s.t64 = reinterpret_cast<double2 *>(take(v64));
        s.rhi = reinterpret_cast<double2 *>(take(v64));
        for (int i = 0; i < sp.n; ++i) {
            s.p[i] = take(vb);
            s.xhi[i] = static_cast<double2 *>(sp.sols[i]);
            s.x[i] = dbl ? sp.sols[i] : take(vb);
        }
        MsState &st = h_st[k];
        std::memset(&st, 0, sizeof(MsState));
        st.n = sp.n;
        st.base = s.base;
        st.tol = opt.tol;
        st.max_iter = opt.max_iter;
        st.rel_delta2 = (!dbl && opt.reliable_every > 0) ? 0.01 : 0.0;
        for (int i = 0; i < sp.n; ++i) st.shift_rel[i] = sp.shifts[i] - sp.shifts[s.base];
        max_n = std::max(max_n, sp.n);
        max_blocks = std::max(max_blocks, (s.nchunk_bl + kBBlock / kWave - 1) / (kBBlock / kWave));
    }

    hipStream_t cs;
    STAG_TRY(get_capture_stream(lat0, &cs));
    hipEvent_t e_in;
    STAG_HIP(hipEventCreateWithFlags(&e_in, hipEventDisableTiming));
    STAG_HIP(hipEventRecord(e_in, user_stream));
    STAG_HIP(hipStreamWaitEvent(cs, e_in, 0));
    hipEventDestroy(e_in);
    STAG_HIP(hipMemcpyAsync(d_lat, h_lat.data(), sizeof(BLat) * nlat, hipMemcpyHostToDevice, cs));
    STAG_HIP(hipMemcpyAsync(d_sys, h_sys.data(), sizeof(BSys) * nsys, hipMemcpyHostToDevice, cs));
    STAG_HIP(hipMemcpyAsync(d_st, h_st.data(), sizeof(MsState) * nsys, hipMemcpyHostToDevice, cs));

    BView v;
    v.lats = d_lat;
    v.sys = d_sys;
    v.tiles = d_tiles;
    v.ntiles = 0;
    v.nsys = nsys;

    // ---- start
    if (std::any_of(spec, spec + nsys, [](const BSpec &p) { return p.x_init; })) {
        for (int k = 0; k < nsys; ++k)
            if (spec[k].x_init && spec[k].n != 1) return invalid("a warm-started system has exactly one shift");
    }
    BDslashCfg cfg0 = {256, 1};
    std::vector<BTile> tiles = build_tiles(groups, cfg0);
    STAG_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(BTile) * tiles.size(), hipMemcpyHostToDevice, cs));
    v.ntiles = (int)tiles.size();
    const bool any_init = std::any_of(spec, spec + nsys, [](const BSpec &p) { return p.x_init; });
    const bool all_init = std::all_of(spec, spec + nsys, [](const BSpec &p) { return p.x_init; });
    if (any_init && !all_init) return invalid("a batch is either all zero-start or all warm-start");
    if (all_init) {
        STAG_HIP(launch_bdslash(dbl, nrow, cfg0, v, BR_OE_X, 0, 0, 0, cs));
        STAG_HIP(launch_bdslash(dbl, nrow, cfg0, v, BR_EO_RESID, 0, 0, 1, cs));
        STAG_HIP(launch_bvec(dbl, v, BV_RESTART, max_blocks, cs));
    } else {
        STAG_HIP(launch_bvec(dbl, v, BV_START, max_blocks, cs));
    }
    STAG_HIP(launch_bvec(dbl, v, BV_NORM_SRC, max_blocks, cs));
    STAG_HIP(launch_btail(v, BT_INIT, 0, cs));

    // ---- launch shape
    std::ostringstream key;
    key << (dbl ? "f64" : "f32") << " nrow" << nrow;
    for (const Group &g : groups)
        key << " " << g.lat->dims[0] << "x" << g.lat->dims[1] << "x" << g.lat->dims[2] << "x" << g.lat->dims[3] << ":"
            << g.sys.size();
    BDslashCfg cfg = {0, 0};
    if (opt.force_block && opt.force_rpt) {
        cfg = {opt.force_block, opt.force_rpt};
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key.str());
        if (it != g_tune.end()) cfg = it->second;
    }
    if (!cfg.block) {
        // time every candidate on this batch (t = D_oe p with p = the start vector)
        hipEvent_t a, b;
        STAG_HIP(hipEventCreate(&a));
        STAG_HIP(hipEventCreate(&b));
        float best = 1e30f;
        for (int rpt : {1, 2, 4, 8}) {
            if (rpt > 1 && (size_t)rpt / 2 >= max_group) continue;
            for (int blk : {64, 128, 256}) {
                BDslashCfg c = {blk, rpt};
                std::vector<BTile> tl = build_tiles(groups, c);
                STAG_HIP(hipMemcpyAsync(d_tiles, tl.data(), sizeof(BTile) * tl.size(), hipMemcpyHostToDevice, cs));
                BView tv = v;
                tv.ntiles = (int)tl.size();
                for (int w = 0; w < 2; ++w) STAG_HIP(launch_bdslash(dbl, nrow, c, tv, BR_OE_P, -1, 0, 0, cs));
                STAG_HIP(hipEventRecord(a, cs));
                for (int w = 0; w < 5; ++w) STAG_HIP(launch_bdslash(dbl, nrow, c, tv, BR_OE_P, -1, 0, 0, cs));
                STAG_HIP(hipEventRecord(b, cs));
                STAG_HIP(hipEventSynchronize(b));
                float ms = 0.f;
                STAG_HIP(hipEventElapsedTime(&ms, a, b));
                if (ms < best) {
                    best = ms;
                    cfg = c;
                }
            }
        }
        hipEventDestroy(a);
        hipEventDestroy(b);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key.str(), cfg);
    }
    g_last_cfg = cfg;
    tiles = build_tiles(groups, cfg);
    STAG_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(BTile) * tiles.size(), hipMemcpyHostToDevice, cs));
    v.ntiles = (int)tiles.size();

    // ---- iteration body
    const int K = 10;   // iterations per replay; divides the reliable-update interval
    auto enqueue = [&](bool reliable) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int k = 0; k < K && e == hipSuccess; ++k) {
            e = launch_bdslash(dbl, nrow, cfg, v, BR_OE_P, -1, 1, 0, cs);
            if (e == hipSuccess) e = launch_bdslash(dbl, nrow, cfg, v, BR_EO_AP, -1, 1, 0, cs);
            if (e == hipSuccess) e = launch_btail(v, BT_ALPHA, 0, cs);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_R_UPDATE, max_blocks, cs);
            if (e == hipSuccess) e = launch_btail(v, BT_BETA, 0, cs);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_SHIFT_UPDATE, max_blocks, cs);
        }
        if (reliable && e == hipSuccess) {
            e = launch_bvec(dbl, v, BV_FLUSH, max_blocks, cs);
            if (e == hipSuccess) e = launch_bdslash(dbl, nrow, cfg, v, BR_OE_X, -1, 2, 0, cs);
            if (e == hipSuccess) e = launch_bdslash(dbl, nrow, cfg, v, BR_EO_RESID, -1, 2, 1, cs);
            if (e == hipSuccess) e = launch_btail(v, BT_RELIABLE, 0, cs);
            if (e == hipSuccess) e = launch_bvec(dbl, v, BV_DEMOTE, max_blocks, cs);
        }
        if (e == hipSuccess) e = launch_ball_done(v, d_flag, cs);
        return e;
    };
    const bool use_rel = !dbl && opt.reliable_every > 0;
    hipGraphExec_t ge[2] = {nullptr, nullptr};
    hipGraph_t gr[2] = {nullptr, nullptr};
    stag_status rc = STAG_OK;
    if (opt.use_graph) {
        for (int g = 0; g < (use_rel ? 2 : 1) && rc == STAG_OK; ++g) {
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue(g == 1);
                e = hipStreamEndCapture(cs, &gr[g]);
                if (e == hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&ge[g], gr[g], nullptr, nullptr, 0);
            if (e != hipSuccess) {
                set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
                rc = STAG_EHIP;
            }
        }
    }
    volatile int *flags = lat0->host_flags;
    flags[0] = flags[1] = 0;
    hipEvent_t ev[2];
    if (rc == STAG_OK) {
        if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
            set_error("event creation failed");
            rc = STAG_EHIP;
        }
    }
    for (int chunk = 0; rc == STAG_OK; ++chunk) {
        const int it_end = (chunk + 1) * K;
        const bool rel = use_rel;   // every replay checks whether a reliable update is due
        hipError_t e = opt.use_graph ? hipGraphLaunch(ge[rel ? 1 : 0], cs) : enqueue(rel);
        const int slot = chunk & 1;
        if (e == hipSuccess) e = hipMemcpyAsync(const_cast<int *>(flags + slot), d_flag, sizeof(int), hipMemcpyDeviceToHost, cs);
        if (e == hipSuccess) e = hipEventRecord(ev[slot], cs);
        if (e == hipSuccess && chunk > 0) {
            e = hipEventSynchronize(ev[slot ^ 1]);
            if (e == hipSuccess && flags[slot ^ 1]) break;
        }
        if (e != hipSuccess) {
            set_error(std::string("batched iteration failed: ") + hipGetErrorString(e));
            rc = STAG_EHIP;
            break;
        }
        if (it_end > opt.max_iter + K) break;
    }
    // the last replay may still run: let it finish before its executable goes
    if (rc == STAG_OK && hipStreamSynchronize(cs) != hipSuccess) {
        set_error("batched iteration failed at the last replay");
        rc = STAG_EHIP;
    }
    if (rc == STAG_OK) {
        hipEventDestroy(ev[0]);
        hipEventDestroy(ev[1]);
    }
    for (int g = 0; g < 2; ++g) {
        if (ge[g]) hipGraphExecDestroy(ge[g]);
        if (gr[g]) hipGraphDestroy(gr[g]);
    }
    if (rc != STAG_OK) return rc;

    // ---- finish: flush single precision accumulators, double precision true residuals
    if (!dbl) STAG_HIP(launch_bvec(dbl, v, BV_FLUSH_FINAL, max_blocks, cs));
    for (int sel = 0; sel < max_n; ++sel) {
        STAG_HIP(launch_bdslash(dbl, nrow, cfg, v, BR_OE_X, sel, 0, 0, cs));
        STAG_HIP(launch_bdslash(dbl, nrow, cfg, v, BR_EO_RESID, sel, 0, 0, cs));
        STAG_HIP(launch_btail(v, BT_TRUE_RESID, sel, cs));
    }
    STAG_HIP(hipMemcpyAsync(h_st.data(), d_st, sizeof(MsState) * nsys, hipMemcpyDeviceToHost, cs));
    STAG_HIP(hipStreamSynchronize(cs));
    for (int k = 0; k < nsys; ++k) {
        const MsState &st = h_st[k];
        BOut &o = out[k];
        o.status = st.status;
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

static stag_status status_of_ms(int ms) {
    switch (ms) {
        case MS_CONVERGED: return STAG_OK;
        case MS_BREAKDOWN: set_error("non-positive or non-finite curvature <p, A p>"); return STAG_EBREAKDOWN;
        default: set_error("maximum number of iterations reached"); return STAG_ENOCONV;
    }
}

// Refine every (system, shift) whose double precision true residual exceeds
// tol: single-shift mixed CG from the current solution, all of them batched
// (systems on one lattice share link loads), repeated for the few that a
// pass leaves above tol.
stag_status refine_batched(const BSpec *spec, int nsys, const BOptions &opt, stag_cg_stats *stats, hipStream_t s) {
    struct Item {
        int k, i;
    };
    std::vector<Item> todo;
    for (int k = 0; k < nsys; ++k)
        for (int i = 0; i < spec[k].n; ++i)
            if (!(stats[k].resid_true[i] <= opt.tol)) todo.push_back({k, i});
    stag_status worst = STAG_OK;
    for (int pass = 0; pass < 4 && !todo.empty(); ++pass) {
        std::vector<Item> next;
        for (size_t c0 = 0; c0 < todo.size(); c0 += kMaxBatch) {
            const int m = (int)std::min<size_t>(kMaxBatch, todo.size() - c0);
            std::vector<BSpec> rs(m);
            std::vector<BOut> ro(m);
            for (int j = 0; j < m; ++j) {
                const Item &it = todo[c0 + j];
                rs[j] = spec[it.k];
                rs[j].n = 1;
                rs[j].shifts = spec[it.k].shifts + it.i;
                rs[j].sols = spec[it.k].sols + it.i;
                rs[j].x_init = true;
            }
            BOptions ro_opt = opt;
            ro_opt.dbl = false;
            ro_opt.reliable_every = 8;
            ro_opt.force_block = ro_opt.force_rpt = 0;
            STAG_TRY(run_batched2(rs.data(), m, ro_opt, ro.data(), s));
            for (int j = 0; j < m; ++j) {
                const Item &it = todo[c0 + j];
                stag_cg_stats &st = stats[it.k];
                st.refine_iters += ro[j].iters;
                st.refine_iters_shift[it.i] += ro[j].iters;
                st.n_reliable += ro[j].n_reliable;
                st.resid_true[it.i] = ro[j].resid_true[0];
                if (ro[j].status == MS_BREAKDOWN) worst = STAG_EBREAKDOWN;
                else if (!(ro[j].resid_true[0] <= opt.tol)) next.push_back(it);
            }
        }
        todo.swap(next);
    }
    if (worst == STAG_OK && !todo.empty()) worst = STAG_ENOCONV;
    if (worst != STAG_OK) status_of_ms(worst == STAG_EBREAKDOWN ? MS_BREAKDOWN : MS_NOCONV);
    return worst;
}

stag_status batched_solve(const BSpec *spec, int nsys, const BOptions &opt0, bool mixed, stag_cg_stats *stats,
                          hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    BOptions opt = opt0;
    std::vector<BOut> out(nsys);
    STAG_TRY(run_batched2(spec, nsys, opt, out.data(), s));
    stag_status rc = STAG_OK;
    for (int k = 0; k < nsys; ++k) {
        stag_cg_stats &st = stats[k];
        std::memset(&st, 0, sizeof(st));
        st.iters = out[k].iters;
        st.n_reliable = out[k].n_reliable;
        for (int i = 0; i < spec[k].n; ++i) {
            st.iters_shift[i] = out[k].iters_shift[i];
            st.resid_iter[i] = out[k].resid_iter[i];
            st.resid_true[i] = out[k].resid_true[i];
            st.resid_unrefined[i] = out[k].resid_true[i];
        }
        const stag_status sk = status_of_ms(out[k].status);
        if (sk == STAG_EBREAKDOWN || (sk != STAG_OK && rc == STAG_OK)) rc = sk;
    }
    if (mixed && rc != STAG_EBREAKDOWN) {
        const stag_status rr = refine_batched(spec, nsys, opt, stats, s);
        if (rr < 0) return rr;
        rc = rr;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nsys; ++k) stats[k].seconds = secs;
    return rc;
}

}  // namespace stag
