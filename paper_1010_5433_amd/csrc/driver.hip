// Host driver of the shifted CG family.
//
// One routine runs the multi-shift CG (zero start, Section 6: the shifted
// solver must start from the null vector) and the single-shift CG from a
// given x (used to refine single precision results).  The iteration is
// enqueued in chunks; all scalars stay on the device and the host only
// reads a 4-byte "done" flag per chunk, one chunk behind, so the GPU queue
// never drains while the host checks convergence.  Kernels enqueued after
// the solve ended see the flag and return at once.
//
// Precision policy (Section 4 and Section 6): STAG_F64 runs everything in
// double; STAG_F32 and STAG_MIXED run the operator and the vectors in
// single precision with double reductions and recursion, accumulating
// solutions in single precision and flushing them into the double
// solutions.  STAG_MIXED adds reliable updates: every `reliable_every`
// iterations the device checks whether |r| fell tenfold since the last
// update; if so the base residual is recomputed as b - A x in double
// precision (the residual-replacement idea the paper discusses, applied to
// the base system of the shifted family) and replaces the single precision
// residual.
//
// Multi-shift solves (two or more shifts, zero start) defer the shifted
// systems' vector updates: the operator acts on the base direction only, so
// the x_i and p_i of every shift are brought up to date once per block of 16
// iterations from the block's base residuals, kept in a ring, and the
// recorded scalars.  In single precision the reliable-update checks fall on
// the same block ends, where the solutions are current.
#include <chrono>
#include <cstring>
#include <vector>

#include "batch.h"
#include "ms_device.h"
#include "solver.h"

namespace stag {

struct ShiftedSolve {
    double mass;
    int n;
    const double *shifts;     // host
    const void *src;          // double library vector
    void *const *x_hi;        // double library vectors (outputs)
    bool x_init;              // start from x_hi (n == 1) instead of zero
    double tol;
    int max_iter;
    bool dbl_iter;            // double precision iterations
    int reliable_every;       // 0: no reliable updates
    // rational application (double precision, zero start): rat_out =
    // rat_w0 src + sum_i rat_w[i] x_i, with no x_i stored (x_hi unused)
    const double *rat_w = nullptr;
    double rat_w0 = 0.0;
    void *rat_out = nullptr;
};

struct ShiftedResult {
    int status;               // MsStatus
    int iters;
    int n_reliable;
    int iters_shift[kMaxShifts];
    double resid_iter[kMaxShifts];
    double resid_true[kMaxShifts];
    double dot;               // rational application: Re <src, out>
};

static constexpr int kChunk = 8;   // iterations enqueued between flag reads
static constexpr int kTresBlock = 128;   // sites per workgroup of the final true-residual launches
static constexpr double kReliableDelta = 0.1;   // reliable update after |r| fell 10x
static constexpr int kReliableCheck = kDefer;   // iterations between reliable-update checks

stag_status run_shifted(stag_lattice *lat, const ShiftedSolve &sp, ShiftedResult *res, hipStream_t s) {
    TraceRange tr(sp.dbl_iter ? "shifted CG, FP64 iterations" : "shifted CG, FP32 iterations");
    const int n = sp.n;
    const bool dbl = sp.dbl_iter;
    const int64_t ne = 3 * lat->Vh;  // complex entries per vector
    const size_t vb = (size_t)vec_bytes(lat, dbl);
    const size_t vb64 = (size_t)vec_bytes(lat, true);
    const void *links_it = dbl ? lat->links64 : lat->links32;

    int base = 0;
    for (int i = 1; i < n; ++i)
        if (sp.shifts[i] < sp.shifts[base]) base = i;
    const double sigma0 = sp.shifts[base];

    // deferred shift updates (see the top of the file)
    const bool rat = sp.rat_out != nullptr;
    if (rat && (!dbl || sp.x_init || sp.reliable_every)) {
        set_error("the rational application runs in double precision from a zero start");
        return STAG_EINVAL;
    }
    const bool defer = rat || (!sp.x_init && n >= 2);
    const int dlen = kDefer;   // iterations per deferred block
    static_assert(kChunk % 8 == 0 && kReliableCheck % kDefer == 0, "deferred block lengths");
    if (defer && sp.reliable_every % dlen != 0) {
        set_error("reliable updates must fall on deferred passes");
        return STAG_EINVAL;
    }

    void *T, *T64, *R, *AP, *P, *XLO = nullptr, *RHI, *PART, *STATE;
    const int ds_grid = dslash_grid(lat->g, kDslashBlock);
    const int bl_grid = blas_grid(ne);
    const int nparts_max = ds_grid > kMaxBlasGrid ? ds_grid : kMaxBlasGrid;
    const size_t state_bytes = (sizeof(MsState) + 255) / 256 * 256;
    STAG_TRY(ws_get(lat, WS_T, vb, &T));
    STAG_TRY(ws_get(lat, WS_T2, vb64, &T64));
    STAG_TRY(ws_get(lat, WS_R, vb * (defer ? dlen : 1), &R));
    STAG_TRY(ws_get(lat, WS_AP, vb, &AP));
    STAG_TRY(ws_get(lat, WS_P, vb * (n + (defer ? 1 : 0)), &P));
    if (!dbl) STAG_TRY(ws_get(lat, WS_XLO, (size_t)vec_bytes(lat, false) * n, &XLO));
    STAG_TRY(ws_get(lat, WS_RHI, vb64, &RHI));
    STAG_TRY(ws_get(lat, WS_PART, sizeof(double) * 2 * nparts_max, &PART));
    STAG_TRY(ws_get(lat, WS_STATE, state_bytes + sizeof(DeferHist), &STATE));
    double *part0 = static_cast<double *>(PART), *part1 = part0 + nparts_max;
    MsState *st = static_cast<MsState *>(STATE);
    DeferHist *hist = reinterpret_cast<DeferHist *>(static_cast<char *>(STATE) + state_bytes);
    // residual r^k of iteration k: slot k mod dlen of the ring (deferred) or R
    auto rslot = [&](int k) -> void * {
        return defer ? static_cast<char *>(R) + vb * (size_t)(((k % dlen) + dlen) % dlen) : R;
    };

    ShiftPtrs it_ptrs, hi_ptrs, lo_ptrs;
    std::memset(&it_ptrs, 0, sizeof(it_ptrs));
    std::memset(&hi_ptrs, 0, sizeof(hi_ptrs));
    std::memset(&lo_ptrs, 0, sizeof(lo_ptrs));
    for (int i = 0; i < n; ++i) {
        it_ptrs.p[i] = static_cast<char *>(P) + vb * i;
        hi_ptrs.x[i] = rat ? nullptr : sp.x_hi[i];
        if (!dbl) lo_ptrs.x[i] = static_cast<char *>(XLO) + (size_t)vec_bytes(lat, false) * i;
        it_ptrs.x[i] = rat ? nullptr : dbl ? sp.x_hi[i] : lo_ptrs.x[i];
    }
    // the direction the operator acts on: the base shift's own p, or (deferred)
    // a separate vector kept current every iteration
    void *pbase = defer ? static_cast<char *>(P) + vb * n : it_ptrs.p[base];

    // static part of the state
    MsState hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.n = n;
    hs.base = base;
    hs.tol = sp.tol;
    hs.max_iter = sp.max_iter;
    hs.rel_delta2 = sp.reliable_every > 0 ? kReliableDelta * kReliableDelta : 0.0;
    hs.hist = defer ? hist : nullptr;   // its record is emptied by the start step
    hs.rat = rat ? 1 : 0;
    if (rat)
        for (int i = 0; i < n; ++i) hs.wgt[i] = sp.rat_w[i];
    for (int i = 0; i < n; ++i) hs.shift_rel[i] = sp.shifts[i] - sigma0;
    STAG_HIP(hipMemcpyAsync(st, &hs, sizeof(hs), hipMemcpyHostToDevice, s));

    const double m2 = sp.mass * sp.mass;
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.link_cache = lat->link_cache;
    const bool nt = dbl && lat->vec_stream;

    // r = b - A x in double precision (into rout if non-null), partials of
    // |r|^2 in `partial` (ds_grid of them)
    auto true_residual = [&](void *x, double shift, void *rout, double *partial, const int *skip) -> hipError_t {
        DslashArgs d = a;
        d.links = lat->links64;
        d.skip = skip;
        d.out_parity = 1;
        d.in = x;
        d.out = T64;
        hipError_t e = launch_dslash(true, lat->nrow, DS_PLAIN, d, s);
        if (e != hipSuccess) return e;
        d.out_parity = 0;
        d.in = T64;
        d.out = rout;
        d.aux = x;
        d.rhs = sp.src;
        d.c = m2 + shift;
        d.partial = partial;
        return launch_dslash(true, lat->nrow, DS_RESID, d, s);
    };

    // ---------------------------------------------------------------- start
    if (!sp.x_init) {
        // r^0 = b sits where iteration 0 reads it (slot dlen - 1 of the ring)
        STAG_HIP(launch_ms_start(dbl, static_cast<const double2 *>(sp.src), rslot(-1), it_ptrs, n, !rat, ne, s));
        if (rat)
            STAG_HIP(launch_scale(static_cast<const double2 *>(sp.src), sp.rat_w0, static_cast<double2 *>(sp.rat_out),
                                  ne, s));
        if (defer) STAG_HIP(hipMemcpyAsync(pbase, rslot(-1), vb, hipMemcpyDeviceToDevice, s));
        if (!dbl)
            for (int i = 0; i < n; ++i) STAG_HIP(hipMemsetAsync(sp.x_hi[i], 0, vb64, s));
        STAG_HIP(launch_norm2(true, sp.src, ne, part0, bl_grid, s));
        STAG_HIP(launch_scalar_init(st, part0, bl_grid, nullptr, 0, s));
    } else {
        STAG_HIP(true_residual(sp.x_hi[0], sp.shifts[0], RHI, part0, nullptr));
        STAG_HIP(launch_restart(dbl, static_cast<const double2 *>(RHI), R, pbase, ne, s));
        if (!dbl) STAG_HIP(hipMemsetAsync(lo_ptrs.x[0], 0, (size_t)vec_bytes(lat, false), s));
        STAG_HIP(launch_norm2(true, sp.src, ne, part1, bl_grid, s));
        STAG_HIP(launch_scalar_init(st, part0, ds_grid, part1, bl_grid, s));
    }

    // ---------------------------------------------------------------- iterate
    a.links = links_it;
    a.skip = &st->done;
    auto iteration = [&](int k) -> stag_status {
        DslashArgs d = a;
        d.out_parity = 1;
        d.in = pbase;
        d.out = T;
        STAG_HIP(launch_dslash(dbl, lat->nrow, DS_PLAIN, d, s));
        d.out_parity = 0;
        d.in = T;
        d.out = AP;
        d.aux = pbase;
        d.c = m2 + sigma0;
        d.partial = part0;
        STAG_HIP(launch_dslash(dbl, lat->nrow, DS_NORMAL_DOT, d, s));
        if (defer) {
            // the scalar steps ride in the two vector kernels (no tail launches)
            STAG_HIP(launch_r_update_fused(dbl, st, part0, ds_grid, rslot(k - 1), rslot(k), AP, ne, part1, bl_grid, s,
                                           nt));
            STAG_HIP(launch_dir_update_fused(dbl, st, part1, bl_grid, rslot(k), pbase, ne, bl_grid, s, nt));
            if ((k + 1) % dlen == 0)
                STAG_HIP(launch_defer_pass(dbl, st, hist, R, ne, it_ptrs, n, ne, bl_grid, s, sp.rat_out, nt));
        } else {
            STAG_HIP(launch_reduce_tail(st, part0, ds_grid, TAIL_ALPHA, 0, s));
            STAG_HIP(launch_r_update(dbl, st, rslot(k - 1), rslot(k), AP, ne, part1, bl_grid, s));
            STAG_HIP(launch_reduce_tail(st, part1, bl_grid, TAIL_BETA, 0, s));
            STAG_HIP(launch_shift_update(dbl, st, R, it_ptrs, n, ne, bl_grid, s));
        }
        if (sp.reliable_every > 0 && (k + 1) % sp.reliable_every == 0) {
            STAG_HIP(launch_x_flush(st, hi_ptrs, lo_ptrs, n, ne, true, s));
            STAG_HIP(true_residual(sp.x_hi[base], sigma0, RHI, part0, &st->rel_skip));
            STAG_HIP(launch_reduce_tail(st, part0, ds_grid, TAIL_RELIABLE, 0, s));
            STAG_HIP(launch_demote(st, static_cast<const double2 *>(RHI), static_cast<float2 *>(rslot(k)), ne, s));
        }
        return STAG_OK;
    };

    hipEvent_t ev[2];
    STAG_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    STAG_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    volatile int *flags = lat->host_flags;
    flags[0] = flags[1] = 0;
    stag_status rc = STAG_OK;
    int chunk = 0;
    bool finished = false;
    for (int k0 = 0; k0 < sp.max_iter + kChunk && !finished; k0 += kChunk, ++chunk) {
        for (int k = k0; k < k0 + kChunk; ++k) {
            rc = iteration(k);
            if (rc != STAG_OK) break;
        }
        if (rc != STAG_OK) break;
        const int slot = chunk & 1;
        if (hipMemcpyAsync(const_cast<int *>(flags + slot), &st->done, sizeof(int), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipEventRecord(ev[slot], s) != hipSuccess) {
            set_error("flag copy failed");
            rc = STAG_EHIP;
            break;
        }
        if (chunk > 0) {
            if (hipEventSynchronize(ev[slot ^ 1]) != hipSuccess) {
                set_error("event synchronize failed");
                rc = STAG_EHIP;
                break;
            }
            if (flags[slot ^ 1]) finished = true;
        }
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc != STAG_OK) return rc;

    // ---------------------------------------------------------------- finish
    // the last block may end between passes (a no-op when it does not)
    if (defer) STAG_HIP(launch_defer_pass(dbl, st, hist, R, ne, it_ptrs, n, ne, bl_grid, s, sp.rat_out, nt));
    if (!dbl) STAG_HIP(launch_x_flush(st, hi_ptrs, lo_ptrs, n, ne, false, s));
    if (rat) {
        // no solutions are kept: report Re <src, out> instead of true residuals
        STAG_HIP(launch_dot_re(static_cast<const double2 *>(sp.src), static_cast<const double2 *>(sp.rat_out), ne,
                               part0, bl_grid, s));
        STAG_HIP(launch_reduce_tail(st, part0, bl_grid, TAIL_SCRATCH, 0, s));
    } else if (n > 1) {
        // every shift's true residual, eight per multi-right-hand-side launch pair
        const int nchunk = (int)((lat->Vh + kWave - 1) / kWave);
        const int ng = n < kMaxRpt ? n : kMaxRpt;
        void *tres = nullptr;
        STAG_TRY(ws_get(lat, WS_TRES, vb64 * ng + sizeof(double) * (size_t)nchunk * n, &tres));
        void *tb[kMaxRpt];
        double *pp[kMaxShifts];
        double cc[kMaxShifts];
        for (int r = 0; r < ng; ++r) tb[r] = static_cast<char *>(tres) + vb64 * r;
        for (int i = 0; i < n; ++i) {
            pp[i] = reinterpret_cast<double *>(static_cast<char *>(tres) + vb64 * ng) + (size_t)nchunk * i;
            cc[i] = m2 + sp.shifts[i];
        }
        STAG_HIP(launch_true_resid_multi(lat, n, reinterpret_cast<const void *const *>(sp.x_hi), cc, sp.src, tb, pp,
                                         kTresBlock, s));
        for (int i = 0; i < n; ++i) STAG_HIP(launch_reduce_tail(st, pp[i], nchunk, TAIL_TRUE_RESID, i, s));
    } else {
        STAG_HIP(true_residual(sp.x_hi[0], sp.shifts[0], nullptr, part0, nullptr));
        STAG_HIP(launch_reduce_tail(st, part0, ds_grid, TAIL_TRUE_RESID, 0, s));
    }
    STAG_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    STAG_HIP(hipStreamSynchronize(s));
    res->status = hs.status;
    res->dot = hs.scratch[0];
    res->iters = hs.iter;
    res->n_reliable = hs.n_reliable;
    for (int i = 0; i < n; ++i) {
        res->iters_shift[i] = hs.active[i] ? hs.iter : hs.iters_shift[i];
        res->resid_iter[i] = hs.resid_iter[i];
        res->resid_true[i] = hs.resid_true[i];
    }
    return STAG_OK;
}

static stag_status status_of(int ms) {
    switch (ms) {
        case MS_CONVERGED: return STAG_OK;
        case MS_BREAKDOWN: set_error("non-positive or non-finite curvature <p, A p>"); return STAG_EBREAKDOWN;
        default: set_error("maximum number of iterations reached"); return STAG_ENOCONV;
    }
}

// Single-shift CG from x: repeat passes until the double precision true
// residual meets tol (one pass in double precision normally suffices; the
// mixed pass may need a second one when the iterated and true residuals
// drift apart near convergence).
static stag_status cg_refine(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol,
                             int max_iter, bool mixed, int *iters, int *n_rel, double *resid, hipStream_t s) {
    ShiftedSolve sp;
    void *xs[1] = {x};
    sp.mass = mass;
    sp.n = 1;
    sp.shifts = &shift;
    sp.src = src;
    sp.x_hi = xs;
    sp.x_init = true;
    sp.tol = tol;
    sp.dbl_iter = !mixed;
    sp.reliable_every = mixed ? kReliableCheck : 0;
    *iters = 0;
    *n_rel = 0;
    ShiftedResult r;
    int ms = MS_NOCONV;
    for (int pass = 0; pass < 6; ++pass) {
        sp.max_iter = max_iter - *iters;
        if (sp.max_iter <= 0) break;
        STAG_TRY(run_shifted(lat, sp, &r, s));
        *iters += r.iters;
        *n_rel += r.n_reliable;
        *resid = r.resid_true[0];
        ms = r.status;
        if (ms == MS_BREAKDOWN) break;
        if (r.resid_true[0] <= tol) {
            ms = MS_CONVERGED;
            break;
        }
        ms = MS_NOCONV;
    }
    return status_of(ms);
}

stag_status multishift_cg(stag_lattice *lat, double mass, const double *shifts, int n, const void *src,
                          void *const *sols, double tol, int max_iter, stag_prec prec, stag_cg_stats *stats,
                          hipStream_t s) {
    TraceRange tr("multi-shift CG");
    const auto t0 = std::chrono::steady_clock::now();
    ShiftedSolve sp;
    sp.mass = mass;
    sp.n = n;
    sp.shifts = shifts;
    sp.src = src;
    sp.x_hi = sols;
    sp.x_init = false;
    sp.tol = tol;
    sp.max_iter = max_iter;
    sp.dbl_iter = prec == STAG_F64;
    sp.reliable_every = prec == STAG_MIXED ? kReliableCheck : 0;
    ShiftedResult r;
    STAG_TRY(run_shifted(lat, sp, &r, s));
    stag_status rc = status_of(r.status);
    stag_cg_stats st;
    std::memset(&st, 0, sizeof(st));
    st.iters = r.iters;
    st.n_reliable = r.n_reliable;
    for (int i = 0; i < n; ++i) {
        st.iters_shift[i] = r.iters_shift[i];
        st.resid_iter[i] = r.resid_iter[i];
        st.resid_true[i] = r.resid_true[i];
        st.resid_unrefined[i] = r.resid_true[i];
    }
    if (prec == STAG_MIXED && rc != STAG_EBREAKDOWN) {
        // refine every shift that misses tol: warm-started single-shift mixed
        // CG, all of them together (one multi-RHS Dslash per phase loads every
        // link once for up to 8 shifts)
        BSpec fam = {lat, mass, n, shifts, src, sols, false};
        BOptions ro{};   // the defaults: graph replays, one launch for all lattices
        ro.tol = tol;
        ro.max_iter = max_iter;
        ro.dbl = false;
        ro.reliable_every = kReliableCheck;
        const stag_status rr = refine_batched(&fam, 1, ro, &st, s);
        if (rr < 0) return rr;
        rc = rr;
    }
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    double worst = 0.0;
    for (int i = 0; i < n; ++i) worst = st.resid_true[i] > worst ? st.resid_true[i] : worst;
    stag_log(1, "multishift_cg: %d shifts, %s, %d iterations + %d refinement, largest true residual %.3g, %.4f s, "
             "status %d", n, prec == STAG_F64 ? "f64" : prec == STAG_F32 ? "f32" : "mixed", st.iters, st.refine_iters,
             worst, st.seconds, (int)rc);
    return rc;
}

stag_status rational_apply(stag_lattice *lat, double mass, double alpha0, const double *alphas, const double *shifts,
                           int n, const void *src, void *out, double tol, int max_iter, double *dot,
                           stag_cg_stats *stats, hipStream_t s) {
    TraceRange tr("rational function of M");
    const auto t0 = std::chrono::steady_clock::now();
    ShiftedSolve sp;
    sp.mass = mass;
    sp.n = n;
    sp.shifts = shifts;
    sp.src = src;
    sp.x_hi = nullptr;
    sp.x_init = false;
    sp.tol = tol;
    sp.max_iter = max_iter;
    sp.dbl_iter = true;
    sp.reliable_every = 0;
    sp.rat_w = alphas;
    sp.rat_w0 = alpha0;
    sp.rat_out = out;
    ShiftedResult r;
    STAG_TRY(run_shifted(lat, sp, &r, s));
    const stag_status rc = status_of(r.status);
    if (dot) *dot = r.dot;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = r.iters;
        for (int i = 0; i < n; ++i) {
            stats->iters_shift[i] = r.iters_shift[i];
            stats->resid_iter[i] = r.resid_iter[i];
        }
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

stag_status single_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol,
                      int max_iter, stag_prec prec, stag_cg_stats *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    int it = 0, nrel = 0;
    double resid = 0.0;
    stag_status rc = cg_refine(lat, mass, shift, src, x, tol, max_iter, prec == STAG_MIXED, &it, &nrel, &resid, s);
    if (rc < 0) return rc;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = it;
        stats->n_reliable = nrel;
        stats->iters_shift[0] = it;
        stats->resid_true[0] = resid;
        stats->resid_unrefined[0] = resid;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

}  // namespace stag
