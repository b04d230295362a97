// Host side of the batched solver: the full solve and the refinement of
// every (system, shift) that a single precision solve left above tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "batch.h"
#include "ms_device.h"

namespace stag {

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
    TraceRange tr("batched refinement");
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
            ro_opt.reliable_every = kDefer;
            ro_opt.force_block = ro_opt.force_rpt = 0;
            STAG_TRY(run_batched(rs.data(), m, ro_opt, ro.data(), s));
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

// One rational function applied to n_rhs fields of one lattice (several
// pseudo-fermions): every field is a deferred system of the batch, so the
// multi-RHS Dslash loads each link once for up to 8 of them.
stag_status rational_apply_multi(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                 const double *shifts, int n, const void *const *srcs, void *const *outs, int n_rhs,
                                 double tol, int max_iter, double *dots, stag_cg_stats *stats, hipStream_t s) {
    TraceRange tr("rational function of M, several fields");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<BSpec> spec(n_rhs);
    for (int k = 0; k < n_rhs; ++k) {
        spec[k].lat = lat;
        spec[k].mass = mass;
        spec[k].n = n;
        spec[k].shifts = shifts;
        spec[k].src = srcs[k];
        spec[k].sols = nullptr;
        spec[k].x_init = false;
        spec[k].rat_w = alphas;
        spec[k].rat_w0 = alpha0;
        spec[k].rat_out = outs[k];
    }
    BOptions opt{};   // the defaults: graph replays, one launch for all lattices
    opt.tol = tol;
    opt.max_iter = max_iter;
    opt.dbl = true;
    std::vector<BOut> out(n_rhs);
    STAG_TRY(run_batched(spec.data(), n_rhs, opt, out.data(), s));
    stag_status rc = STAG_OK;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < n_rhs; ++k) {
        if (dots) dots[k] = out[k].dot;
        if (stats) {
            stag_cg_stats &st = stats[k];
            std::memset(&st, 0, sizeof(st));
            st.iters = out[k].iters;
            for (int i = 0; i < n; ++i) {
                st.iters_shift[i] = out[k].iters_shift[i];
                st.resid_iter[i] = out[k].resid_iter[i];
            }
            st.seconds = secs;
        }
        const stag_status sk = status_of_ms(out[k].status);
        if (sk == STAG_EBREAKDOWN || (sk != STAG_OK && rc == STAG_OK)) rc = sk;
    }
    return rc;
}

stag_status batched_solve(const BSpec *spec, int nsys, const BOptions &opt0, bool mixed, stag_cg_stats *stats,
                          hipStream_t s) {
    TraceRange tr("batched multi-shift CG");
    const auto t0 = std::chrono::steady_clock::now();
    BOptions opt = opt0;
    std::vector<BOut> out(nsys);
    STAG_TRY(run_batched(spec, nsys, opt, out.data(), s));
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
