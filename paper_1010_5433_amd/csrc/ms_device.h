// Device-side scalar steps of the shifted CG, shared by the single-system
// and the batched solvers.  They run in a one-workgroup kernel that first
// sums the per-workgroup partials of a reduction in a fixed order.
// (Folding them into the reduction kernels -- the last workgroup to finish
// completes the sum -- was measured slower on gfx950: the agent-scope
// release each workgroup then needs writes back its XCD's L2, which costs
// more than the launch it saves.)
#pragma once

#include <math.h>

#include "common.h"
#include "solver.h"

namespace stag {

// Start of a solve: rho = <r,r>, ||b||^2 = b2; every shift active unless
// the start vector already meets the tolerance.  Threads 0..63.
__device__ __forceinline__ void ms_init_step(MsState *st, double rho, double b2) {
    const int l = threadIdx.x;
    const bool conv = rho <= st->tol * st->tol * b2;
    if (l < st->n) {
        st->zeta[l] = st->zeta_prev[l] = st->zeta_next[l] = 1.0;
        st->a[l] = st->b[l] = 0.0;
        st->active[l] = conv ? 0 : 1;
        st->upd[l] = 0;
        st->iters_shift[l] = 0;
        st->resid_iter[l] = b2 > 0.0 ? sqrt(rho / b2) : 0.0;
        st->resid_true[l] = 0.0;
    }
    if (l == 0) {
        st->bnorm2 = b2;
        st->rho = rho;
        st->alpha = 0.0;
        st->alpha_prev = 1.0;
        st->beta = 0.0;
        st->beta_prev = 0.0;
        st->iter = 0;
        st->upd_valid = 0;
        st->upd_p = 0;
        st->n_reliable = 0;
        st->rho_rel = rho;
        st->rel_skip = 1;
        if (st->hist) st->hist->len = 0;
        st->done = conv ? 1 : 0;
        st->status = conv ? MS_CONVERGED : MS_RUNNING;
    }
}

// alpha_k = rho_k / <p, A p> and zeta_i^{k+1} for every active shift.
// Threads 0..63 cover the shifts.
__device__ __forceinline__ void ms_alpha_step(MsState *st, double pap) {
    const int l = threadIdx.x;
    if (!(pap > 0.0) || !isfinite(pap)) {
        if (l == 0) {
            st->status = MS_BREAKDOWN;
            st->done = 1;
        }
        return;
    }
    const double alpha = st->rho / pap;
    if (l < st->n && st->active[l]) {
        if (l == st->base) {
            st->zeta_next[l] = 1.0;
        } else {
            const double z = st->zeta[l], zp = st->zeta_prev[l];
            const double den = alpha * st->beta_prev * (zp - z) + zp * st->alpha_prev * (1.0 + st->shift_rel[l] * alpha);
            st->zeta_next[l] = z * zp * st->alpha_prev / den;
        }
    }
    if (l == 0) st->alpha = alpha;
}

// beta_k, alpha_k^i, beta_k^i, the freeze test of every shift, and the
// histories; flags the shift update of this iteration as valid.
// Run by the first wave of one workgroup (threads 0..63).
__device__ __forceinline__ void ms_beta_step(MsState *st, double rho_new) {
    const int l = threadIdx.x;
    if (l >= kWave) return;
    const double beta = rho_new / st->rho;
    const double alpha = st->alpha;
    const int it = st->iter + 1;
    DeferHist *h = st->hist;
    const int pos = h ? h->len : 0;   // read by every lane before lane 0 advances it
    bool act = false;
    if (l < st->n) {
        const bool was = st->active[l] != 0;
        st->upd[l] = was ? 1 : 0;
        if (h && pos < kDefer) h->u[pos][l] = was ? 1 : 0;
        if (was) {
            const double zn = st->zeta_next[l];
            const double ratio = zn / st->zeta[l];
            st->a[l] = alpha * ratio;
            st->b[l] = beta * ratio * ratio;
            if (h && pos < kDefer) {
                h->a[pos][l] = alpha * ratio;
                h->b[pos][l] = beta * ratio * ratio;
                h->z[pos][l] = zn;
            }
            const double res = fabs(zn) * sqrt(rho_new / st->bnorm2);
            st->resid_iter[l] = res;
            if (res <= st->tol) {
                st->active[l] = 0;
                st->iters_shift[l] = it;
            } else {
                act = true;
            }
            st->zeta_prev[l] = st->zeta[l];
            st->zeta[l] = zn;
        }
    }
    const unsigned long long any = __ballot(act);
    const int upd_base = __shfl(l < st->n ? st->upd[l] : 0, st->base);
    if (l == 0) {
        if (h) h->len = pos + 1;
        st->upd_p = (upd_base || any) ? 1 : 0;
        st->beta = beta;
        st->beta_prev = beta;
        st->alpha_prev = alpha;
        st->rho = rho_new;
        st->iter = it;
        st->upd_valid = 1;
        if (!any) {
            st->done = 1;
            st->status = MS_CONVERGED;
        } else if (it >= st->max_iter) {
            st->done = 1;
            st->status = MS_NOCONV;
        }
        // A reliable update replaces the iterated residual by b - A x.  It is
        // due once |r| fell by the factor sqrt(rel_delta2) since the last
        // one: then the single precision drift of the iterated residual is
        // still small against |r| itself, and the replaced residual stays
        // consistent with the search direction.  (A fixed schedule lets |r|
        // drop below the single precision floor between updates; the
        // replaced residual then no longer fits the direction and the
        // recursion diverges.)
        st->rel_skip = (st->rel_delta2 > 0.0 && !st->done && rho_new < st->rel_delta2 * st->rho_rel) ? 0 : 1;
    }
}

// Coefficients of a deferred pass from the recorded scalars (lane = shift,
// lanes 0..n-1 of one workgroup).  Starting from p = p_i (index 0), every
// recorded iteration j at which shift i was updated does x += a_j p, then
// p = b_j p + z_j r^{k0+1+j} (index 1 + j).  Resets the record.  Every
// thread of the workgroup must call it.  With weights w (rational
// application) the x coefficients of shift i are scaled by w[i].
__device__ __forceinline__ void defer_coef_step(int n, DeferHist *h, const double *w = nullptr) {
    const int l = threadIdx.x;
    const int len = h->len;
    const int nv = len < kDefer ? len : kDefer;
    if (l < n) {
        double cx[kDefer + 1], cp[kDefer + 1];
#pragma unroll
        for (int q = 0; q <= kDefer; ++q) {
            cx[q] = 0.0;
            cp[q] = q == 0 ? 1.0 : 0.0;
        }
        int any = 0;
        for (int j = 0; j < nv; ++j) {
            if (!h->u[j][l]) continue;
            any = 1;
            const double aj = h->a[j][l], bj = h->b[j][l];
#pragma unroll
            for (int q = 0; q <= kDefer; ++q) {
                cx[q] += aj * cp[q];
                cp[q] *= bj;
            }
            cp[1 + j] += h->z[j][l];
        }
        const double wl = w ? w[l] : 1.0;
#pragma unroll
        for (int q = 0; q <= kDefer; ++q) {
            h->cx[l][q] = wl * cx[q];
            h->cp[l][q] = cp[q];
        }
        h->act[l] = any;
    }
    __syncthreads();   // every lane has read len
    if (l == 0) {
        h->nvalid = nv;
        h->len = 0;
    }
}

// One entry of the deferred pass for shift i:
// x += cx0 p + sum_m cx_m r_m,  p = cp0 p + sum_m cp_m r_m (rr[m] = 0 past the block).
template <typename V, typename R>
__device__ __forceinline__ void defer_combine(const DeferHist *h, int i, const V (&rr)[kDefer], V &xv, V &pv) {
    const R cx0 = R(h->cx[i][0]), cp0 = R(h->cp[i][0]);
    xv.x += cx0 * pv.x;
    xv.y += cx0 * pv.y;
    V np;
    np.x = cp0 * pv.x;
    np.y = cp0 * pv.y;
#pragma unroll
    for (int m = 0; m < kDefer; ++m) {
        const R cxm = R(h->cx[i][1 + m]), cpm = R(h->cp[i][1 + m]);
        xv.x += cxm * rr[m].x;
        xv.y += cxm * rr[m].y;
        np.x += cpm * rr[m].x;
        np.y += cpm * rr[m].y;
    }
    pv = np;
}

// What the one-workgroup reduction kernel does with the reduced sum.
enum TailKind {
    TAIL_ALPHA = 1,      // total = <p, A p>: alpha and zeta; retires the update flag once done
    TAIL_BETA = 2,       // total = |r|^2: beta, shift coefficients, freeze tests
    TAIL_RELIABLE = 3,   // total = ||b - A x||^2 after a reliable update
    TAIL_TRUE_RESID = 4, // total = ||b - (M + sigma_i) x_i||^2 of shift idx
    TAIL_SCRATCH = 5     // total into scratch[idx]
};

}  // namespace stag
