// Device-resident state of the shifted CG and the launchers of the solver
// kernels.  All scalars of the recursion live in device memory and are
// updated by single-wave kernels, so an iteration needs no host round trip.
#pragma once

#include "internal.h"

namespace stag {

constexpr int kMaxShifts = STAG_MAX_SHIFTS;
constexpr int kBlasBlock = 256;
constexpr int kMaxBlasGrid = 2048;
constexpr int kMaxPartials = 16384;

enum MsStatus { MS_RUNNING = 0, MS_NOCONV = 1, MS_BREAKDOWN = 2, MS_CONVERGED = 3 };

// Deferred shift updates.  The shifted systems' vectors never enter the
// operator: only the base direction does.  Over L iterations
//   x_i += a_i^k p_i,   p_i = zeta_i^{k+1} r^{k+1} + b_i^k p_i
// keeps p_i in the span of its value at the start of the block and the base
// residuals r^{k0+1} .. r^{k0+L}, so one pass at the end of the block, with
// coefficients built from the recorded scalars, does the work of L
// per-iteration passes: each p_i and x_i is read and written once per block
// instead of once per iteration.  Blocks hold up to kDefer iterations.
constexpr int kDefer = 16;

struct DeferHist {
    int len;        // iterations recorded since the last pass
    int nvalid;     // iterations covered by the coefficients of the pass
    int pad[2];
    double a[kDefer][kMaxShifts], b[kDefer][kMaxShifts], z[kDefer][kMaxShifts];
    int u[kDefer][kMaxShifts];          // shift i was updated at that iteration
    int act[kMaxShifts];                // shift i changes in this pass
    double cx[kMaxShifts][kDefer + 1];  // x_i += cx[0] p_i + sum_m cx[1+m] r_m
    double cp[kMaxShifts][kDefer + 1];  // p_i  = cp[0] p_i + sum_m cp[1+m] r_m
};

struct MsState {
    double rho;          // <r, r>
    double alpha, alpha_prev, beta, beta_prev;
    double bnorm2;       // ||b||^2 of the reference right-hand side
    double tol;          // relative tolerance
    double rho_rel;      // |r|^2 right after the last reliable update (or the start)
    double rel_delta2;   // reliable update once |r|^2 < rel_delta2 * rho_rel (0: never)
    double rho_snap;     // rho of this iteration, kept for the fused beta step
    double scratch[4];   // reduced values handed to the host
    int n, base;
    int iter, max_iter;
    int done;            // set once the solve ended: later kernels are no-ops
    int status;          // MsStatus
    int upd_valid;       // the shift-update kernel applies this iteration
    int upd_p;           // the base direction is updated this iteration
    int n_reliable;
    int rel_skip;        // 1: the reliable-update kernels of this iteration are no-ops
    int rat;             // rational application: the deferred passes weight shift i by wgt[i]
    int pad;
    DeferHist *hist;     // non-null: the scalar steps record per-iteration coefficients
    double shift_rel[kMaxShifts];   // s_i = sigma_i - sigma_base
    double zeta[kMaxShifts], zeta_prev[kMaxShifts], zeta_next[kMaxShifts];
    double a[kMaxShifts], b[kMaxShifts];
    double resid_iter[kMaxShifts];
    double resid_true[kMaxShifts];
    double wgt[kMaxShifts];         // weights of the rational application
    int active[kMaxShifts];
    int upd[kMaxShifts];
    int iters_shift[kMaxShifts];
};

// Pointers to the per-shift vectors, passed by value.
struct ShiftPtrs {
    void *x[kMaxShifts];
    void *p[kMaxShifts];
};

int blas_grid(int64_t n_elems);

// ||v||^2 partials of a library vector (n_elems complex entries).
hipError_t launch_norm2(bool dbl, const void *v, int64_t n, double *partial, int grid, hipStream_t s);
// dst[k] = src[k] (+ dst zero for every x) : multi-shift start x_i = 0, p_i = b, r = b
hipError_t launch_ms_start(bool dbl, const double2 *b, void *r, ShiftPtrs ptrs, int n_shift, bool zero_x,
                           int64_t n, hipStream_t s);
hipError_t launch_scalar_init(MsState *st, const double *partial_r, int nparts_r, const double *partial_b,
                              int nparts_b, hipStream_t s);
// r = rin - alpha A p (rin may equal r), and the partials of ||r||^2.
hipError_t launch_r_update(bool dbl, MsState *st, const void *rin, void *r, const void *ap, int64_t n, double *partial,
                           int grid, hipStream_t s);
// Deferred updates, every iteration: r = rin - alpha A p into the next ring
// slot and pd = r + beta pd (the base direction the operator acts on), with
// the scalar recursion folded in: every block sums
// the partials of the previous reduction itself (the fixed order of the
// one-workgroup tail, so the scalars are bit for bit those of the separate
// tail kernel) and block 0 also advances the recursion.
//   r update: <p, A p> from pq_part (npq) -> alpha, zeta_i; r = rin - alpha A p; |r|^2 partials
//   direction: |r|^2 from r_part (nr) -> beta, shift coefficients, freeze tests; pd = r + beta pd
// nt (double precision): nontemporal vector loads and stores, for a lattice
// whose Dslash keeps part of the link field in the Infinity Cache.
hipError_t launch_r_update_fused(bool dbl, MsState *st, const double *pq_part, int npq, const void *rin, void *r,
                                 const void *ap, int64_t n, double *partial, int grid, hipStream_t s, bool nt = false);
hipError_t launch_dir_update_fused(bool dbl, MsState *st, const double *r_part, int nr, const void *r, void *pd,
                                   int64_t n, int grid, hipStream_t s, bool nt = false);
// At the end of a block of deferred iterations: the coefficients and the
// pass over every shift changed in it.  ring: one residual vector per
// iteration of the block, slot m holding r^{k0+1+m}.
// out == nullptr: x_i += ... for every shift; otherwise (rational
// application, double precision) out += sum_i wgt_i (x_i increment) and no
// x_i is kept.  nt as above.
hipError_t launch_defer_pass(bool dbl, MsState *st, DeferHist *h, const void *ring, int64_t slot_elems, ShiftPtrs ptrs,
                             int n_shift, int64_t n, int grid, hipStream_t s, void *out = nullptr, bool nt = false);
// out = c * b (double precision)
hipError_t launch_scale(const double2 *b, double c, double2 *out, int64_t n, hipStream_t s);
// partials of Re <a, b> (double precision), one per block of `grid`
hipError_t launch_dot_re(const double2 *a, const double2 *b, int64_t n, double *partial, int grid, hipStream_t s);
hipError_t launch_shift_update(bool dbl, MsState *st, const void *r, ShiftPtrs ptrs, int n_shift, int64_t n, int grid,
                               hipStream_t s);
// One workgroup sums nparts partials (fixed order) and applies a TailKind step.
hipError_t launch_reduce_tail(MsState *st, const double *partial, int nparts, int kind, int idx, hipStream_t s);
// x_hi += x_lo; x_lo = 0 for every shift (single precision accumulators).
hipError_t launch_x_flush(MsState *st, ShiftPtrs hi, ShiftPtrs lo, int n_shift, int64_t n, bool skip_on_done,
                          hipStream_t s);
// dst (float) = src (double), skipped when the solve is done.
hipError_t launch_demote(MsState *st, const double2 *src, float2 *dst, int64_t n, hipStream_t s);
// r = b - Ax computed elsewhere in double; copy r into a float/double residual and set directions p = r
hipError_t launch_restart(bool dbl, const double2 *rhi, void *r, void *p, int64_t n, hipStream_t s);

}  // namespace stag
