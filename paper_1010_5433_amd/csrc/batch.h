// Batched shifted CG: many systems (pseudo-fermions x shifts, and lattices
// of different sizes) advanced together.  Systems that share a gauge field
// are processed by a multi-RHS Dslash that loads every link once for up to
// 8 right-hand sides (one launch per lattice and phase); the vector updates
// and recursions of all systems run in one launch per phase.
//
// Reductions are grouped per 64 consecutive sites (Dslash) or per 256
// consecutive vector entries (vector kernels) -- one wave each -- and the
// per-system tail kernel sums those partials in a fixed order.  The result
// therefore does not depend on the launch shape the autotuner picks.
#pragma once

#include "solver.h"

namespace stag {

constexpr int kMaxBatch = 64;       // systems per batched call
constexpr int kMaxRpt = 8;          // right-hand sides per thread in the multi-RHS Dslash
constexpr int kBChunk = 256;        // vector entries per reduction chunk (one wave, 4 per lane)
constexpr int kBBlock = 256;        // threads per block of the vector kernels

struct BLat {
    Geom g;
    int nrow;
    int pad;
    const void *links;     // iteration precision
    const void *links64;   // double precision (residual checks)
};

struct BSys {
    int lat;               // index into the lattice table
    int n;                 // shifts
    int base;              // index of the smallest shift
    int nchunk_ds;         // Dslash partials: ceil(Vh / 64)
    int nchunk_bl;         // vector partials: ceil(3 Vh / kBChunk)
    int x_init;            // start from xhi[0] (single shift) instead of zero
    int dlen;              // deferred shift updates in blocks of dlen iterations (0: every iteration)
    int rat;               // rational application: the pass sums the weighted increments into out
    double m2;             // mass^2
    double shifts[kMaxShifts];
    MsState *st;
    double *part_ds;
    double *part_bl;
    const double2 *src;
    void *r, *ap, *t;      // iteration precision
    double2 *out;          // rational application output (double precision)
    double w0;             // its weight of src
    void *ring;            // deferred: dlen residual vectors, r^k in slot k mod dlen
    void *pd;              // deferred: the base direction the operator acts on
    DeferHist *hist;       // deferred: recorded scalars and pass coefficients
    double2 *t64, *rhi;    // double precision work vectors
    void *p[kMaxShifts];
    void *x[kMaxShifts];   // iteration precision accumulators (== xhi for double)
    double2 *xhi[kMaxShifts];
};

// Tables read by the vector and recursion kernels of a batch.
struct BView {
    const BLat *lats;
    const BSys *sys;
    int nsys;
};

// Launch configuration of the multi-RHS Dslash.
struct BDslashCfg {
    int block;   // sites per block: 64, 128 or 256
    int rpt;     // right-hand sides per thread: 1, 2, 4 or 8
};

// Vector kernels over every system (grid.y = system).
enum BVecOp {
    BV_START = 0,      // r = b, p_i = b, x_i = 0 (and xhi = 0 for single precision)
    BV_RESTART = 1,    // r = rhi, p_base = r, x = 0 (single precision accumulator)
    BV_NORM_SRC = 2,   // partial |b|^2
    BV_R_UPDATE = 3,   // r -= alpha ap, partial |r|^2
    BV_SHIFT_UPDATE = 4,
    BV_FLUSH = 5,      // xhi += x, x = 0 (single precision), when a reliable update is due
    BV_FLUSH_FINAL = 6,// same, always
    BV_DEMOTE = 7,     // r = (float) rhi, when a reliable update is due
    BV_DEFER_APPLY = 8,// deferred systems: the pass over every shift changed in the block
    // batches whose systems are all deferred: the alpha and beta steps ride in
    // the vector kernels (each block sums its system's partials in kb_tail's
    // order; block 0 of the system advances the recursion)
    BV_R_UPDATE_FUSED = 9,
    BV_DIR_FUSED = 10
};
// it: the iteration the op belongs to (selects ring slots of deferred systems;
// BV_START writes r^0 to the slot iteration 0 reads)
hipError_t launch_bvec(bool dbl, BView v, int op, int max_blocks, hipStream_t s, int it = 0);
// coefficients of the deferred pass of every deferred system
hipError_t launch_bdefer_coef(BView v, hipStream_t s);

enum BTail {
    BT_INIT = 0,       // zero start: rho = |b|^2 from part_bl
    BT_ALPHA = 1,      // <p, A p> from part_ds
    BT_BETA = 2,       // |r|^2 from part_bl
    BT_TRUE_RESID = 3  // |b - (M + sigma_idx) x_idx|^2 from part_ds (systems with a shift idx, no rational ones)
};
hipError_t launch_btail(BView v, int kind, hipStream_t s, int idx = 0);
hipError_t launch_ball_done(BView v, int *flag, hipStream_t s);

// ---------------------------------------------------------------- host side

struct BSpec {
    stag_lattice *lat;
    double mass;
    int n;
    const double *shifts;   // host
    const void *src;        // double library vector
    void *const *sols;      // double library vectors: outputs (and the start when x_init)
    bool x_init;
    // rational application (double precision, zero start): rat_out =
    // rat_w0 src + sum_i rat_w[i] (M + shifts[i])^-1 src, sols unused
    const double *rat_w = nullptr;
    double rat_w0 = 0.0;
    void *rat_out = nullptr;
};

struct BOut {
    int status, iters, n_reliable;
    int iters_shift[kMaxShifts];
    double resid_iter[kMaxShifts];
    double resid_true[kMaxShifts];
    double dot;             // rational application: Re <src, out>
};

struct BOptions {
    double tol;
    int max_iter;
    bool dbl;
    int reliable_every;     // 0: none
    int force_block;        // 0: autotune
    int force_rpt;
    bool use_graph = true;  // replay captured blocks of iterations (false: launch every kernel)
    bool merge_lattices = true;   // one multi-RHS Dslash launch per phase for all lattices
};

// per-lattice multi-RHS Dslash with arguments by value; everything on stream s
stag_status run_batched(const BSpec *spec, int nsys, const BOptions &opt, BOut *out, hipStream_t s);
// refine every (system, shift) whose true residual in stats exceeds opt.tol
stag_status refine_batched(const BSpec *spec, int nsys, const BOptions &opt, stag_cg_stats *stats, hipStream_t s);
stag_status batched_solve(const BSpec *spec, int nsys, const BOptions &opt, bool mixed, stag_cg_stats *stats,
                          hipStream_t s);
stag_status rational_apply_multi(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                 const double *shifts, int n, const void *const *srcs, void *const *outs, int n_rhs,
                                 double tol, int max_iter, double *dots, stag_cg_stats *stats, hipStream_t s);
// launch shape chosen by the last batched solve on this thread
BDslashCfg last_batch_cfg();

}  // namespace stag
