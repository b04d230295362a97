/*
 * stag.h -- C ABI of the MI355X (gfx950) even/odd staggered solver library.
 *
 * The library solves the problem the paper states (Bonati, Cossu, D'Elia,
 * Di Giacomo, "Staggered fermions simulations on GPUs", Lattice 2010):
 * unimproved staggered fermions with even/odd preconditioning (Section 2),
 * inverted with CG and with the Krylov solver for shifted systems whose
 * start vector must be zero (Section 6), in double precision for the
 * Metropolis inversions and single precision elsewhere (Section 4).
 *
 * Operator (textbook Kogut-Susskind form; the paper prints no formula):
 *   (D psi)(x) = 1/2 sum_mu eta_mu(x) [ s_mu(x) U_mu(x) psi(x+mu)
 *                                      - s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   eta_mu(x) = (-1)^(x0+...+x_{mu-1}); s_mu(x) = -1 on the time links from
 *   x3 = L3-1 to x3 = 0 when the time direction is antiperiodic, else +1.
 *   D_eo = D from odd to even sites, D_oe from even to odd sites.
 *   M = m^2 - D_eo D_oe on even sites (Hermitian positive definite).
 *
 * Geometry: dims = (L0,L1,L2,L3) = (x,y,z,t), every L_mu even and >= 2.
 *   lex(x) = x0 + L0*(x1 + L1*(x2 + L2*x3)), parity = (x0+x1+x2+x3) mod 2,
 *   eo(x) = lex(x) >> 1 indexes the V/2 sites of one parity.
 *
 * Layouts.
 *   Canonical links : complex128 (4, V, 3, 3) [mu][lex][row][col].
 *   Canonical vector: complex128 (V/2, 3) [eo][colour].
 *   Library vector  : structure of arrays [colour][eo] of complex numbers,
 *                     i.e. 3 planes of V/2 {re,im} pairs; double2 planes for
 *                     STAG_F64 (48*V/2 bytes), float2 planes for STAG_F32
 *                     (24*V/2 bytes).  stag_vec_pack/unpack convert.
 *   Packed links live inside the lattice handle (see stag_links_set).
 *
 * Pointers: every field pointer is a DEVICE pointer unless marked host.
 * The caller owns every buffer it passes; the library owns only the lattice
 * handle and the work buffers it allocates inside it.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 * are ordered on that stream; stag_dslash_eo, stag_normal_op, stag_vec_*,
 * stag_tables and stag_links_set are asynchronous, the solvers return after
 * the stream has finished their work.  One handle must not be used from two
 * streams (or host threads) at once.
 * Errors: no C++ exception crosses this boundary.  Every call returns a
 * stag_status; stag_last_error() gives a message for the calling thread.
 * Environment: STAG_LOG=1 prints one line per solve and trajectory on
 * stderr ("[stag] ..."); STAG_AUTOTUNE_CACHE=<file> keeps the batched
 * solver's timed launch shapes across processes (one line per layout). */
#ifndef STAG_H
#define STAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STAG_OK = 0,
    STAG_ENOCONV = 1,     /* max_iter reached; best iterate and stats returned */
    STAG_EBREAKDOWN = 2,  /* non-positive or non-finite curvature <p, A p> */
    STAG_EINVAL = -1,     /* invalid argument (see each call) */
    STAG_ENOMEM = -2,     /* device allocation failed */
    STAG_EHIP = -3,       /* a HIP runtime call failed */
    STAG_STATUS_INT_RANGE_ = 0x7fffffff   /* not a status: makes every int a valid value of the
                                            type, so a status received as an int can be checked */
} stag_status;

typedef enum {
    STAG_F64 = 0,    /* double precision vectors and links */
    STAG_F32 = 1,    /* single precision vectors and links, double reductions */
    STAG_MIXED = 2,  /* solvers only: single precision iterations with double
                        precision reliable updates and per-shift refinement */
    STAG_PREC_INT_RANGE_ = 0x7fffffff   /* not a precision: every int is a valid value of the type
                                           (callers pass ints; unknown ones get STAG_EINVAL) */
} stag_prec;

typedef enum {
    STAG_LINK18 = 0, /* all 9 complex entries of each link */
    STAG_LINK12 = 1, /* first two rows; third rebuilt as conj(row0 x row1)
                        (Section 5, 12-real representation); needs SU(3) links */
    STAG_LINK8 = 2,  /* not in the paper: U01, U02, U10 and the phases of U00
                        and U20; the rest rebuilt from unitarity and det U = 1.
                        Needs SU(3) links with U01, U02 not both zero */
    STAG_LINK18_PAIRS = 3, /* Section 5's float pairs: each double a stored as
                        b = float(a) and c = float(a - b) (a = b + c to about
                        2^-48 |a|), as the only device copy: the single
                        precision kernels read the b half, the double
                        precision ones b + c.  All 9 entries */
    STAG_LINK12_PAIRS = 4, /* the same for the first two rows (SU(3) links) */
    STAG_LINK_FMT_INT_RANGE_ = 0x7fffffff  /* not a format: every int is a valid value of the type */
} stag_link_fmt;

#define STAG_MAX_SHIFTS 64

typedef struct stag_lattice stag_lattice;

/* Solver statistics (host struct). */
typedef struct {
    int iters;                              /* Krylov iterations (multi-shift or CG) */
    int n_reliable;                         /* double precision reliable updates */
    int refine_iters;                       /* iterations of the per-shift refinement */
    int fallback_used;                      /* learned preconditioner abandoned */
    int iters_shift[STAG_MAX_SHIFTS];       /* iteration at which shift i froze */
    double resid_iter[STAG_MAX_SHIFTS];     /* iterated |zeta_i| ||r|| / ||b|| at freeze */
    double resid_true[STAG_MAX_SHIFTS];     /* FP64 ||b - (M+sigma_i) x_i|| / ||b|| at exit */
    double resid_unrefined[STAG_MAX_SHIFTS];/* STAG_MIXED: FP64 true residual before refinement */
    int refine_iters_shift[STAG_MAX_SHIFTS];/* STAG_MIXED: refinement iterations of shift i */
    double seconds;                         /* wall time of the call */
} stag_cg_stats;

/* Create a lattice handle for dims[4] (host array).  antiperiodic_t != 0
 * selects the antiperiodic fermion boundary in time.  Every L_mu must be
 * even, >= 2, and V/2 < 2^30.  STAG_EINVAL otherwise.  Uses the current
 * HIP device; the handle is tied to it. */
stag_status stag_lattice_create(const int dims[4], int antiperiodic_t, stag_lattice **out);

/* Free the handle and every device buffer it owns.  NULL is allowed. */
stag_status stag_lattice_destroy(stag_lattice *lat);

/* Number of sites of one parity, V/2 (0 for a NULL handle). */
int64_t stag_half_volume(const stag_lattice *lat);

/* Pack a gauge field into the handle.  links: device, canonical complex128
 * (4,V,3,3).  Both a double and a single precision copy are stored in the
 * even/odd structure-of-arrays layout (element-major, site index fastest;
 * Section 5 and its Figure 2), keeping all 9 entries, the first two rows or
 * 8 reals (fmt); the _PAIRS formats keep one field of float pairs for
 * both precisions instead (2/3 of the memory of the two copies).  Links
 * must be SU(3) for STAG_LINK12, STAG_LINK12_PAIRS and STAG_LINK8.  For
 * STAG_LINK8 the call rebuilds the double precision field on the device and
 * returns STAG_EINVAL (links left unset) if any entry is off by more than
 * 1e-12, which catches links that have no 8-real form; it then waits for
 * the stream.  Replaces earlier links. */
stag_status stag_links_set(stag_lattice *lat, const void *links, stag_link_fmt fmt, void *stream);

/* Test hook: write the geometry tables computed by the same device index
 * functions the operator kernels use.  All int32 device arrays:
 *   nbr  [2][8][V/2]: eo index of neighbour d of site (parity, eo);
 *                     d = 0..3 forward x+mu, d = 4..7 backward x-mu.
 *   coord[2][V/2][4]: coordinates.
 *   sign [2][8][V/2]: eta_mu(x) s_mu(x) (forward) / eta_mu(x) s_mu(x-mu)
 *                     (backward), excluding the 1/2 and the backward minus.
 * Any of the three may be NULL. */
stag_status stag_tables(const stag_lattice *lat, int32_t *nbr, int32_t *coord, int32_t *sign,
                        void *stream);

/* Canonical complex128 (V/2,3) vector <-> library vector of precision prec
 * (STAG_F64 or STAG_F32; F32 rounds to nearest). */
stag_status stag_vec_pack(const stag_lattice *lat, const void *canonical, void *vec, stag_prec prec,
                          void *stream);
stag_status stag_vec_unpack(const stag_lattice *lat, const void *vec, void *canonical, stag_prec prec,
                            void *stream);

/* Half hopping term.  out_parity = 0: out = D_eo in (odd -> even);
 * out_parity = 1: out = D_oe in (even -> odd).  in and out are library
 * vectors of precision prec (STAG_F64 or STAG_F32, using the matching link
 * copy); they must not share any byte (STAG_EINVAL otherwise).  Asynchronous. */
stag_status stag_dslash_eo(const stag_lattice *lat, int out_parity, const void *in, void *out,
                           stag_prec prec, void *stream);

/* out = (m^2 + shift) in - D_eo D_oe in on even sites; library vectors of
 * precision prec, sharing no byte (STAG_EINVAL otherwise).  Uses a work
 * vector inside the handle.
 * mass > 0, shift >= 0.  Asynchronous. */
stag_status stag_normal_op(stag_lattice *lat, double mass, double shift, const void *in, void *out,
                           stag_prec prec, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): stag_normal_op with the
 * odd-site temporary taken from a static device array of
 * stag_noalloc_scratch_bytes() bytes (32 MiB) instead of a work buffer.
 * Arguments, result and asynchrony as stag_normal_op; the same kernels run.
 * Allocates nothing (no hipMalloc, hipFree or allocating library call).
 * Returns STAG_EINVAL when the temporary (48 V/2 bytes in STAG_F64, 24 V/2
 * in STAG_F32) exceeds the array: a 32^4 lattice fits in either precision.
 * Each GPU holds its own copy of the array until the process ends; every
 * call on that GPU uses it, so calls that overlap in time on one GPU (two
 * streams or two host threads) race and must not be issued. */
size_t stag_noalloc_scratch_bytes(void);
stag_status stag_normal_op_noalloc(stag_lattice *lat, double mass, double shift, const void *in, void *out,
                                   stag_prec prec, void *stream);

/* Multi-shift CG (Section 6; Jegerlehner's method): solve
 *   (M + shifts[i]) x_i = src,  i = 0..n_shifts-1,
 * from x_i = 0 (the shifted solver needs the zero start: sols are outputs
 * only).  src and every sols[i] are STAG_F64 library vectors; shifts and
 * sols are HOST arrays (sols holds device pointers).  Shift i stops when
 * its iterated residual |zeta_i| ||r|| <= tol ||src||; the FP64 true
 * residual of every shift is computed at the end.
 *   prec = STAG_F64   : all double precision.
 *   prec = STAG_F32   : single precision vectors and links with double
 *                       reductions and recursion (reaches only the single
 *                       precision floor, Section 6).
 *   prec = STAG_MIXED : single precision iterations, double precision
 *                       reliable updates of the base residual (b - A x
 *                       recomputed whenever |r| fell tenfold since the last
 *                       one; checked every 8 iterations), then a mixed CG
 *                       refinement of every shift whose true residual
 *                       exceeds tol.
 * Requires mass > 0, shifts >= 0, tol > 0, 1 <= n_shifts <= 64, links set,
 * and no byte shared between two solutions or a solution and src.
 * ||src|| = 0 gives zero solutions and 0 iterations.  Returns STAG_ENOCONV
 * after max_iter iterations (stats filled), STAG_EBREAKDOWN on a
 * non-positive curvature.  stats may be NULL. */
stag_status stag_multishift_cg(stag_lattice *lat, double mass, const double *shifts, int n_shifts,
                               const void *src, void *const *sols, double tol, int max_iter,
                               stag_prec prec, stag_cg_stats *stats, void *stream);

/* Single-shift CG for (M + shift) x = src starting from the x passed in
 * (STAG_F64 library vectors sharing no byte; x is read and overwritten).  Stops when the
 * FP64 true residual is <= tol ||src||.  prec = STAG_F64, or STAG_MIXED for
 * single precision iterations with double precision reliable updates. */
stag_status stag_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x,
                    double tol, int max_iter, stag_prec prec, stag_cg_stats *stats, void *stream);

/* One system of a batched solve: (M + shifts[i]) x_i = src on `lat`
 * (links set), i < n_shifts.  src and sols[i] are STAG_F64 library vectors
 * of that lattice; shifts and sols are host arrays.  No solution may share a
 * byte with another solution or with any source of the batch. */
typedef struct {
    stag_lattice *lat;
    double mass;
    int n_shifts;
    const double *shifts;
    const void *src;
    void *const *sols;
} stag_system;

/* flags of stag_multishift_cg_batched */
#define STAG_BATCH_NO_GRAPH 0x1                 /* launch every kernel of every iteration instead of replaying graphs */
#define STAG_BATCH_PER_LATTICE 0x2              /* one multi-RHS Dslash launch per lattice instead of one for all */
#define STAG_BATCH_RPT(r) (((r) & 0xF) << 4)   /* force r right-hand sides per thread (1, 2, 4, 8) ... */
#define STAG_BATCH_BLOCK(b) ((((b) / 64) & 0xF) << 8) /* ... and b sites per block (64, 128, 256) */

/* Batched multi-shift CG: n_systems (1..64) independent shifted families --
 * several pseudo-fermions on one gauge field and/or lattices of different
 * sizes -- advanced together (Section 2 lists multiple pseudo-fermions among
 * the algorithm's tricks).  Systems whose `lat` is the same handle share
 * link loads in a multi-RHS Dslash (up to 8 right-hand sides per group);
 * the groups of every lattice run in one launch per phase, each group on
 * its own range of workgroups (STAG_BATCH_PER_LATTICE: one launch per
 * lattice and group instead); the vector updates and the scalar
 * recursions of all systems, whatever their lattice, run in one launch per
 * phase.  The launch shape of the multi-RHS Dslash (sites per block,
 * right-hand sides per launch) is timed on the first batch of each layout
 * and cached in the process, unless forced through flags.  The kernels of
 * a block of 16 iterations are captured once per call as a HIP graph (on a
 * private stream, where nothing executes) and the graph is replayed on
 * `stream` for every block; STAG_BATCH_NO_GRAPH launches them one by one
 * instead (same kernels, bit-identical results).  A done flag is read
 * after every block (every 8 iterations without graphs), one block behind.
 * Every shift of every system freezes on its own; each system has its own
 * recursion, mass and shifts; tol and max_iter are shared.
 * prec as for stag_multishift_cg (STAG_MIXED refines every shift that
 * misses tol in a second batched pass, warm-started).  All lattices must
 * use the same link format and device.  stats, if non-NULL, receives
 * n_systems entries.  Returns the worst status over the systems. */
stag_status stag_multishift_cg_batched(const stag_system *systems, int n_systems, double tol, int max_iter,
                                       stag_prec prec, int flags, stag_cg_stats *stats, void *stream);

/* Launch shape (sites per block, right-hand sides per thread) used by the
 * last batched solve of the calling thread. */
stag_status stag_batch_last_config(int *block, int *rpt);

/* ------------------------------------------------------------------ rational functions
 * The RHMC of Section 2 applies rational functions of M, in partial
 * fractions r(M) = alpha0 + sum_i alpha_i (M + shifts[i])^-1, to the
 * pseudo-fermion fields: r(M) ~ M^(1/4) (or another power) in the heatbath,
 * r(M) ~ M^(-1/2) in the action of the Metropolis step, whose inversions
 * Section 4 keeps in double precision.
 *
 * out = alpha0 src + sum_i alpha_i (M + shifts[i])^-1 src by one double
 * precision multi-shift CG from zero (Section 6).  The weighted solutions
 * are summed into out as the solver goes: no per-shift solution vector is
 * stored or returned.  src and out are STAG_F64 library vectors (sharing no
 * byte); alphas and shifts are HOST arrays of n (1..64) entries.  Shift
 * i stops when |zeta_i| ||r|| <= tol ||src||, so in exact arithmetic
 *   ||out - r(M) src|| <= tol ||src|| sum_i |alpha_i| / (m^2 + shifts[i]).
 * *dot (host, may be NULL) receives Re <src, out> (the action when src is
 * the pseudo-fermion field).  stats: iters, iters_shift, resid_iter and
 * seconds are filled; resid_true is left zero (no solutions are kept).
 * Requires mass > 0, shifts >= 0, finite alphas, tol > 0, links set.
 * Returns STAG_ENOCONV after max_iter iterations (out then holds the sum at
 * that iteration), STAG_EBREAKDOWN on a non-positive curvature.
 * Synchronous. */
stag_status stag_rational_apply(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                const double *shifts, int n, const void *src, void *out, double tol,
                                int max_iter, double *dot, stag_cg_stats *stats, void *stream);

/* The same rational function applied to n_rhs (1..64) fields of one
 * lattice -- several pseudo-fermions (Section 2) -- in one call: each field
 * is a system of the batched solver, so the multi-RHS half-Dslash loads
 * every link once for up to 8 fields.  srcs and outs are HOST arrays of
 * n_rhs device pointers (STAG_F64 library vectors; no output may share a
 * byte with a source or another output: STAG_EINVAL); dots (host, n_rhs entries, may be NULL)
 * receives Re <src_k, out_k>; stats (host, n_rhs entries, may be NULL) as
 * for stag_rational_apply.  Each field stops on its own; the error bound of
 * stag_rational_apply holds for each.  Synchronous. */
stag_status stag_rational_apply_multi(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                      const double *shifts, int n, const void *const *srcs, void *const *outs,
                                      int n_rhs, double tol, int max_iter, double *dots, stag_cg_stats *stats,
                                      void *stream);

/* Zolotarev's optimal relative approximation of x^(-1/2) (power = -1) or
 * x^(1/2) = x * x^(-1/2) (power = +1) on [lo, hi] (0 < lo < hi), with n
 * poles (1..64): writes *alpha0, alphas[n], shifts[n] (HOST arrays; all
 * shifts > 0) and *max_rel_err = max |r(x) / x^power - 1| over [lo, hi]
 * (may be NULL).  Host computation, no GPU needed. */
stag_status stag_zolotarev(int power, double lo, double hi, int n, double *alpha0, double *alphas,
                           double *shifts, double *max_rel_err);

/* Best relative rational approximation of x^power on [lo, hi] for power in
 * (-1, 0) or (0, 1) (M^(1/4) for the two-flavour heatbath, M^(-1/4),
 * M^(1/8), ...), same output convention as stag_zolotarev.  Negative powers
 * get type (n-1, n) (alpha0 = 0, residues > 0); positive powers q use
 * x^q = x * x^(q-1) (alpha0 > 0, residues < 0).  +-1/2 is Zolotarev's
 * closed form; other powers come from Remez's exchange algorithm, continued
 * in the power from that closed form (1 <= n <= 24).  Once the error falls
 * below 1e-12 the coefficients are returned as they stand (double precision
 * rounding leaves no alternation to resolve); STAG_EINVAL if the iteration
 * fails to converge above that level.  Host computation. */
stag_status stag_rational_power(double power, double lo, double hi, int n, double *alpha0, double *alphas,
                                double *shifts, double *max_rel_err);

/* Pseudo-fermion force of the RHMC (Section 2: the molecular dynamics force
 * of the rational action, from the multi-shift solutions).  For
 * S = sum_i alphas[i] <phi, (M + sigma_i)^-1 phi> with the solutions
 * x[i] = (M + sigma_i)^-1 phi (n DEVICE pointers in a HOST array, even-site
 * vectors in the library layout, double precision), writes
 *   force[mu][lex] = TA(U_mu(x) W_mu(x))
 * where W_mu(x) = sum_i alphas[i] eta_mu(x) s_mu(x) (D_oe x_i)(x+mu) x_i(x)^dag
 * for even x and -sum_i alphas[i] eta_mu(x) s_mu(x) x_i(x+mu) (D_oe x_i)(x)^dag
 * for odd x, and TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6.  Moving one link
 * U -> exp(i eps T) U (T Hermitian, traceless) changes S at the rate
 * i tr(T F).  force: DEVICE buffer of 4*V*9 complex doubles in the layout of
 * stag_links_set's input (mu, lex, row, col), overwritten.  0 <= n <= 64
 * (n = 0 writes zeros); alphas finite.  Uses the double precision link field
 * of any format.  Asynchronous on `stream`; x and force must stay valid
 * until the stream reaches this point.  STAG_EINVAL on a null pointer, n out
 * of range, a non-finite alpha, a force buffer sharing a byte with a
 * solution, or links not set. */
stag_status stag_fermion_force(stag_lattice *lat, int n, const double *alphas, const void *const *x, void *force,
                               void *stream);

/* ------------------------------------------------------------------ RHMC trajectory
 * Section 2 of the paper: RHMC for staggered fermions with a multi-step
 * second order minimum norm integrator that splits the action into its
 * gauge and fermion parts, several pseudo-fermions and rational
 * approximations; Section 4: the gauge update in single precision with a
 * double precision reunitarisation, single precision inversions in the
 * molecular dynamics, double precision inversions for the Metropolis step.
 * The paper prints no formula; the library takes:
 *   S_g = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3)      (Wilson)
 *   P_mu(x) = sum_a p_a lambda_a / 2, K = (1/2) sum p_a^2, dU/dt = i P U,
 *   a force F (dS/deps = i tr(T F) for U -> exp(i eps T) U) kicks
 *   p_a += h Im tr(lambda_a F) / 2,
 *   gauge force -(beta/3) TA(U_mu(x) A_mu(x)) (A: the six staples),
 *   S_f = sum_k <phi_k, r(M) phi_k>, heatbath phi_k = r_hb(M) xi_k.
 * Momenta are DEVICE float64 arrays (4, V, 8) [mu][lex][a] (algebra
 * coordinates p_a, Gell-Mann order).  The calls that change the links need
 * them stored as STAG_LINK18_PAIRS or STAG_LINK12_PAIRS (the paper's
 * float-pair field, Section 5): an update in single precision reads the
 * single precision half, multiplies by exp(i h P) in single precision and
 * reorthonormalises in double precision (rows 0 and 1 by Gram-Schmidt, row
 * 2 = conj(row0 x row1)) before storing the new pair. */
#define STAG_MAX_PSEUDOFERMIONS 16

/* r(M) = alpha0 + sum_{i<n} alpha[i] (M + shift[i])^-1, 1 <= n <= 64. */
typedef struct {
    double alpha0;
    int n;
    double alpha[STAG_MAX_SHIFTS];
    double shift[STAG_MAX_SHIFTS];
} stag_rational;

typedef struct {
    double beta;        /* gauge coupling, >= 0 */
    double mass;        /* > 0 */
    double tau;         /* trajectory length, > 0 */
    int n_md;           /* outer (fermion) steps of the integrator, >= 1 */
    int n_g;            /* gauge steps per half outer step, >= 1 */
    stag_prec md_prec;  /* STAG_F32: single precision momenta, gauge update and force
                           inversions (the paper's choice); STAG_F64: all double */
    int max_iter;       /* iteration limit of every inversion */
    double tol_md;      /* relative residual of the molecular-dynamics inversions */
    double tol_act;     /* relative residual of the heatbath and Metropolis inversions */
    stag_rational rat_md;   /* force of the molecular dynamics */
    stag_rational rat_act;  /* Metropolis action */
    stag_rational rat_hb;   /* heatbath */
} stag_rhmc_params;

typedef struct {
    double dH;          /* H(end) - H(start) */
    double H0[3];       /* kinetic, gauge, fermion energy at the start */
    double H1[3];       /* the same at the end of the molecular dynamics */
    int accepted;
    int fermion_forces; /* pseudo-fermion force evaluations (all fields) */
    int gauge_forces;
    int md_iters;       /* multi-shift iterations of the molecular dynamics */
    int action_iters;   /* multi-shift iterations of the heatbath and the action */
    double seconds;
} stag_rhmc_info;

/* Canonical complex128 (4, V, 3, 3) copy of the double precision link field
 * (rows a compressed format does not store are rebuilt).  Asynchronous. */
stag_status stag_links_get(const stag_lattice *lat, void *links, void *stream);

/* Gauge force F_mu(x) = -(beta/3) TA(U_mu(x) A_mu(x)) into force (DEVICE,
 * (4, V, 3, 3) complex128), computed in prec (STAG_F64: double precision
 * links and arithmetic; STAG_F32: the single precision field and
 * arithmetic).  Any link format.  Asynchronous. */
stag_status stag_gauge_force(stag_lattice *lat, double beta, void *force, stag_prec prec, void *stream);

/* S_g in double precision from the double precision field (any format),
 * summed in a fixed order; *action is a HOST double.  Synchronous. */
stag_status stag_gauge_action(stag_lattice *lat, double beta, double *action, void *stream);

/* One molecular-dynamics step each, on momenta mom (DEVICE (4, V, 8)
 * float64, converted to prec and back), in precision prec:
 *   stag_gauge_kick : p_a += h Im tr(lambda_a F_g) / 2 (gauge force, beta);
 *   stag_force_kick : p_a += h Im tr(lambda_a F) / 2 for a given force
 *                     (DEVICE (4, V, 3, 3) complex128, e.g. stag_fermion_force's);
 *   stag_link_update: U <- reunitarise(exp(i h P) U), pair formats only; mom
 *                     is read only.
 * Asynchronous. */
stag_status stag_gauge_kick(stag_lattice *lat, double beta, double h, double *mom, stag_prec prec, void *stream);
stag_status stag_force_kick(stag_lattice *lat, const void *force, double h, double *mom, stag_prec prec,
                            void *stream);
stag_status stag_link_update(stag_lattice *lat, const double *mom, double h, stag_prec prec, void *stream);

/* Molecular dynamics for a time prm->tau from the lattice's links and the
 * momenta mom (both updated in place) with the n_pf pseudo-fermion fields
 * phis (HOST array of DEVICE double precision library vectors, fixed during
 * the integration), in prm->md_prec.  info (HOST, may be NULL) receives the
 * force and iteration counts.  Several fields (the paper's multiple
 * pseudo-fermions, Section 2) whose solutions number at most 64 in all
 * (n_pf * prm->rat_md.n) have their solves run as one batched solve and
 * their force as one force call per kick; otherwise field by field.  The
 * result is the same up to rounding.  Synchronous.  STAG_EINVAL on invalid
 * parameters or links not stored as float pairs. */
stag_status stag_md_integrate(stag_lattice *lat, const stag_rhmc_params *prm, double *mom, int n_pf,
                              const void *const *phis, stag_rhmc_info *info, void *stream);

/* One RHMC trajectory: phi_k = r_hb(M) xi_k (double precision), H0 = K +
 * S_g + sum_k |xi_k|^2, the molecular dynamics with r_md, H1 = K + S_g +
 * sum_k <phi_k, r_act(M) phi_k> (double precision), and the Metropolis test
 * against the uniform number u: accepted when u < 0 or u < exp(-dH).  On
 * rejection the links return to their initial values.  mom (DEVICE (4, V,
 * 8) float64) holds the momenta drawn by the caller on entry and the final
 * momenta on exit; xis: HOST array of n_pf DEVICE double precision
 * Gaussian library vectors.  With several fields the heatbath and the
 * action apply their rational function to all fields in one batched call.
 * Synchronous. */
stag_status stag_rhmc_trajectory(stag_lattice *lat, const stag_rhmc_params *prm, double *mom, int n_pf,
                                 const void *const *xis, double u, stag_rhmc_info *info, void *stream);

/* ------------------------------------------------------------------ learned preconditioner
 * Not part of the paper: an extension that preconditions the double
 * precision single-shift solve of the Metropolis step (Section 4 keeps that
 * inversion in double precision; Section 6 uses CG for it).
 *
 * Network P(r), r on even sites, 8 channels, weights shared by all sites and
 * colours (so P commutes with gauge transformations and is linear in r):
 *   hops    (T_{+mu} psi)(x) = eta_mu(x) s_mu(x)    U_mu(x)        psi(x+mu)
 *           (T_{-mu} psi)(x) = eta_mu(x) s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu)
 *           d = mu for +mu, d = 4 + mu for -mu (eta, s as in the operator).
 *   layer 1 phi1[c](x) = w1s[c] r(x) on even x,
 *           phi1[c](y) = sum_d w1h[c][d] (T_d r)(y) on odd y;
 *   layer 2 on even x: inputs f_c' = phi1[c'](x), f_{8+8d+c'} = (T_d phi1[c'])(x),
 *           phi2[c](x) = sum_k W2[c][k] f_k(x)  (72 inputs per channel);
 *   output  P(r)(x) = sum_c wout[c] phi2[c](x).
 * Parameters: 656 complex numbers theta = [w1s(8) | w1h(8x8, [c][d]) |
 * W2(8x72, [c][k]) | wout(8)], passed through the ABI as 1312 doubles
 * (re, im interleaved); the device keeps FP32 master copies.
 * r and outputs are STAG_F32 library vectors of the lattice; the network
 * reads the lattice's single precision links.
 * mode 0: layer-2 channel mixing in BF16 on the matrix cores with FP32
 *         accumulation;
 * mode 1: the same mixing in FP32 on the vector ALU (a check of mode 0);
 * mode 2: the folded form.  The network is linear and the hops act on
 *         colour only, so with v_k = sum_c wout[c] W2[c][k] it equals
 *           P r = s r + sum_d T_d psi_d,  psi_d = sum_d' A[d][d'] T_d' r (odd sites),
 *           s = sum_c v_c w1s[c],  A[d][d'] = sum_c v_{8+8d+c} w1h[c][d'];
 *         evaluated in FP32, layer 2 then gathers one colour vector per hop
 *         instead of eight.  Forward only (stag_net_apply, stag_fcg_solve).
 * mode 3: the folded form reading a bfloat16 copy of the links (12 reals,
 *         third row rebuilt; made from the single precision field on first
 *         use, kept with the lattice until its links are replaced) and
 *         storing psi_d in bfloat16; arithmetic in FP32.  Entries of P r
 *         carry relative errors of order 1e-2, which the flexible CG
 *         absorbs.  Forward only.
 * The backward pass is FP32 in modes 0 and 1; gradients are summed in a
 * fixed order (deterministic). */
typedef struct stag_net stag_net;

/* Create a network on the current device with every parameter zero. */
stag_status stag_net_create(stag_net **out);
stag_status stag_net_destroy(stag_net *net);

/* Set / read the 656 complex parameters (HOST arrays of 1312 doubles).
 * Setting them resets the optimiser state.  Synchronous. */
stag_status stag_net_set_params(stag_net *net, const double *theta);
stag_status stag_net_get_params(const stag_net *net, double *theta);

/* out = P(r).  Asynchronous on `stream`.  r and out must not share a byte
 * (STAG_EINVAL). */
stag_status stag_net_apply(stag_net *net, stag_lattice *lat, const void *r, void *out, int mode,
                           void *stream);

/* Gradient of L = Re sum_x <g(x), P(r)(x)> with respect to the parameters,
 * written to the HOST array grad[1312] as dL/dRe, dL/dIm of each theta_j.
 * r, g: STAG_F32 library vectors; mode 0 or 1.  Synchronous. */
stag_status stag_net_grad(stag_net *net, stag_lattice *lat, const void *r, const void *g, double *grad,
                          int mode, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on the
 * loss (1/n) sum_k ||P(b_k) - x_k||^2 / ||x_k||^2 over n pairs (1..1024).
 * b, x: n STAG_F32 library vectors stored back to back (3*V/2 float2 each).
 * *loss (host, may be NULL) receives the loss before the step; when loss
 * is non-NULL the call waits for the stream. */
stag_status stag_net_train_step(stag_net *net, stag_lattice *lat, const void *b, const void *x, int n,
                                double lr, int mode, double *loss, void *stream);

/* Flexible CG with P as preconditioner (Polak-Ribiere beta) for
 * (M + shift) x = src from the x passed in (STAG_F64 library vectors sharing
 * no byte; sol
 * is read and overwritten).  The network is evaluated in `mode` (0 to 3)
 * on a single precision copy of the residual; everything else is double
 * precision.  net == NULL runs plain double precision CG.  The residual is
 * re-computed in double precision from x whenever the iterated one reaches
 * tol ||src|| (the double precision check); the iteration stops if it
 * meets tol, else it restarts from it.  The solver falls back to plain double precision CG,
 * warm-started, when <r, P r> <= 0, a curvature is not positive or finite,
 * or the residual stalls for 50 iterations (stats->fallback_used = 1).
 * stats->iters counts both parts; stats->resid_true[0] is the final
 * relative true residual.  Synchronous. */
stag_status stag_fcg_solve(stag_lattice *lat, double mass, double shift, const void *src, void *sol,
                           stag_net *net, int mode, double tol, int max_iter, stag_cg_stats *stats,
                           void *stream);

/* Bandwidth probe used by the benchmark to measure the achievable HBM rate
 * in the same run.  kind 0: read `bytes` from src (dst receives nothing in
 * practice but must hold 8192*256 floats); kind 1: copy `bytes` from src to
 * dst.  bytes must be a multiple of 16.  Asynchronous. */
stag_status stag_hbm_probe(const void *src, void *dst, int64_t bytes, int kind, void *stream);

/* Message of a status code, and the last error message of this thread. */
const char *stag_status_string(stag_status s);
const char *stag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STAG_H */
