// Host-side internals shared by the library's translation units: the
// lattice handle, work buffers, error reporting and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "stag.h"
#include "geom.h"

namespace stag {

// A named range of rocprofv3's marker trace (`--marker-trace`) over a scope:
// the solver phases show up as ranges beside their kernels.  Without a tool
// attached a push or pop is a call that returns at once.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
const char *last_error();

#define STAG_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::stag::set_error(std::string(#call) + ": " + hipGetErrorString(e_));            \
            return e_ == hipErrorOutOfMemory ? STAG_ENOMEM : STAG_EHIP;                       \
        }                                                                                    \
    } while (0)

#define STAG_TRY(call)                                                                       \
    do {                                                                                     \
        stag_status s_ = (call);                                                             \
        if (s_ != STAG_OK) return s_;                                                        \
    } while (0)

// Diagnostic messages on stderr, "[stag] ..." plus a newline, when the
// environment variable STAG_LOG is set to a level >= `level` (1: one line
// per solve or trajectory, 2: also per phase).  Read at every call.
void stag_log(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

inline stag_status invalid(const std::string &msg) {
    set_error(msg);
    return STAG_EINVAL;
}

// A device buffer the caller passes: its first byte and its length.
struct ByteRange {
    const void *p;
    size_t n;
};
inline bool ranges_overlap(const ByteRange &a, const ByteRange &b) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a.p), y = reinterpret_cast<uintptr_t>(b.p);
    return a.n && b.n && x < y + b.n && y < x + a.n;
}
// True when the outputs are pairwise disjoint and none overlaps an input
// (inputs may overlap each other: they are only read).  O(n log n).
bool outputs_disjoint(const ByteRange *outs, int n_out, const ByteRange *ins, int n_in);

// ---------------------------------------------------------------- kernels
enum DslashMode {
    DS_PLAIN = 0,       // out = D in
    DS_NORMAL = 1,      // out = c aux - D in
    DS_NORMAL_DOT = 2,  // out = c aux - D in, partial[block] = sum Re<aux, out>
    DS_RESID = 3        // r = rhs - (c aux - D in), partial[block] = sum |r|^2, out = r if non-null
};

struct DslashArgs {
    Geom g;
    int out_parity;
    const void *links;   // packed links matching the precision
    const void *in;      // opposite-parity vector
    void *out;           // output-parity vector
    const void *aux;     // output-parity vector (p for DS_NORMAL*, x for DS_RESID)
    const void *rhs;     // DS_RESID: right-hand side (double)
    double c;            // m^2 + shift
    double *partial;     // per-block partial sums (dot modes)
    const int *skip;     // if non-null and *skip != 0 the launch does nothing
    unsigned link_cache; // 8-real double precision links: bit b set = link block b read with ordinary loads
};

constexpr int kDslashBlock = 256;
int dslash_grid(const Geom &g, int block);
hipError_t launch_dslash(bool dbl, int nrow, int mode, const DslashArgs &a, hipStream_t s);
// D_oe in double precision of n even-site vectors of `lat`, rpt (1, 2, 4
// or 8) per launch of the multi-right-hand-side half-Dslash (the links read
// once for all of them); block: 64, 128 or 256 sites per workgroup.
hipError_t launch_dslash_oe_multi(const stag_lattice *lat, int n, const void *const *in, void *const *out, int block,
                                  int rpt, hipStream_t s);
// The double precision true residuals r_i = b - (M + shift_i) x_i of n
// solutions, eight per launch pair: t_r = D_oe x_r into t[r] (8 odd-site
// vectors), then r_i = b - (c[i] x_i - D_eo t_r) with c[i] = m^2 + shift_i
// and one partial of |r_i|^2 per 64 consecutive sites into part[i]
// (ceil(V/2 / 64) of them); r_i itself is not stored.
hipError_t launch_true_resid_multi(const stag_lattice *lat, int n, const void *const *x, const double *c,
                                   const void *b, void *const *t, double *const *part, int block, hipStream_t s);

hipError_t launch_pack_links(const Geom &g, const void *canon, void *dst, bool dbl, int nrow, hipStream_t s);
// bfloat16 12-real copy from a packed single precision field of any format
hipError_t launch_pack_links16(const Geom &g, const void *links32, int nrow, void *dst, hipStream_t s);
// largest entry-wise |rebuilt - canonical| of a packed double precision field, one partial per block
int check_links_blocks(const Geom &g);
hipError_t launch_check_links(const Geom &g, const void *canon, const void *packed64, int nrow, double *partial,
                              hipStream_t s);
// packed double precision field -> canonical complex128 (4,V,3,3)
hipError_t launch_unpack_links(const Geom &g, const void *packed64, int nrow, void *canon, hipStream_t s);
hipError_t launch_pack_vec(const Geom &g, const void *canon, void *dst, bool dbl, hipStream_t s);
hipError_t launch_unpack_vec(const Geom &g, const void *src, void *canon, bool dbl, hipStream_t s);
hipError_t launch_tables(const Geom &g, int32_t *nbr, int32_t *coord, int32_t *sign, hipStream_t s);

}  // namespace stag

// ---------------------------------------------------------------- handle
enum WsSlot {
    WS_T = 0,      // odd-parity temporary (double or float)
    WS_T2,         // second odd temporary
    WS_R,          // residual
    WS_AP,         // A p
    WS_P,          // search directions of every shift
    WS_XLO,        // single precision solution accumulators (mixed)
    WS_RHI,        // double precision residual (reliable updates)
    WS_E,          // even temporary
    WS_E2,         // second even temporary
    WS_PART,       // reduction partials
    WS_STATE,      // solver scalar state
    WS_BATCH,      // arena of the batched solver
    WS_FORCE,      // odd-site vectors D_oe X_i of the fermion force
    WS_TRES,       // odd-site temporaries and partials of the final true residuals
    WS_MD_MOM,     // momenta of the molecular dynamics (library layout)
    WS_MD_SOLS,    // multi-shift solutions of the molecular-dynamics force
    WS_MD_FORCE,   // pseudo-fermion force (4, V, 3, 3)
    WS_MD_LINKS,   // copy of the links at the start of a trajectory (rejection)
    WS_MD_PHI,     // pseudo-fermion fields of a trajectory
    WS_MD_OUT,     // output vector of the Metropolis action
    WS_MD_PART,    // reduction partials of the energies
    WS_NSLOTS
};

struct stag_lattice {
    int dims[4];
    int antiperiodic;
    int64_t V, Vh;
    stag::Geom g;
    int device;
    int nrow;            // rows stored per link (3 or 2), 0 before stag_links_set
    void *links64;
    void *links32;
    void *links16;       // bfloat16 12-real copy for the learned preconditioner (packed on first use)
    unsigned link_cache; // link blocks the solver's double precision Dslash reads cached (link_cache_mask)
    bool vec_stream;     // the solver's double precision vector kernels stream (nontemporal access)
    void *ws[WS_NSLOTS];
    size_t ws_bytes[WS_NSLOTS];
    int *host_flags;     // pinned host mirror of solver flags
};

namespace stag {

// Work buffer of at least `bytes` bytes in slot `slot` (grown on demand).
stag_status ws_get(stag_lattice *lat, int slot, size_t bytes, void **out);

inline int64_t vec_bytes(const stag_lattice *lat, bool dbl) { return (dbl ? 48 : 24) * lat->Vh; }

// Infinity Cache residency of a double precision link field of `nrow` rows
// (only the 8-real form, nrow = 1, gets any): the set of
// its 8 link blocks (parity * 4 + mu) that the solver's Dslash reads with
// ordinary loads, so that they stay in the 256 MB Infinity Cache from one
// launch to the next.  A field within the budget is cached whole; a larger
// one caches whole blocks in the order 0, 4, 1, 5, 2, 6, 3, 7 while they
// fit, and streams the rest.  *stream tells whether the solver's vector
// kernels should then stream too (a partly cached field), so that they do
// not push those blocks out.
unsigned link_cache_mask(int nrow, int64_t vh, bool *stream);

}  // namespace stag
