// The C ABI (include/stag.h): argument validation, handle and work-buffer
// management, and dispatch to the kernels and solver drivers.  No C++
// exception crosses this boundary.
#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "links.h"
#include "batch.h"
#include "solver.h"

namespace stag {

bool outputs_disjoint(const ByteRange *outs, int n_out, const ByteRange *ins, int n_in) {
    std::vector<ByteRange> o(outs, outs + n_out);
    std::sort(o.begin(), o.end(), [](const ByteRange &a, const ByteRange &b) {
        return reinterpret_cast<uintptr_t>(a.p) < reinterpret_cast<uintptr_t>(b.p);
    });
    for (size_t k = 1; k < o.size(); ++k)
        if (ranges_overlap(o[k - 1], o[k])) return false;
    for (int j = 0; j < n_in; ++j) {
        // the only outputs that can overlap ins[j] start before its end: check the last of them
        const uintptr_t end = reinterpret_cast<uintptr_t>(ins[j].p) + ins[j].n;
        auto it = std::lower_bound(o.begin(), o.end(), end, [](const ByteRange &a, uintptr_t e) {
            return reinterpret_cast<uintptr_t>(a.p) < e;
        });
        if (it != o.begin() && ranges_overlap(*(it - 1), ins[j])) return false;
    }
    return true;
}

void stag_log(int level, const char *fmt, ...) {
    const char *env = std::getenv("STAG_LOG");
    if (!env || std::atoi(env) < level) return;
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[stag] %s\n", buf);
    std::fflush(stderr);
}

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

stag_status ws_get(stag_lattice *lat, int slot, size_t bytes, void **out) {
    if (bytes == 0) bytes = 16;
    if (lat->ws_bytes[slot] < bytes) {
        if (lat->ws[slot]) {
            // the buffer may still be in use by queued work
            STAG_HIP(hipDeviceSynchronize());
            STAG_HIP(hipFree(lat->ws[slot]));
            lat->ws[slot] = nullptr;
            lat->ws_bytes[slot] = 0;
        }
        STAG_HIP(hipMalloc(&lat->ws[slot], bytes));
        lat->ws_bytes[slot] = bytes;
    }
    *out = lat->ws[slot];
    return STAG_OK;
}

stag_status multishift_cg(stag_lattice *lat, double mass, const double *shifts, int n, const void *src,
                          void *const *sols, double tol, int max_iter, stag_prec prec, stag_cg_stats *stats,
                          hipStream_t s);
stag_status single_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol,
                      int max_iter, stag_prec prec, stag_cg_stats *stats, hipStream_t s);
stag_status fermion_force(stag_lattice *lat, int n, const double *alphas, const void *const *x, void *force,
                          hipStream_t s);
stag_status rational_apply(stag_lattice *lat, double mass, double alpha0, const double *alphas, const double *shifts,
                           int n, const void *src, void *out, double tol, int max_iter, double *dot,
                           stag_cg_stats *stats, hipStream_t s);
stag_status zolotarev(int power, double lo, double hi, int n, double *alpha0, double *alphas, double *shifts,
                      double *delta_out);
stag_status rational_power(double power, double lo, double hi, int n, double *alpha0, double *alphas, double *shifts,
                           double *delta_out);

stag_status gauge_action(stag_lattice *lat, double beta, double *out, hipStream_t s);
stag_status gauge_force_out(stag_lattice *lat, double beta, void *force, bool dbl, hipStream_t s);
stag_status mom_step(stag_lattice *lat, double *mom_canon, int kind, double beta, const void *force, double h,
                     bool dbl, hipStream_t s);
stag_status check_md_params(const stag_lattice *lat, const stag_rhmc_params *prm, int n_pf, bool trajectory);
stag_status md_integrate(stag_lattice *lat, const stag_rhmc_params *prm, double *mom_canon, int n_pf,
                         const void *const *phis, stag_rhmc_info *info, hipStream_t s);
stag_status rhmc_trajectory(stag_lattice *lat, const stag_rhmc_params *prm, double *mom_canon, int n_pf,
                            const void *const *xis, double u, stag_rhmc_info *info, hipStream_t s);

static stag_status use_device(const stag_lattice *lat) {
    int dev = -1;
    STAG_HIP(hipGetDevice(&dev));
    if (dev != lat->device) STAG_HIP(hipSetDevice(lat->device));
    return STAG_OK;
}

static stag_status check_lattice(const stag_lattice *lat, bool need_links) {
    if (!lat) return invalid("null lattice handle");
    if (need_links && !lat->nrow) return invalid("links not set (call stag_links_set first)");
    return use_device(lat);
}

static bool prec_ok(stag_prec p) { return p == STAG_F64 || p == STAG_F32; }

// The budget leaves about a third of the 256 MB Infinity Cache to the
// vectors.  Measured with the 32^4 FP64 multi-shift solve on 8-real links
// (33.5 MB per block; two machines), cached blocks against solve time, the
// vector kernels streaming: none 0.0993-0.1007 s, 4: 0.0945-0.0948, 5:
// 0.0927, 6: 0.0930-0.0943, 7: 0.0939-0.0945, all 8: 0.0979-0.0983; 6
// blocks with cached vector kernels 0.0972.
constexpr int64_t kLinkCacheBudget = 176ll << 20;

unsigned link_cache_mask(int nrow, int64_t vh, bool *stream) {
    *stream = false;
    if (nrow != 1) return 0u;   // 18- and 12-real fields stream (not measured with cached blocks)
    const int64_t blk = link_field_bytes(true, nrow, vh) / 8;
    if (8 * blk <= kLinkCacheBudget) return 0xffu;
    static const int order[8] = {0, 4, 1, 5, 2, 6, 3, 7};
    unsigned m = 0;
    int64_t used = 0;
    for (int k = 0; k < 8 && used + blk <= kLinkCacheBudget; ++k) {
        m |= 1u << order[k];
        used += blk;
    }
    *stream = m != 0;
    return m;
}

}  // namespace stag

using namespace stag;

extern "C" {

stag_status stag_lattice_create(const int dims[4], int antiperiodic_t, stag_lattice **out) {
    try {
        if (!dims || !out) return invalid("null argument");
        *out = nullptr;
        int64_t v = 1;
        for (int mu = 0; mu < 4; ++mu) {
            if (dims[mu] < 2 || (dims[mu] & 1))
                return invalid("every lattice extent must be even and >= 2 (dim " + std::to_string(mu) + " = " +
                               std::to_string(dims[mu]) + ")");
            v *= dims[mu];
        }
        if (v / 2 >= (int64_t(1) << 30)) return invalid("lattice too large (V/2 must be < 2^30)");
        stag_lattice *lat = new stag_lattice;
        std::memset(lat, 0, sizeof(*lat));
        for (int mu = 0; mu < 4; ++mu) lat->dims[mu] = dims[mu];
        lat->antiperiodic = antiperiodic_t ? 1 : 0;
        lat->V = v;
        lat->Vh = v / 2;
        lat->g = make_geom(dims, lat->antiperiodic);
        hipError_t e = hipGetDevice(&lat->device);
        if (e == hipSuccess) e = hipHostMalloc((void **)&lat->host_flags, 4 * sizeof(int), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_error(std::string("device set-up failed: ") + hipGetErrorString(e));
            delete lat;
            return STAG_EHIP;
        }
        *out = lat;
        return STAG_OK;
    } catch (...) {
        set_error("allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_lattice_destroy(stag_lattice *lat) {
    if (!lat) return STAG_OK;
    (void)hipSetDevice(lat->device);
    (void)hipDeviceSynchronize();
    if (lat->links64 != lat->links32) (void)hipFree(lat->links64);   // one field when stored as float pairs
    (void)hipFree(lat->links32);
    (void)hipFree(lat->links16);
    for (int k = 0; k < WS_NSLOTS; ++k) (void)hipFree(lat->ws[k]);
    (void)hipHostFree(lat->host_flags);
    delete lat;
    return STAG_OK;
}

int64_t stag_half_volume(const stag_lattice *lat) { return lat ? lat->Vh : 0; }

// Largest entry error accepted when a field is stored in 8 reals (double
// precision rebuild; smoothed and Haar fields stay below 3e-14).
static constexpr double kLink8MaxError = 1e-12;

stag_status stag_links_set(stag_lattice *lat, const void *links, stag_link_fmt fmt, void *stream) {
    STAG_TRY(check_lattice(lat, false));
    if (!links) return invalid("null links");
    if (fmt != STAG_LINK18 && fmt != STAG_LINK12 && fmt != STAG_LINK8 && fmt != STAG_LINK18_PAIRS &&
        fmt != STAG_LINK12_PAIRS)
        return invalid("unknown link format");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nrow = fmt == STAG_LINK8 ? 1 : fmt == STAG_LINK12 ? 2 : fmt == STAG_LINK18 ? 3
                                                                 : fmt == STAG_LINK12_PAIRS ? kHiLo + 2 : kHiLo + 3;
    STAG_HIP(hipStreamSynchronize(s));
    if (lat->links64 && lat->links64 != lat->links32) STAG_HIP(hipFree(lat->links64));
    if (lat->links32) STAG_HIP(hipFree(lat->links32));
    if (lat->links16) STAG_HIP(hipFree(lat->links16));
    lat->links64 = lat->links32 = lat->links16 = nullptr;
    lat->nrow = 0;
    lat->link_cache = 0;
    lat->vec_stream = false;
    if (nrow > kHiLo) {
        // one field: single precision values, then their double precision remainders
        STAG_HIP(hipMalloc(&lat->links32, link_field_bytes(true, nrow, lat->Vh)));
        lat->links64 = lat->links32;
        STAG_HIP(launch_pack_links(lat->g, links, lat->links64, true, nrow, s));
    } else {
        STAG_HIP(hipMalloc(&lat->links64, link_field_bytes(true, nrow, lat->Vh)));
        STAG_HIP(hipMalloc(&lat->links32, link_field_bytes(false, nrow, lat->Vh)));
        STAG_HIP(launch_pack_links(lat->g, links, lat->links64, true, nrow, s));
        STAG_HIP(launch_pack_links(lat->g, links, lat->links32, false, nrow, s));
    }
    if (nrow == 1) {
        // the 8-real form needs u01, u02 not both zero: check the rebuilt field
        const int nb = check_links_blocks(lat->g);
        void *part = nullptr;
        STAG_TRY(ws_get(lat, WS_PART, sizeof(double) * nb, &part));
        STAG_HIP(launch_check_links(lat->g, links, lat->links64, nrow, static_cast<double *>(part), s));
        std::vector<double> h(nb);
        STAG_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
        STAG_HIP(hipStreamSynchronize(s));
        double worst = 0.0;
        for (double v : h) worst = (v > worst || v != v) ? v : worst;
        if (!(worst <= kLink8MaxError)) {
            char buf[32];
            std::snprintf(buf, sizeof(buf), "%.3g", worst);
            set_error(std::string("links not representable in 8 reals (rebuilt entries off by ") + buf +
                      "; a link with u01 = u02 = 0, e.g. the unit matrix, has no 8-real form)");
            return STAG_EINVAL;
        }
    }
    lat->nrow = nrow;
    lat->link_cache = link_cache_mask(nrow, lat->Vh, &lat->vec_stream);
    return STAG_OK;
}

stag_status stag_tables(const stag_lattice *lat, int32_t *nbr, int32_t *coord, int32_t *sign, void *stream) {
    STAG_TRY(check_lattice(lat, false));
    STAG_HIP(launch_tables(lat->g, nbr, coord, sign, static_cast<hipStream_t>(stream)));
    return STAG_OK;
}

stag_status stag_vec_pack(const stag_lattice *lat, const void *canonical, void *vec, stag_prec prec, void *stream) {
    STAG_TRY(check_lattice(lat, false));
    if (!canonical || !vec) return invalid("null vector");
    if (!prec_ok(prec)) return invalid("vector precision must be STAG_F64 or STAG_F32");
    if (ranges_overlap({canonical, (size_t)vec_bytes(lat, true)}, {vec, (size_t)vec_bytes(lat, prec == STAG_F64)}))
        return invalid("canonical and library vectors must not overlap");
    STAG_HIP(launch_pack_vec(lat->g, canonical, vec, prec == STAG_F64, static_cast<hipStream_t>(stream)));
    return STAG_OK;
}

stag_status stag_vec_unpack(const stag_lattice *lat, const void *vec, void *canonical, stag_prec prec, void *stream) {
    STAG_TRY(check_lattice(lat, false));
    if (!canonical || !vec) return invalid("null vector");
    if (!prec_ok(prec)) return invalid("vector precision must be STAG_F64 or STAG_F32");
    if (ranges_overlap({canonical, (size_t)vec_bytes(lat, true)}, {vec, (size_t)vec_bytes(lat, prec == STAG_F64)}))
        return invalid("canonical and library vectors must not overlap");
    STAG_HIP(launch_unpack_vec(lat->g, vec, canonical, prec == STAG_F64, static_cast<hipStream_t>(stream)));
    return STAG_OK;
}

stag_status stag_dslash_eo(const stag_lattice *lat, int out_parity, const void *in, void *out, stag_prec prec,
                           void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!in || !out) return invalid("null vector");
    if (out_parity != 0 && out_parity != 1) return invalid("out_parity must be 0 or 1");
    if (!prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    const bool dbl = prec == STAG_F64;
    if (ranges_overlap({in, (size_t)vec_bytes(lat, dbl)}, {out, (size_t)vec_bytes(lat, dbl)}))
        return invalid("in and out must not overlap");
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.out_parity = out_parity;
    a.links = dbl ? lat->links64 : lat->links32;
    a.link_cache = lat->link_cache;
    a.in = in;
    a.out = out;
    STAG_HIP(launch_dslash(dbl, lat->nrow, DS_PLAIN, a, static_cast<hipStream_t>(stream)));
    return STAG_OK;
}

stag_status stag_normal_op(stag_lattice *lat, double mass, double shift, const void *in, void *out, stag_prec prec,
                           void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!in || !out) return invalid("null vector");
    if (!(mass > 0) || !std::isfinite(mass)) return invalid("mass must be > 0");
    if (!(shift >= 0) || !std::isfinite(shift)) return invalid("shift must be >= 0");
    if (!prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    const bool dbl = prec == STAG_F64;
    if (ranges_overlap({in, (size_t)vec_bytes(lat, dbl)}, {out, (size_t)vec_bytes(lat, dbl)}))
        return invalid("in and out must not overlap");
    void *t = nullptr;
    STAG_TRY(ws_get(lat, WS_E, (size_t)vec_bytes(lat, dbl), &t));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.links = dbl ? lat->links64 : lat->links32;
    a.link_cache = lat->link_cache;
    a.out_parity = 1;
    a.in = in;
    a.out = t;
    STAG_HIP(launch_dslash(dbl, lat->nrow, DS_PLAIN, a, s));
    a.out_parity = 0;
    a.in = t;
    a.out = out;
    a.aux = in;
    a.c = mass * mass + shift;
    STAG_HIP(launch_dslash(dbl, lat->nrow, DS_NORMAL, a, s));
    return STAG_OK;
}

static stag_status check_solver_args(double mass, double tol, int max_iter, stag_prec prec) {
    if (!(mass > 0) || !std::isfinite(mass)) return invalid("mass must be > 0");
    if (!(tol > 0) || !std::isfinite(tol)) return invalid("tol must be > 0");
    if (max_iter < 1) return invalid("max_iter must be >= 1");
    if (prec != STAG_F64 && prec != STAG_F32 && prec != STAG_MIXED) return invalid("unknown precision");
    return STAG_OK;
}

stag_status stag_multishift_cg(stag_lattice *lat, double mass, const double *shifts, int n_shifts, const void *src,
                               void *const *sols, double tol, int max_iter, stag_prec prec, stag_cg_stats *stats,
                               void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_solver_args(mass, tol, max_iter, prec));
        if (!shifts || !src || !sols) return invalid("null argument");
        if (n_shifts < 1 || n_shifts > STAG_MAX_SHIFTS) return invalid("n_shifts must be in [1, 64]");
        const size_t vb = (size_t)vec_bytes(lat, true);
        std::vector<ByteRange> outs(n_shifts);
        for (int i = 0; i < n_shifts; ++i) {
            if (!(shifts[i] >= 0) || !std::isfinite(shifts[i])) return invalid("shifts must be >= 0 and finite");
            if (!sols[i]) return invalid("null solution pointer");
            outs[i] = {sols[i], vb};
        }
        const ByteRange in{src, vb};
        if (!outputs_disjoint(outs.data(), n_shifts, &in, 1))
            return invalid("the solutions must not overlap each other or the source");
        return multishift_cg(lat, mass, shifts, n_shifts, src, sols, tol, max_iter, prec, stats,
                             static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_rational_apply(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                const double *shifts, int n, const void *src, void *out, double tol, int max_iter,
                                double *dot, stag_cg_stats *stats, void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_solver_args(mass, tol, max_iter, STAG_F64));
        if (!alphas || !shifts || !src || !out) return invalid("null argument");
        if (ranges_overlap({out, (size_t)vec_bytes(lat, true)}, {src, (size_t)vec_bytes(lat, true)}))
            return invalid("out overlaps the source");
        if (n < 1 || n > STAG_MAX_SHIFTS) return invalid("n must be in [1, 64]");
        if (!std::isfinite(alpha0)) return invalid("alpha0 must be finite");
        for (int i = 0; i < n; ++i) {
            if (!(shifts[i] >= 0) || !std::isfinite(shifts[i])) return invalid("shifts must be >= 0 and finite");
            if (!std::isfinite(alphas[i])) return invalid("alphas must be finite");
        }
        return rational_apply(lat, mass, alpha0, alphas, shifts, n, src, out, tol, max_iter, dot, stats,
                              static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_rational_apply_multi(stag_lattice *lat, double mass, double alpha0, const double *alphas,
                                      const double *shifts, int n, const void *const *srcs, void *const *outs,
                                      int n_rhs, double tol, int max_iter, double *dots, stag_cg_stats *stats,
                                      void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_solver_args(mass, tol, max_iter, STAG_F64));
        if (!alphas || !shifts || !srcs || !outs) return invalid("null argument");
        if (n < 1 || n > STAG_MAX_SHIFTS) return invalid("n must be in [1, 64]");
        if (n_rhs < 1 || n_rhs > 64) return invalid("n_rhs must be in [1, 64]");
        if (!std::isfinite(alpha0)) return invalid("alpha0 must be finite");
        for (int i = 0; i < n; ++i) {
            if (!(shifts[i] >= 0) || !std::isfinite(shifts[i])) return invalid("shifts must be >= 0 and finite");
            if (!std::isfinite(alphas[i])) return invalid("alphas must be finite");
        }
        const size_t vb = (size_t)vec_bytes(lat, true);
        std::vector<ByteRange> ro(n_rhs), ri(n_rhs);
        for (int k = 0; k < n_rhs; ++k) {
            if (!srcs[k] || !outs[k]) return invalid("null field pointer");
            ro[k] = {outs[k], vb};
            ri[k] = {srcs[k], vb};
        }
        if (!outputs_disjoint(ro.data(), n_rhs, ri.data(), n_rhs))
            return invalid("an output overlaps a source or another output");
        return rational_apply_multi(lat, mass, alpha0, alphas, shifts, n, srcs, outs, n_rhs, tol, max_iter, dots,
                                    stats, static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_fermion_force(stag_lattice *lat, int n, const double *alphas, const void *const *x, void *force,
                               void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        if (n < 0 || n > STAG_MAX_SHIFTS) return invalid("n must be in [0, 64]");
        if (!force || (n > 0 && (!alphas || !x))) return invalid("null argument");
        const ByteRange fr{force, (size_t)(4 * 9 * 16) * (size_t)lat->V};
        std::vector<ByteRange> xr(n > 0 ? n : 1);
        for (int i = 0; i < n; ++i) {
            if (!x[i]) return invalid("null solution pointer");
            if (!std::isfinite(alphas[i])) return invalid("alphas must be finite");
            xr[i] = {x[i], (size_t)vec_bytes(lat, true)};
        }
        if (!outputs_disjoint(&fr, 1, xr.data(), n)) return invalid("force overlaps a solution");
        return fermion_force(lat, n, alphas, x, force, static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

// ---------------------------------------------------------------- RHMC trajectory
static size_t force_bytes(const stag_lattice *lat) { return (size_t)(4 * 9 * 16) * (size_t)lat->V; }
static size_t mom_bytes(const stag_lattice *lat) { return (size_t)(4 * 8 * 8) * (size_t)lat->V; }
static bool md_prec_ok(stag_prec p) { return p == STAG_F64 || p == STAG_F32; }

stag_status stag_links_get(const stag_lattice *lat, void *links, void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!links) return invalid("null links");
    STAG_HIP(launch_unpack_links(lat->g, lat->links64, lat->nrow, links, static_cast<hipStream_t>(stream)));
    return STAG_OK;
}

stag_status stag_gauge_force(stag_lattice *lat, double beta, void *force, stag_prec prec, void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!force) return invalid("null force");
    if (!(beta >= 0) || !std::isfinite(beta)) return invalid("beta must be >= 0 and finite");
    if (!md_prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    return gauge_force_out(lat, beta, force, prec == STAG_F64, static_cast<hipStream_t>(stream));
}

stag_status stag_gauge_action(stag_lattice *lat, double beta, double *action, void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        if (!action) return invalid("null action");
        if (!(beta >= 0) || !std::isfinite(beta)) return invalid("beta must be >= 0 and finite");
        return gauge_action(lat, beta, action, static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_gauge_kick(stag_lattice *lat, double beta, double h, double *mom, stag_prec prec, void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!mom) return invalid("null momenta");
    if (!(beta >= 0) || !std::isfinite(beta) || !std::isfinite(h)) return invalid("beta >= 0 and h must be finite");
    if (!md_prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    return mom_step(lat, mom, 0, beta, nullptr, h, prec == STAG_F64, static_cast<hipStream_t>(stream));
}

stag_status stag_force_kick(stag_lattice *lat, const void *force, double h, double *mom, stag_prec prec,
                            void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!mom || !force) return invalid("null argument");
    if (!std::isfinite(h)) return invalid("h must be finite");
    if (!md_prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    if (ranges_overlap({force, force_bytes(lat)}, {mom, mom_bytes(lat)})) return invalid("force overlaps the momenta");
    return mom_step(lat, mom, 1, 0.0, force, h, prec == STAG_F64, static_cast<hipStream_t>(stream));
}

stag_status stag_link_update(stag_lattice *lat, const double *mom, double h, stag_prec prec, void *stream) {
    STAG_TRY(check_lattice(lat, true));
    if (!mom) return invalid("null momenta");
    if (!std::isfinite(h)) return invalid("h must be finite");
    if (!md_prec_ok(prec)) return invalid("precision must be STAG_F64 or STAG_F32");
    if (lat->nrow != kHiLo + 2 && lat->nrow != kHiLo + 3)
        return invalid("link updates need the links stored as STAG_LINK18_PAIRS or STAG_LINK12_PAIRS");
    return mom_step(lat, const_cast<double *>(mom), 2, 0.0, nullptr, h, prec == STAG_F64,
                    static_cast<hipStream_t>(stream));
}

static stag_status check_fields(const stag_lattice *lat, const double *mom, int n_pf, const void *const *f) {
    if (!mom) return invalid("null momenta");
    if (n_pf > 0 && !f) return invalid("null field array");
    const size_t vb = (size_t)vec_bytes(lat, true);
    std::vector<ByteRange> in(n_pf > 0 ? n_pf : 1);
    for (int k = 0; k < n_pf; ++k) {
        if (!f[k]) return invalid("null pseudo-fermion field");
        in[k] = {f[k], vb};
    }
    const ByteRange out{mom, mom_bytes(lat)};
    if (!outputs_disjoint(&out, 1, in.data(), n_pf)) return invalid("the momenta overlap a pseudo-fermion field");
    return STAG_OK;
}

stag_status stag_md_integrate(stag_lattice *lat, const stag_rhmc_params *prm, double *mom, int n_pf,
                              const void *const *phis, stag_rhmc_info *info, void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_md_params(lat, prm, n_pf, false));
        STAG_TRY(check_fields(lat, mom, n_pf, phis));
        stag_rhmc_info local;
        std::memset(&local, 0, sizeof(local));
        const stag_status rc = md_integrate(lat, prm, mom, n_pf, phis, &local, static_cast<hipStream_t>(stream));
        if (info) *info = local;
        return rc;
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_rhmc_trajectory(stag_lattice *lat, const stag_rhmc_params *prm, double *mom, int n_pf,
                                 const void *const *xis, double u, stag_rhmc_info *info, void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_md_params(lat, prm, n_pf, true));
        STAG_TRY(check_fields(lat, mom, n_pf, xis));
        if (!(u < 1.0) || std::isnan(u)) return invalid("u must be < 1 (u < 0 accepts unconditionally)");
        stag_rhmc_info local;
        std::memset(&local, 0, sizeof(local));
        const stag_status rc = rhmc_trajectory(lat, prm, mom, n_pf, xis, u, &local, static_cast<hipStream_t>(stream));
        if (info) *info = local;
        return rc;
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_zolotarev(int power, double lo, double hi, int n, double *alpha0, double *alphas, double *shifts,
                           double *max_rel_err) {
    if (power != -1 && power != 1) return invalid("power must be -1 (x^-1/2) or +1 (x^1/2)");
    if (!(lo > 0) || !(hi > lo) || !std::isfinite(hi)) return invalid("need 0 < lo < hi");
    if (n < 1 || n > STAG_MAX_SHIFTS) return invalid("n must be in [1, 64]");
    if (!alpha0 || !alphas || !shifts) return invalid("null argument");
    try {
        return zolotarev(power, lo, hi, n, alpha0, alphas, shifts, max_rel_err);
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_rational_power(double power, double lo, double hi, int n, double *alpha0, double *alphas,
                                double *shifts, double *max_rel_err) {
    if (!(power > -1.0 && power < 1.0) || power == 0.0) return invalid("power must lie in (-1, 0) or (0, 1)");
    if (!(lo > 0) || !(hi > lo) || !std::isfinite(hi)) return invalid("need 0 < lo < hi");
    const int nmax = (power == 0.5 || power == -0.5) ? STAG_MAX_SHIFTS : 24;
    if (n < 1 || n > nmax) return invalid("n must be in [1, 64] for powers +-1/2 and in [1, 24] otherwise");
    if (!alpha0 || !alphas || !shifts) return invalid("null argument");
    try {
        return rational_power(power, lo, hi, n, alpha0, alphas, shifts, max_rel_err);
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol, int max_iter,
                    stag_prec prec, stag_cg_stats *stats, void *stream) {
    try {
        STAG_TRY(check_lattice(lat, true));
        STAG_TRY(check_solver_args(mass, tol, max_iter, prec));
        if (prec == STAG_F32) return invalid("stag_cg takes STAG_F64 or STAG_MIXED");
        if (!(shift >= 0) || !std::isfinite(shift)) return invalid("shift must be >= 0");
        if (!src || !x) return invalid("null vector");
        if (ranges_overlap({src, (size_t)vec_bytes(lat, true)}, {x, (size_t)vec_bytes(lat, true)}))
            return invalid("x overlaps the source");
        return single_cg(lat, mass, shift, src, x, tol, max_iter, prec, stats, static_cast<hipStream_t>(stream));
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_multishift_cg_batched(const stag_system *systems, int n_systems, double tol, int max_iter,
                                       stag_prec prec, int flags, stag_cg_stats *stats, void *stream) {
    try {
        if (!systems) return invalid("null systems");
        if (n_systems < 1 || n_systems > 64) return invalid("n_systems must be in [1, 64]");
        if (!(tol > 0) || !std::isfinite(tol)) return invalid("tol must be > 0");
        if (max_iter < 1) return invalid("max_iter must be >= 1");
        if (prec != STAG_F64 && prec != STAG_F32 && prec != STAG_MIXED) return invalid("unknown precision");
        std::vector<BSpec> spec(n_systems);
        std::vector<ByteRange> b_outs, b_ins;
        int device = -1;
        for (int k = 0; k < n_systems; ++k) {
            const stag_system &y = systems[k];
            STAG_TRY(check_lattice(y.lat, true));
            if (device < 0) device = y.lat->device;
            if (y.lat->device != device) return invalid("all lattices of a batch must live on one device");
            if (y.lat->nrow != systems[0].lat->nrow) return invalid("all lattices of a batch must use one link format");
            if (!(y.mass > 0) || !std::isfinite(y.mass)) return invalid("mass must be > 0");
            if (y.n_shifts < 1 || y.n_shifts > STAG_MAX_SHIFTS) return invalid("n_shifts must be in [1, 64]");
            if (!y.shifts || !y.src || !y.sols) return invalid("null argument in a system");
            const size_t vb = (size_t)vec_bytes(y.lat, true);
            for (int i = 0; i < y.n_shifts; ++i) {
                if (!(y.shifts[i] >= 0) || !std::isfinite(y.shifts[i])) return invalid("shifts must be >= 0 and finite");
                if (!y.sols[i]) return invalid("null solution pointer");
                b_outs.push_back({y.sols[i], vb});
            }
            b_ins.push_back({y.src, vb});
            spec[k] = {y.lat, y.mass, y.n_shifts, y.shifts, y.src, y.sols, false};
        }
        if (!outputs_disjoint(b_outs.data(), (int)b_outs.size(), b_ins.data(), (int)b_ins.size()))
            return invalid("the solutions of a batch must not overlap each other or any source");
        BOptions opt;
        opt.tol = tol;
        opt.max_iter = max_iter;
        opt.dbl = prec == STAG_F64;
        opt.reliable_every = prec == STAG_MIXED ? kDefer : 0;
        opt.use_graph = !(flags & STAG_BATCH_NO_GRAPH);
        opt.merge_lattices = !(flags & STAG_BATCH_PER_LATTICE);
        opt.force_rpt = (flags >> 4) & 0xF;
        opt.force_block = ((flags >> 8) & 0xF) * 64;
        if (opt.force_rpt || opt.force_block) {
            if (!(opt.force_rpt == 1 || opt.force_rpt == 2 || opt.force_rpt == 4 || opt.force_rpt == 8) ||
                !(opt.force_block == 64 || opt.force_block == 128 || opt.force_block == 256))
                return invalid("forced launch shape must be rpt in {1,2,4,8} and block in {64,128,256}");
        }
        std::vector<stag_cg_stats> st(n_systems);
        const stag_status rc = batched_solve(spec.data(), n_systems, opt, prec == STAG_MIXED, st.data(),
                                             static_cast<hipStream_t>(stream));
        if (stats && rc >= 0)
            for (int k = 0; k < n_systems; ++k) stats[k] = st[k];
        return rc;
    } catch (...) {
        set_error("host allocation failed");
        return STAG_ENOMEM;
    }
}

stag_status stag_batch_last_config(int *block, int *rpt) {
    if (!block || !rpt) return invalid("null argument");
    const BDslashCfg c = last_batch_cfg();
    *block = c.block;
    *rpt = c.rpt;
    return STAG_OK;
}

const char *stag_status_string(stag_status s) {
    switch (s) {
        case STAG_OK: return "ok";
        case STAG_ENOCONV: return "not converged within max_iter";
        case STAG_EBREAKDOWN: return "breakdown: non-positive or non-finite curvature";
        case STAG_EINVAL: return "invalid argument";
        case STAG_ENOMEM: return "out of memory";
        case STAG_EHIP: return "HIP runtime error";
        default: break;
    }
    return "unknown status";
}

const char *stag_last_error(void) { return stag::last_error(); }

}  // extern "C"
