// Flexible CG preconditioned by the learned network, for (M + shift) x = b.
//
// Flexible CG (Notay; Golub and Ye) differs from CG in the direction update:
// with a preconditioner that varies from call to call (here: a network
// evaluated in reduced precision), beta is the Polak-Ribiere form
//   beta_k = <z_{k+1}, r_{k+1} - r_k> / <z_k, r_k>,
// which keeps the directions conjugate to first order.  Vectors, the
// operator and every reduction are double precision; only the network runs
// in single precision / BF16, on a single precision copy of the residual.
//
// As in the shifted CG driver, all scalars live on the device.  The host
// enqueues chunks of iterations and reads a 4-byte state word one chunk
// behind; kernels enqueued after the state left "running" return at once.
// When the iterated residual reaches tol ||b|| the host recomputes the
// residual b - (M + shift) x in double precision (the final check) and either
// stops or restarts the iteration from the true residual.  A non-positive
// or non-finite <r, P r> or <p, A p>, or 50 iterations without a new
// smallest residual, hand the solve to plain double precision CG from the
// current x.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "common.h"
#include "internal.h"
#include "net.h"
#include "solver.h"

namespace stag {

stag_status single_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol,
                      int max_iter, stag_prec prec, stag_cg_stats *stats, hipStream_t s);

enum FcgRun { FCG_RUNNING = 0, FCG_CONVERGED = 1, FCG_FALLBACK = 2, FCG_MAXITER = 3 };

struct FcgState {
    double rz;          // <r, z> of the current direction
    double alpha, beta;
    double rr;          // iterated |r|^2
    double bb;          // |b|^2
    double tol2bb;      // tol^2 |b|^2
    double best;        // smallest iterated |r|^2 so far
    double resid_true2; // |b - A x|^2 of the last check
    double rz_snap;     // <r, z> of the current direction, kept for the fused beta step
    int since_best;
    int iter;
    int max_iter;
    int run;            // FcgRun
};

constexpr int kFcgBlock = 256;
constexpr int kFcgStall = 50;

__device__ __forceinline__ double fixed_sum(const double *part, int n, double *red) {
    return block_sum(part_sum<kFcgBlock>(part, n), red);
}

// |b|^2 and the stopping threshold
__global__ void __launch_bounds__(kFcgBlock) k_fcg_init(FcgState *st, const double *part, int n, double tol,
                                                     int max_iter) {
    __shared__ double red[kFcgBlock / kWave];
    const double bb = fixed_sum(part, n, red);
    if (threadIdx.x == 0) {
        st->bb = bb;
        st->tol2bb = tol * tol * bb;
        st->iter = 0;
        st->max_iter = max_iter;
        st->run = FCG_RUNNING;
    }
}

// after r = b - A x: |r|^2 (kind 0: start or restart; kind 1: check only)
__global__ void __launch_bounds__(kFcgBlock) k_fcg_resid(FcgState *st, const double *part, int n, int kind) {
    __shared__ double red[kFcgBlock / kWave];
    const double rr = fixed_sum(part, n, red);
    if (threadIdx.x != 0) return;
    st->resid_true2 = rr;
    if (kind == 0) {
        st->rr = rr;
        st->best = rr;
        st->since_best = 0;
        st->run = rr <= st->tol2bb ? FCG_CONVERGED : FCG_RUNNING;
    }
}

// <r, z> of the first direction (p = z)
__global__ void __launch_bounds__(kFcgBlock) k_fcg_start(FcgState *st, const double *part_b, int n) {
    __shared__ double red[kFcgBlock / kWave];
    if (st->run != FCG_RUNNING) return;
    const double rz = fixed_sum(part_b, n, red);
    if (threadIdx.x == 0) {
        st->rz = rz;
        if (!(rz > 0.0) || !isfinite(rz)) st->run = FCG_FALLBACK;
    }
}

// |r|^2, convergence, stagnation; beta (Polak-Ribiere) and the new <r, z>,
// from the reduced sums (thread 0 of one workgroup).
// r_{k+1} - r_k = -alpha_k q_k, so <z_{k+1}, r_{k+1} - r_k> = -alpha_k <z_{k+1}, q_k>.
__device__ __forceinline__ void fcg_beta_step(FcgState *st, double rr, double za, double rz) {
    st->iter += 1;
    st->rr = rr;
    if (!isfinite(rr)) {
        st->run = FCG_FALLBACK;
        return;
    }
    if (rr <= st->tol2bb) {
        st->run = FCG_CONVERGED;
        return;
    }
    if (rr < st->best) {
        st->best = rr;
        st->since_best = 0;
    } else if (++st->since_best >= kFcgStall) {
        st->run = FCG_FALLBACK;
        return;
    }
    if (st->iter >= st->max_iter) {
        st->run = FCG_MAXITER;
        return;
    }
    if (!(rz > 0.0) || !isfinite(rz) || !isfinite(za)) {
        st->run = FCG_FALLBACK;
        return;
    }
    st->beta = za / st->rz;
    st->rz = rz;
}

// alpha with the step, beta with the direction: every workgroup reduces the
// previous kernel's partials itself, in one fixed order (so all workgroups
// hold the same scalars, and every run the same bits); workgroup 0 also
// advances the state.  A workgroup that runs after workgroup 0 ended the
// iteration (converged, fall-back, limit) may still write p: the host then
// restarts from p = z or leaves p unused.
__global__ void __launch_bounds__(kFcgBlock) k_fcg_step_fused(FcgState *st, const double *part_pq, int n_pq,
                                                           double2 *x, double2 *r, float2 *r32, const double2 *p,
                                                           const double2 *q, int64_t n, double *part) {
    __shared__ double red[kFcgBlock / kWave];
    if (st->run != FCG_RUNNING) return;
    const double pq = fixed_sum(part_pq, n_pq, red);
    const bool bad = !(pq > 0.0) || !isfinite(pq);
    const double alpha = st->rz / pq;   // rz is not written by this kernel
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rz_snap = st->rz;
        if (bad) st->run = FCG_FALLBACK;
        else st->alpha = alpha;
    }
    if (bad) return;
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const double2 pv = p[j], qv = q[j];
        double2 xv = x[j], rv = r[j];
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        rv.x -= alpha * qv.x;
        rv.y -= alpha * qv.y;
        x[j] = xv;
        r[j] = rv;
        r32[j] = make_float2(float(rv.x), float(rv.y));
        acc += rv.x * rv.x + rv.y * rv.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kFcgBlock) k_fcg_dir_fused(FcgState *st, const double *part_rr, int n_rr,
                                                          const double *part_a, const double *part_b, int n_ab,
                                                          double2 *p, const float2 *z32, int64_t n) {
    __shared__ double red[kFcgBlock / kWave];
    if (st->run != FCG_RUNNING) return;
    const double rr = fixed_sum(part_rr, n_rr, red);
    const double za = -st->alpha * fixed_sum(part_a, n_ab, red);
    const double rz = fixed_sum(part_b, n_ab, red);
    const double beta = za / st->rz_snap;   // workgroup 0 rewrites rz below, not rz_snap
    if (blockIdx.x == 0 && threadIdx.x == 0) fcg_beta_step(st, rr, za, rz);
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const float2 zv = z32[j];
        double2 pv = p[j];
        pv.x = double(zv.x) + beta * pv.x;
        pv.y = double(zv.y) + beta * pv.y;
        p[j] = pv;
    }
}

// r32 = (float) r (start and restart)
__global__ void __launch_bounds__(kFcgBlock) k_fcg_demote(const FcgState *st, const double2 *r, float2 *r32,
                                                       int64_t n) {
    if (st->run != FCG_RUNNING) return;
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock)
        r32[j] = make_float2(float(r[j].x), float(r[j].y));
}

// z = P r arrives in single precision: partials of <z, q> and <r, z> (q = A p
// of the step that produced r); p = z when `first`
__global__ void __launch_bounds__(kFcgBlock) k_fcg_z(const FcgState *st, const float2 *z32, double2 *p, int first,
                                                  const double2 *r, const double2 *q, int64_t n, double *part_a,
                                                  double *part_b) {
    __shared__ double red[kFcgBlock / kWave];
    if (st->run != FCG_RUNNING) return;
    double a = 0.0, b = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const double2 zv = make_double2(double(z32[j].x), double(z32[j].y));
        if (first) {
            p[j] = zv;
        } else {
            const double2 qv = q[j];
            a += zv.x * qv.x + zv.y * qv.y;
        }
        const double2 rv = r[j];
        b += zv.x * rv.x + zv.y * rv.y;
    }
    const double sa = block_sum(a, red);
    const double sb = block_sum(b, red);
    if (threadIdx.x == 0) {
        part_a[blockIdx.x] = sa;
        part_b[blockIdx.x] = sb;
    }
}

// the run word and the iteration count, for the host
__global__ void k_fcg_report(const FcgState *st, int *out) {
    if (threadIdx.x == 0) {
        out[0] = st->run;
        out[1] = st->iter;
    }
}

__global__ void k_fcg_set_run(FcgState *st, int run) {
    if (threadIdx.x == 0) st->run = run;
}

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

static constexpr int kFcgChunk = 8;   // iterations enqueued between reads of the run word

stag_status fcg_solve(stag_lattice *lat, double mass, double shift, const void *src, void *sol, stag_net *net,
                      int mode, double tol, int max_iter, stag_cg_stats *stats, hipStream_t s) {
    TraceRange tr("flexible CG");
    const auto t0 = std::chrono::steady_clock::now();
    stag_cg_stats st;
    std::memset(&st, 0, sizeof(st));
    if (!net) {   // plain double precision CG
        STAG_TRY(single_cg(lat, mass, shift, src, sol, tol, max_iter, STAG_F64, &st, s));
        if (stats) *stats = st;
        return STAG_OK;
    }
    STAG_TRY(net_prepare_links(lat, mode, s));
    const int64_t ne = 3 * lat->Vh;
    const size_t vb = sizeof(double2) * ne;
    const int ds_grid = dslash_grid(lat->g, kDslashBlock);
    const int grid = (int)std::min<int64_t>((ne + kFcgBlock - 1) / kFcgBlock, 2048);
    const int nparts = std::max(ds_grid, grid);
    void *W = nullptr;
    const size_t bytes = 4 * al(vb) + 2 * al(sizeof(float2) * ne) + 4 * al(sizeof(double) * nparts) +
                         al(sizeof(FcgState)) + 256;
    STAG_TRY(ws_get(lat, WS_E2, bytes, &W));
    char *cur = static_cast<char *>(W);
    auto take = [&](size_t n) {
        char *q = cur;
        cur += al(n);
        return q;
    };
    double2 *x = static_cast<double2 *>(sol), *b = static_cast<double2 *>(const_cast<void *>(src));
    double2 *r = reinterpret_cast<double2 *>(take(vb)), *p = reinterpret_cast<double2 *>(take(vb));
    double2 *q = reinterpret_cast<double2 *>(take(vb)), *t = reinterpret_cast<double2 *>(take(vb));
    float2 *r32 = reinterpret_cast<float2 *>(take(sizeof(float2) * ne));
    float2 *z32 = reinterpret_cast<float2 *>(take(sizeof(float2) * ne));
    double *pq = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *prr = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *pa = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *pb = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    FcgState *dst = reinterpret_cast<FcgState *>(take(sizeof(FcgState)));
    int *dreport = reinterpret_cast<int *>(take(256));
    NetBufs nb;
    STAG_TRY(net_work(net, lat, 1, &nb));
    const int *skip = &dst->run;
    const double c = mass * mass + shift;
    DslashArgs d;
    std::memset(&d, 0, sizeof(d));
    d.g = lat->g;
    d.links = lat->links64;
    d.skip = skip;

    // r = b - (M + shift) x, partial |r|^2 into pq
    auto residual = [&](bool gated) -> hipError_t {
        DslashArgs e = d;
        if (!gated) e.skip = nullptr;
        e.out_parity = 1;
        e.in = x;
        e.out = t;
        hipError_t err = launch_dslash(true, lat->nrow, DS_PLAIN, e, s);
        if (err != hipSuccess) return err;
        e.out_parity = 0;
        e.in = t;
        e.out = r;
        e.aux = x;
        e.rhs = b;
        e.c = c;
        e.partial = pq;
        return launch_dslash(true, lat->nrow, DS_RESID, e, s);
    };
    // z = P(r) from r (double), p = z, <r, z>
    auto start_direction = [&]() -> hipError_t {
        hipLaunchKernelGGL(k_fcg_demote, dim3(grid), dim3(kFcgBlock), 0, s, (const FcgState *)dst, (const double2 *)r,
                           r32, ne);
        NetArgs a = net_args(net, lat, r32, z32, nb, false);
        a.skip = skip;
        hipError_t err = net_launch_forward(a, 1, mode, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_fcg_z, dim3(grid), dim3(kFcgBlock), 0, s, (const FcgState *)dst, (const float2 *)z32, p, 1,
                           (const double2 *)r, (const double2 *)q, ne, pa, pb);
        hipLaunchKernelGGL(k_fcg_start, dim3(1), dim3(kFcgBlock), 0, s, dst, (const double *)pb, grid);
        return hipGetLastError();
    };
    auto iteration = [&]() -> hipError_t {
        DslashArgs e = d;
        e.out_parity = 1;
        e.in = p;
        e.out = t;
        hipError_t err = launch_dslash(true, lat->nrow, DS_PLAIN, e, s);
        if (err != hipSuccess) return err;
        e.out_parity = 0;
        e.in = t;
        e.out = q;
        e.aux = p;
        e.c = c;
        e.partial = pq;
        err = launch_dslash(true, lat->nrow, DS_NORMAL_DOT, e, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_fcg_step_fused, dim3(grid), dim3(kFcgBlock), 0, s, dst, (const double *)pq, ds_grid, x,
                           r, r32, (const double2 *)p, (const double2 *)q, ne, prr);
        NetArgs a = net_args(net, lat, r32, z32, nb, false);
        a.skip = skip;
        err = net_launch_forward(a, 1, mode, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_fcg_z, dim3(grid), dim3(kFcgBlock), 0, s, (const FcgState *)dst, (const float2 *)z32, p, 0,
                           (const double2 *)r, (const double2 *)q, ne, pa, pb);
        hipLaunchKernelGGL(k_fcg_dir_fused, dim3(grid), dim3(kFcgBlock), 0, s, dst, (const double *)prr, grid,
                           (const double *)pa, (const double *)pb, grid, p, (const float2 *)z32, ne);
        return hipGetLastError();
    };
    int rep[2] = {0, 0};
    auto read_report = [&]() -> stag_status {
        hipLaunchKernelGGL(k_fcg_report, dim3(1), dim3(64), 0, s, (const FcgState *)dst, dreport);
        STAG_HIP(hipGetLastError());
        STAG_HIP(hipMemcpyAsync(rep, dreport, sizeof(rep), hipMemcpyDeviceToHost, s));
        STAG_HIP(hipStreamSynchronize(s));
        return STAG_OK;
    };

    // ---- start: |b|^2, r = b - A x, first direction
    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    STAG_HIP(launch_norm2(true, b, ne, pa, grid, s));
    hipLaunchKernelGGL(k_fcg_init, dim3(1), dim3(kFcgBlock), 0, s, dst, (const double *)pa, grid, tol, max_iter);
    STAG_HIP(hipGetLastError());
    STAG_HIP(residual(false));
    hipLaunchKernelGGL(k_fcg_resid, dim3(1), dim3(kFcgBlock), 0, s, dst, (const double *)pq, ds_grid, 0);
    STAG_HIP(hipGetLastError());
    double bb = 0.0;
    STAG_HIP(hipMemcpyAsync(&bb, &dst->bb, sizeof(double), hipMemcpyDeviceToHost, s));
    STAG_HIP(hipStreamSynchronize(s));
    if (bb == 0.0) {   // b = 0: x = 0
        STAG_HIP(hipMemsetAsync(x, 0, vb, s));
        STAG_HIP(hipStreamSynchronize(s));
        if (stats) *stats = st;
        return STAG_OK;
    }
    STAG_HIP(start_direction());

    hipEvent_t ev[2];
    STAG_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    STAG_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    volatile int *flags = lat->host_flags;
    bool converged = false, fallback = false;
    stag_status rc = STAG_OK;
    int restarts = 0;
    for (;;) {
        // chunks until the run word leaves "running"
        flags[0] = flags[1] = 0;
        int run = FCG_RUNNING;
        for (int chunk = 0;; ++chunk) {
            hipError_t e = hipSuccess;
            for (int k = 0; k < kFcgChunk && e == hipSuccess; ++k) e = iteration();
            const int slot = chunk & 1;
            if (e == hipSuccess) e = hipMemcpyAsync(const_cast<int *>(flags + slot), &dst->run, sizeof(int),
                                                    hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipEventRecord(ev[slot], s);
            if (e == hipSuccess && chunk > 0) {
                e = hipEventSynchronize(ev[slot ^ 1]);
                if (e == hipSuccess && flags[slot ^ 1] != FCG_RUNNING) break;
            }
            if (e != hipSuccess) {
                set_error(std::string("flexible CG iteration failed: ") + hipGetErrorString(e));
                rc = STAG_EHIP;
                break;
            }
        }
        if (rc != STAG_OK) break;
        if (read_report() != STAG_OK) {
            rc = STAG_EHIP;
            break;
        }
        run = rep[0];
        if (run == FCG_CONVERGED) {
            // the final check: the double precision residual of x
            if (residual(false) != hipSuccess) {
                rc = STAG_EHIP;
                break;
            }
            hipLaunchKernelGGL(k_fcg_resid, dim3(1), dim3(kFcgBlock), 0, s, dst, (const double *)pq, ds_grid, 0);
            if (read_report() != STAG_OK) {
                rc = STAG_EHIP;
                break;
            }
            if (rep[0] == FCG_CONVERGED) {
                converged = true;
                break;
            }
            if (++restarts > 20 || rep[1] >= max_iter) break;
            if (start_direction() != hipSuccess) {   // restart from the true residual
                rc = STAG_EHIP;
                break;
            }
            continue;
        }
        if (run == FCG_FALLBACK) fallback = true;
        break;   // fallback or max_iter
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc != STAG_OK) return rc;
    st.iters = rep[1];
    double rt2 = 0.0;
    if (fallback && st.iters < max_iter) {
        stag_cg_stats cs;
        stag_status r2 = single_cg(lat, mass, shift, src, sol, tol, max_iter - st.iters, STAG_F64, &cs, s);
        if (r2 < 0) return r2;
        st.iters += cs.iters;
        st.fallback_used = 1;
        st.resid_true[0] = cs.resid_true[0];
        converged = r2 == STAG_OK;
    } else {
        if (!converged) {   // max_iter (or a fallback with no iterations left): report the true residual
            STAG_HIP(residual(false));
            hipLaunchKernelGGL(k_fcg_resid, dim3(1), dim3(kFcgBlock), 0, s, dst, (const double *)pq, ds_grid, 1);
            STAG_HIP(hipGetLastError());
        }
        STAG_HIP(hipMemcpyAsync(&rt2, &dst->resid_true2, sizeof(double), hipMemcpyDeviceToHost, s));
        STAG_HIP(hipStreamSynchronize(s));
        st.resid_true[0] = std::sqrt(rt2 / bb);
        st.fallback_used = fallback ? 1 : 0;
    }
    st.iters_shift[0] = st.iters;
    st.resid_unrefined[0] = st.resid_true[0];
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    if (!converged) {
        set_error("flexible CG did not reach tol within max_iter");
        return STAG_ENOCONV;
    }
    return STAG_OK;
}

}  // namespace stag
