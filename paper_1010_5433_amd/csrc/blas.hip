// Solver kernels: FP64 reductions, the shifted-CG scalar recursion on the
// device, and the fused vector updates.
//
// Scalar recursion (Jegerlehner's multi-shift CG, the Krylov solver for
// shifted systems cited in Section 6), base shift sigma_0 = min sigma_i,
// s_i = sigma_i - sigma_0, alpha_{-1} = 1, beta_{-1} = 0, zeta^{-1} = zeta^0 = 1:
//   alpha_k = rho_k / Re<p, A p>
//   zeta_i^{k+1} = zeta_i^k zeta_i^{k-1} alpha_{k-1} /
//        [alpha_k beta_{k-1} (zeta_i^{k-1} - zeta_i^k) + zeta_i^{k-1} alpha_{k-1} (1 + s_i alpha_k)]
//   beta_k = rho_{k+1} / rho_k
//   alpha_k^i = alpha_k zeta_i^{k+1} / zeta_i^k,  beta_k^i = beta_k (zeta_i^{k+1} / zeta_i^k)^2
// Shift i freezes once |zeta_i^{k+1}| sqrt(rho_{k+1}) <= tol ||b||.
//
// All sums run in a fixed order (per-block partials, then one wave that
// reads them in a fixed stride and finishes with a DPP reduction), so a
// solve is bitwise reproducible from run to run.
#include <math.h>

#include "common.h"
#include "ms_device.h"
#include "solver.h"

namespace stag {

int blas_grid(int64_t n) {
    int64_t g = (n + kBlasBlock - 1) / kBlasBlock;
    if (g > kMaxBlasGrid) g = kMaxBlasGrid;
    if (g < 1) g = 1;
    return (int)g;
}

// Sum of nparts partials by one wave (blockDim.x == 64), fixed order.
__device__ __forceinline__ double sum_partials(const double *part, int nparts) {
    return wave_sum(part_sum<kWave>(part, nparts));
}

template <typename R> using T2 = typename vtype<R>::t2;

// Vector access of the solver's per-iteration kernels: with NT the loads and
// stores are nontemporal, so that the streamed vectors do not push the link
// blocks that the Dslash keeps in the Infinity Cache out of it.
template <bool NT, typename V> __device__ __forceinline__ V ldv(const V *p) {
    if constexpr (NT) return ld_nt(p);
    else return *p;
}
template <bool NT, typename V> __device__ __forceinline__ void stv(V *p, V v) {
    if constexpr (NT) st_nt(p, v);
    else *p = v;
}

template <typename R> __device__ __forceinline__ double abs2(T2<R> v) {
    return double(v.x) * double(v.x) + double(v.y) * double(v.y);
}

// ---------------------------------------------------------------- vectors

template <typename R>
__global__ void __launch_bounds__(kBlasBlock) k_norm2(const T2<R> *v, int64_t n, double *partial) {
    __shared__ double red[kBlasBlock / kWave];
    double part = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock)
        part += abs2<R>(v[j]);
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename R>
__global__ void __launch_bounds__(kBlasBlock) k_ms_start(const double2 *b, T2<R> *r, ShiftPtrs ptrs, int n_shift,
                                                      int zero_x, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const double2 bj = b[j];
        T2<R> v;
        v.x = R(bj.x);
        v.y = R(bj.y);
        r[j] = v;
        for (int i = 0; i < n_shift; ++i) {
            static_cast<T2<R> *>(ptrs.p[i])[j] = v;
            if (zero_x) {
                T2<R> z;
                z.x = R(0);
                z.y = R(0);
                static_cast<T2<R> *>(ptrs.x[i])[j] = z;
            }
        }
    }
}

// r = rin - alpha A p, and the partial of ||r||^2.
template <typename R>
__global__ void __launch_bounds__(kBlasBlock) k_r_update(const MsState *st, const T2<R> *rin, T2<R> *r,
                                                      const T2<R> *ap, int64_t n, double *partial) {
    if (st->done) return;
    __shared__ double red[kBlasBlock / kWave];
    const R alpha = R(st->alpha);
    double part = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        T2<R> rv = rin[j];
        const T2<R> q = ap[j];
        rv.x -= alpha * q.x;
        rv.y -= alpha * q.y;
        r[j] = rv;
        part += abs2<R>(rv);
    }
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// For every shift updated this iteration: x_i += alpha_i p_i and
// p_i = zeta_i r + beta_i p_i, reading r once for all shifts.  A frozen base
// system still advances its direction p = r + beta p while other shifts run.
template <typename R>
__global__ void __launch_bounds__(kBlasBlock) k_shift_update(const MsState *st, const T2<R> *r, ShiftPtrs ptrs,
                                                          int n_shift, int64_t n) {
    if (!st->upd_valid) return;
    const int base = st->base;
    const int upd_p = st->upd_p;
    const R beta = R(st->beta);
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const T2<R> rv = r[j];
        for (int i = 0; i < n_shift; ++i) {
            T2<R> *pi = static_cast<T2<R> *>(ptrs.p[i]);
            if (st->upd[i]) {
                T2<R> *xi = static_cast<T2<R> *>(ptrs.x[i]);
                const R ai = R(st->a[i]), bi = R(st->b[i]), zi = R(st->zeta[i]);
                const T2<R> pv = pi[j];
                T2<R> xv = xi[j];
                xv.x += ai * pv.x;
                xv.y += ai * pv.y;
                xi[j] = xv;
                T2<R> np;
                np.x = zi * rv.x + bi * pv.x;
                np.y = zi * rv.y + bi * pv.y;
                pi[j] = np;
            } else if (i == base && upd_p) {
                const T2<R> pv = pi[j];
                T2<R> np;
                np.x = rv.x + beta * pv.x;
                np.y = rv.y + beta * pv.y;
                pi[j] = np;
            }
        }
    }
}

// Fused forms (see solver.h).  Every block reduces the partials in the order
// of k_reduce_tail (threads stride kBlasBlock, then block_sum), so alpha and
// beta equal the tail kernel's bit for bit.  A thread loads its first group
// of partials, then the vectors of its first kPrefetch grid-stride trips,
// before it adds anything, so that all those memory latencies overlap.
constexpr int kPrefetch = 4;

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlasBlock) k_r_update_fused(MsState *st, const double *pq_part, int npq,
                                                            const T2<R> *rin, T2<R> *r, const T2<R> *ap, int64_t n,
                                                            double *partial) {
    if (st->done) return;
    __shared__ double red[kBlasBlock / kWave];
    double pre[kPartGroup];
    part_load_group<kBlasBlock>(pq_part, npq, threadIdx.x, pre);
    const int64_t j0 = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlasBlock;
    T2<R> rv[kPrefetch], q[kPrefetch];
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int64_t j = j0 + u * stride;
        if (j < n) {
            rv[u] = ldv<NT>(&rin[j]);
            q[u] = ldv<NT>(&ap[j]);
        }
    }
    double t = part_add_group<kBlasBlock>(0.0, npq, threadIdx.x, pre);
    t = part_sum_from<kBlasBlock>(t, pq_part, npq, threadIdx.x + kPartGroup * kBlasBlock);
    const double pap = block_sum(t, red);
    const bool bad = !(pap > 0.0) || !isfinite(pap);
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) st->rho_snap = st->rho;
        ms_alpha_step(st, pap);   // records a breakdown and ends the solve when bad
    }
    if (bad) return;
    const R alpha = R(st->rho / pap);   // rho is not written by this kernel
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int64_t j = j0 + u * stride;
        if (j < n) {
            rv[u].x -= alpha * q[u].x;
            rv[u].y -= alpha * q[u].y;
            stv<NT>(&r[j], rv[u]);
            part += abs2<R>(rv[u]);
        }
    }
    for (int64_t j = j0 + kPrefetch * stride; j < n; j += stride) {
        T2<R> v = ldv<NT>(&rin[j]);
        const T2<R> w = ldv<NT>(&ap[j]);
        v.x -= alpha * w.x;
        v.y -= alpha * w.y;
        stv<NT>(&r[j], v);
        part += abs2<R>(v);
    }
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlasBlock) k_dir_update_fused(MsState *st, const double *r_part, int nr,
                                                              const T2<R> *r, T2<R> *pd, int64_t n) {
    if (st->done) return;
    __shared__ double red[kBlasBlock / kWave];
    double pre[kPartGroup];
    part_load_group<kBlasBlock>(r_part, nr, threadIdx.x, pre);
    const int64_t j0 = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlasBlock;
    T2<R> rv[kPrefetch], pv[kPrefetch];
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int64_t j = j0 + u * stride;
        if (j < n) {
            rv[u] = ldv<NT>(&r[j]);
            pv[u] = ldv<NT>(&pd[j]);
        }
    }
    double t = part_add_group<kBlasBlock>(0.0, nr, threadIdx.x, pre);
    t = part_sum_from<kBlasBlock>(t, r_part, nr, threadIdx.x + kPartGroup * kBlasBlock);
    const double rho_new = block_sum(t, red);
    const R beta = R(rho_new / st->rho_snap);   // block 0 rewrites rho below, not rho_snap
    if (blockIdx.x == 0) ms_beta_step(st, rho_new);
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
        const int64_t j = j0 + u * stride;
        if (j < n) {
            pv[u].x = rv[u].x + beta * pv[u].x;
            pv[u].y = rv[u].y + beta * pv[u].y;
            stv<NT>(&pd[j], pv[u]);
        }
    }
    for (int64_t j = j0 + kPrefetch * stride; j < n; j += stride) {
        const T2<R> v = ldv<NT>(&r[j]);
        T2<R> w = ldv<NT>(&pd[j]);
        w.x = v.x + beta * w.x;
        w.y = v.y + beta * w.y;
        stv<NT>(&pd[j], w);
    }
}

// Coefficients of a deferred pass (one wave, lane = shift).
__global__ void __launch_bounds__(kWave) k_defer_coef(MsState *st, DeferHist *h) {
    defer_coef_step(st->n, h, st->rat ? st->wgt : nullptr);
}

// The deferred pass: for every shift changed in the block,
// x_i += cx0 p_i + sum_m cx_m r_m and p_i = cp0 p_i + sum_m cp_m r_m,
// the block's residuals read once for all shifts.  RAT: the (weighted)
// increments of all shifts go into one output vector instead.
template <typename R, bool RAT, bool NT>
__global__ void __launch_bounds__(kBlasBlock) k_defer_apply(const MsState *st, const DeferHist *h, const T2<R> *ring,
                                                         int64_t slot, ShiftPtrs ptrs, int n_shift, int64_t n,
                                                         T2<R> *out) {
    const int nv = h->nvalid;
    if (nv == 0) return;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        T2<R> rr[kDefer];
#pragma unroll
        for (int m = 0; m < kDefer; ++m) {
            if (m < nv) {
                rr[m] = ldv<NT>(&ring[m * slot + j]);
            } else {
                rr[m].x = R(0);
                rr[m].y = R(0);
            }
        }
        T2<R> acc;
        if (RAT) acc = ldv<NT>(&out[j]);
        for (int i = 0; i < n_shift; ++i) {
            if (!h->act[i]) continue;
            T2<R> *pi = static_cast<T2<R> *>(ptrs.p[i]);
            T2<R> pv = ldv<NT>(&pi[j]);
            if (RAT) {
                defer_combine<T2<R>, R>(h, i, rr, acc, pv);
            } else {
                T2<R> *xi = static_cast<T2<R> *>(ptrs.x[i]);
                T2<R> xv = ldv<NT>(&xi[j]);
                defer_combine<T2<R>, R>(h, i, rr, xv, pv);
                stv<NT>(&xi[j], xv);
            }
            stv<NT>(&pi[j], pv);
        }
        if (RAT) stv<NT>(&out[j], acc);
    }
}

__global__ void __launch_bounds__(kBlasBlock) k_scale(const double2 *b, double c, double2 *out, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const double2 v = b[j];
        out[j] = make_double2(c * v.x, c * v.y);
    }
}

__global__ void __launch_bounds__(kBlasBlock) k_dot_re(const double2 *a, const double2 *b, int64_t n,
                                                    double *partial) {
    __shared__ double red[kBlasBlock / kWave];
    double part = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const double2 u = a[j], v = b[j];
        part += u.x * v.x + u.y * v.y;
    }
    const double s = block_sum(part, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlasBlock) k_x_flush(const MsState *st, ShiftPtrs hi, ShiftPtrs lo, int n_shift,
                                                     int64_t n, int gated) {
    if (gated && st->rel_skip) return;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        for (int i = 0; i < n_shift; ++i) {
            double2 *h = static_cast<double2 *>(hi.x[i]);
            float2 *l = static_cast<float2 *>(lo.x[i]);
            const float2 lv = l[j];
            double2 hv = h[j];
            hv.x += double(lv.x);
            hv.y += double(lv.y);
            h[j] = hv;
            l[j] = make_float2(0.f, 0.f);
        }
    }
}

__global__ void __launch_bounds__(kBlasBlock) k_demote(const MsState *st, const double2 *src, float2 *dst, int64_t n) {
    if (st->rel_skip) return;
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const double2 v = src[j];
        dst[j] = make_float2(float(v.x), float(v.y));
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlasBlock) k_restart(const double2 *rhi, T2<R> *r, T2<R> *p, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kBlasBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlasBlock) {
        const double2 v = rhi[j];
        T2<R> w;
        w.x = R(v.x);
        w.y = R(v.y);
        r[j] = w;
        p[j] = w;
    }
}

// ---------------------------------------------------------------- scalars (one wave)

// rho from partial_r; ||b||^2 from partial_b, or equal to rho when
// partial_b is null (zero start: r = b).  One wave.
__global__ void __launch_bounds__(kWave) k_scalar_init(MsState *st, const double *partial_r, int nparts_r,
                                                    const double *partial_b, int nparts_b) {
    const double rho = sum_partials(partial_r, nparts_r);
    const double b2 = partial_b ? sum_partials(partial_b, nparts_b) : rho;
    ms_init_step(st, rho, b2);
}

// One workgroup: sum the partials in a fixed order, then apply the step.
constexpr int kTailBlock = 256;
__global__ void __launch_bounds__(kTailBlock) k_reduce_tail(MsState *st, const double *partial, int nparts, int kind,
                                                         int idx) {
    __shared__ double red[kTailBlock / kWave];
    if (kind == TAIL_ALPHA && st->done) {
        // the solve ended: retire the last update so later launches skip it
        if (threadIdx.x == 0) st->upd_valid = 0;
        return;
    }
    if (kind == TAIL_BETA && st->done) return;
    if (kind == TAIL_RELIABLE && st->rel_skip) return;
    const double total = block_sum(part_sum<kTailBlock>(partial, nparts), red);
    if (kind == TAIL_ALPHA) {
        if (threadIdx.x == 0) st->upd_valid = 0;
        ms_alpha_step(st, total);
    } else if (kind == TAIL_BETA) {
        ms_beta_step(st, total);
    } else if (kind == TAIL_RELIABLE) {
        if (threadIdx.x == 0) {
            st->rho = total;
            st->rho_rel = total;
            st->n_reliable += 1;
        }
    } else if (kind == TAIL_TRUE_RESID) {
        if (threadIdx.x == 0) st->resid_true[idx] = st->bnorm2 > 0.0 ? sqrt(total / st->bnorm2) : sqrt(total);
    } else if (kind == TAIL_SCRATCH) {
        if (threadIdx.x == 0) st->scratch[idx] = total;
    }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_reduce_tail(MsState *st, const double *partial, int nparts, int kind, int idx, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_tail, dim3(1), dim3(kTailBlock), 0, s, st, partial, nparts, kind, idx);
    return hipGetLastError();
}

hipError_t launch_norm2(bool dbl, const void *v, int64_t n, double *partial, int grid, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_norm2<double>, dim3(grid), dim3(kBlasBlock), 0, s, static_cast<const double2 *>(v), n, partial);
    else hipLaunchKernelGGL(k_norm2<float>, dim3(grid), dim3(kBlasBlock), 0, s, static_cast<const float2 *>(v), n, partial);
    return hipGetLastError();
}

hipError_t launch_ms_start(bool dbl, const double2 *b, void *r, ShiftPtrs ptrs, int n_shift, bool zero_x, int64_t n,
                           hipStream_t s) {
    const int grid = blas_grid(n);
    if (dbl) hipLaunchKernelGGL(k_ms_start<double>, dim3(grid), dim3(kBlasBlock), 0, s, b, static_cast<double2 *>(r), ptrs, n_shift, zero_x ? 1 : 0, n);
    else hipLaunchKernelGGL(k_ms_start<float>, dim3(grid), dim3(kBlasBlock), 0, s, b, static_cast<float2 *>(r), ptrs, n_shift, zero_x ? 1 : 0, n);
    return hipGetLastError();
}

hipError_t launch_scalar_init(MsState *st, const double *partial_r, int nparts_r, const double *partial_b,
                              int nparts_b, hipStream_t s) {
    hipLaunchKernelGGL(k_scalar_init, dim3(1), dim3(kWave), 0, s, st, partial_r, nparts_r, partial_b, nparts_b);
    return hipGetLastError();
}

hipError_t launch_r_update(bool dbl, MsState *st, const void *rin, void *r, const void *ap, int64_t n, double *partial,
                           int grid, hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_r_update<double>, dim3(grid), dim3(kBlasBlock), 0, s, st, static_cast<const double2 *>(rin), static_cast<double2 *>(r), static_cast<const double2 *>(ap), n, partial);
    else hipLaunchKernelGGL(k_r_update<float>, dim3(grid), dim3(kBlasBlock), 0, s, st, static_cast<const float2 *>(rin), static_cast<float2 *>(r), static_cast<const float2 *>(ap), n, partial);
    return hipGetLastError();
}

template <bool RAT, bool NT>
static void defer_apply64(const MsState *st, const DeferHist *h, const void *ring, int64_t slot_elems, ShiftPtrs ptrs,
                          int n_shift, int64_t n, int grid, hipStream_t s, void *out) {
    hipLaunchKernelGGL((k_defer_apply<double, RAT, NT>), dim3(grid), dim3(kBlasBlock), 0, s, st, h,
                       static_cast<const double2 *>(ring), slot_elems, ptrs, n_shift, n, static_cast<double2 *>(out));
}

hipError_t launch_defer_pass(bool dbl, MsState *st, DeferHist *h, const void *ring, int64_t slot_elems, ShiftPtrs ptrs,
                             int n_shift, int64_t n, int grid, hipStream_t s, void *out, bool nt) {
    hipLaunchKernelGGL(k_defer_coef, dim3(1), dim3(kWave), 0, s, st, h);
    if (out && !dbl) return hipErrorInvalidValue;
    if (dbl) {
        if (out) {
            if (nt) defer_apply64<true, true>(st, h, ring, slot_elems, ptrs, n_shift, n, grid, s, out);
            else defer_apply64<true, false>(st, h, ring, slot_elems, ptrs, n_shift, n, grid, s, out);
        } else {
            if (nt) defer_apply64<false, true>(st, h, ring, slot_elems, ptrs, n_shift, n, grid, s, nullptr);
            else defer_apply64<false, false>(st, h, ring, slot_elems, ptrs, n_shift, n, grid, s, nullptr);
        }
    } else {
        hipLaunchKernelGGL((k_defer_apply<float, false, false>), dim3(grid), dim3(kBlasBlock), 0, s, (const MsState *)st, (const DeferHist *)h, static_cast<const float2 *>(ring), slot_elems, ptrs, n_shift, n, (float2 *)nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_r_update_fused(bool dbl, MsState *st, const double *pq_part, int npq, const void *rin, void *r,
                                 const void *ap, int64_t n, double *partial, int grid, hipStream_t s, bool nt) {
    if (dbl && nt) hipLaunchKernelGGL((k_r_update_fused<double, true>), dim3(grid), dim3(kBlasBlock), 0, s, st, pq_part, npq, static_cast<const double2 *>(rin), static_cast<double2 *>(r), static_cast<const double2 *>(ap), n, partial);
    else if (dbl) hipLaunchKernelGGL((k_r_update_fused<double, false>), dim3(grid), dim3(kBlasBlock), 0, s, st, pq_part, npq, static_cast<const double2 *>(rin), static_cast<double2 *>(r), static_cast<const double2 *>(ap), n, partial);
    else hipLaunchKernelGGL((k_r_update_fused<float, false>), dim3(grid), dim3(kBlasBlock), 0, s, st, pq_part, npq, static_cast<const float2 *>(rin), static_cast<float2 *>(r), static_cast<const float2 *>(ap), n, partial);
    return hipGetLastError();
}

hipError_t launch_dir_update_fused(bool dbl, MsState *st, const double *r_part, int nr, const void *r, void *pd,
                                   int64_t n, int grid, hipStream_t s, bool nt) {
    if (dbl && nt) hipLaunchKernelGGL((k_dir_update_fused<double, true>), dim3(grid), dim3(kBlasBlock), 0, s, st, r_part, nr, static_cast<const double2 *>(r), static_cast<double2 *>(pd), n);
    else if (dbl) hipLaunchKernelGGL((k_dir_update_fused<double, false>), dim3(grid), dim3(kBlasBlock), 0, s, st, r_part, nr, static_cast<const double2 *>(r), static_cast<double2 *>(pd), n);
    else hipLaunchKernelGGL((k_dir_update_fused<float, false>), dim3(grid), dim3(kBlasBlock), 0, s, st, r_part, nr, static_cast<const float2 *>(r), static_cast<float2 *>(pd), n);
    return hipGetLastError();
}

hipError_t launch_scale(const double2 *b, double c, double2 *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(blas_grid(n)), dim3(kBlasBlock), 0, s, b, c, out, n);
    return hipGetLastError();
}

hipError_t launch_dot_re(const double2 *a, const double2 *b, int64_t n, double *partial, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_re, dim3(grid), dim3(kBlasBlock), 0, s, a, b, n, partial);
    return hipGetLastError();
}

hipError_t launch_shift_update(bool dbl, MsState *st, const void *r, ShiftPtrs ptrs, int n_shift, int64_t n, int grid,
                               hipStream_t s) {
    if (dbl) hipLaunchKernelGGL(k_shift_update<double>, dim3(grid), dim3(kBlasBlock), 0, s, st, static_cast<const double2 *>(r), ptrs, n_shift, n);
    else hipLaunchKernelGGL(k_shift_update<float>, dim3(grid), dim3(kBlasBlock), 0, s, st, static_cast<const float2 *>(r), ptrs, n_shift, n);
    return hipGetLastError();
}

hipError_t launch_x_flush(MsState *st, ShiftPtrs hi, ShiftPtrs lo, int n_shift, int64_t n, bool gated,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_x_flush, dim3(blas_grid(n)), dim3(kBlasBlock), 0, s, st, hi, lo, n_shift, n, gated ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_demote(MsState *st, const double2 *src, float2 *dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_demote, dim3(blas_grid(n)), dim3(kBlasBlock), 0, s, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_restart(bool dbl, const double2 *rhi, void *r, void *p, int64_t n, hipStream_t s) {
    const int grid = blas_grid(n);
    if (dbl) hipLaunchKernelGGL(k_restart<double>, dim3(grid), dim3(kBlasBlock), 0, s, rhi, static_cast<double2 *>(r), static_cast<double2 *>(p), n);
    else hipLaunchKernelGGL(k_restart<float>, dim3(grid), dim3(kBlasBlock), 0, s, rhi, static_cast<float2 *>(r), static_cast<float2 *>(p), n);
    return hipGetLastError();
}

}  // namespace stag
