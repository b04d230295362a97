// Vector kernels and scalar tails of the batched shifted CG.
//
// grid.y indexes the system; grid.x covers its vector in chunks of 256
// entries, one wave per chunk (4 entries per lane, coalesced).  Blocks past a
// system's last chunk return at once, so lattices of different sizes share
// a launch.  Reductions leave one partial per chunk; the tail kernel (one
// workgroup per system) sums them in a fixed order and advances that
// system's recursion.
#include <math.h>

#include "batch.h"
#include "ms_device.h"

namespace stag {

template <typename R> using T2 = typename vtype<R>::t2;

template <typename R> __device__ __forceinline__ T2<R> mk2(R a, R b) {
    T2<R> v;
    v.x = a;
    v.y = b;
    return v;
}

__host__ __device__ __forceinline__ int ring_slot(int k, int d) { return ((k % d) + d) % d; }

template <typename R>
__global__ void __launch_bounds__(kBBlock) kb_vec(BView v, int op, int it) {
    const BSys &s = v.sys[blockIdx.y];
    constexpr int kWavesPerBlock = kBBlock / kWave;
    if ((int)blockIdx.x * kWavesPerBlock >= s.nchunk_bl) return;
    MsState *st = s.st;
    const int64_t n = 3 * (int64_t)v.lats[s.lat].g.Vh;
    const int lane = threadIdx.x & (kWave - 1);
    const int chunk = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t j0 = (int64_t)chunk * kBChunk + lane;
    double part = 0.0;
    bool reduce = false;
    // residual of iteration k: its ring slot (deferred systems) or s.r
    auto rvec = [&](int k) -> T2<R> * {
        return s.dlen ? static_cast<T2<R> *>(s.ring) + (int64_t)ring_slot(k, s.dlen) * n : static_cast<T2<R> *>(s.r);
    };

    if (op == BV_START) {
        T2<R> *r = rvec(-1);
        T2<R> *pd = static_cast<T2<R> *>(s.pd);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            const double2 b = s.src[j];
            const T2<R> bv = mk2<R>(R(b.x), R(b.y));
            r[j] = bv;
            if (s.dlen) pd[j] = bv;
            if (s.rat) {   // out = w0 src; no solution vectors
                s.out[j] = make_double2(s.w0 * b.x, s.w0 * b.y);
                for (int i = 0; i < s.n; ++i) static_cast<T2<R> *>(s.p[i])[j] = bv;
                continue;
            }
            for (int i = 0; i < s.n; ++i) {
                static_cast<T2<R> *>(s.p[i])[j] = bv;
                static_cast<T2<R> *>(s.x[i])[j] = mk2<R>(R(0), R(0));
                if (sizeof(R) != sizeof(double)) s.xhi[i][j] = make_double2(0.0, 0.0);
            }
        }
    } else if (op == BV_RESTART) {
        T2<R> *r = static_cast<T2<R> *>(s.r);
        T2<R> *p = static_cast<T2<R> *>(s.p[s.base]);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            const double2 h = s.rhi[j];
            const T2<R> rv = mk2<R>(R(h.x), R(h.y));
            r[j] = rv;
            p[j] = rv;
            if (sizeof(R) != sizeof(double)) static_cast<T2<R> *>(s.x[0])[j] = mk2<R>(R(0), R(0));
        }
    } else if (op == BV_NORM_SRC) {
        reduce = true;
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j < n) {
                const double2 b = s.src[j];
                part += b.x * b.x + b.y * b.y;
            }
        }
    } else if (op == BV_R_UPDATE || op == BV_R_UPDATE_FUSED) {
        if (st->done) return;
        reduce = true;
        R alpha;
        if (op == BV_R_UPDATE_FUSED) {
            __shared__ double red[kBBlock / kWave];
            const double pap = block_sum(part_sum<kBBlock>(s.part_ds, s.nchunk_ds), red);
            if (blockIdx.x == 0) {
                if (threadIdx.x == 0) st->rho_snap = st->rho;
                ms_alpha_step(st, pap);
            }
            if (!(pap > 0.0) || !isfinite(pap)) return;
            alpha = R(st->rho / pap);   // rho is not written by this kernel
        } else {
            alpha = R(st->alpha);
        }
        const T2<R> *rin = rvec(it - 1);
        T2<R> *r = rvec(it);
        const T2<R> *ap = static_cast<const T2<R> *>(s.ap);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j < n) {
                T2<R> rv = rin[j];
                const T2<R> q = ap[j];
                rv.x -= alpha * q.x;
                rv.y -= alpha * q.y;
                r[j] = rv;
                part += double(rv.x) * double(rv.x) + double(rv.y) * double(rv.y);
            }
        }
    } else if ((op == BV_SHIFT_UPDATE && s.dlen) || op == BV_DIR_FUSED) {
        // deferred system: only the base direction pd = r + beta pd
        if (st->done) return;
        const T2<R> *r = rvec(it);
        T2<R> *pd = static_cast<T2<R> *>(s.pd);
        R beta;
        if (op == BV_DIR_FUSED) {
            __shared__ double red[kBBlock / kWave];
            const double rho_new = block_sum(part_sum<kBBlock>(s.part_bl, s.nchunk_bl), red);
            beta = R(rho_new / st->rho_snap);   // block 0 rewrites rho below, not rho_snap
            if (blockIdx.x == 0) ms_beta_step(st, rho_new);
        } else {
            beta = R(st->beta);
        }
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            const T2<R> rv = r[j];
            const T2<R> pv = pd[j];
            pd[j] = mk2<R>(rv.x + beta * pv.x, rv.y + beta * pv.y);
        }
    } else if (op == BV_SHIFT_UPDATE) {
        if (!st->upd_valid) return;
        const T2<R> *r = static_cast<const T2<R> *>(s.r);
        const int base = s.base, upd_p = st->upd_p;
        const R beta = R(st->beta);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            const T2<R> rv = r[j];
            for (int i = 0; i < s.n; ++i) {
                T2<R> *pi = static_cast<T2<R> *>(s.p[i]);
                if (st->upd[i]) {
                    T2<R> *xi = static_cast<T2<R> *>(s.x[i]);
                    const R ai = R(st->a[i]), bi = R(st->b[i]), zi = R(st->zeta[i]);
                    const T2<R> pv = pi[j];
                    T2<R> xv = xi[j];
                    xv.x += ai * pv.x;
                    xv.y += ai * pv.y;
                    xi[j] = xv;
                    pi[j] = mk2<R>(zi * rv.x + bi * pv.x, zi * rv.y + bi * pv.y);
                } else if (i == base && upd_p) {
                    const T2<R> pv = pi[j];
                    pi[j] = mk2<R>(rv.x + beta * pv.x, rv.y + beta * pv.y);
                }
            }
        }
    } else if (op == BV_FLUSH || op == BV_FLUSH_FINAL) {
        if (op == BV_FLUSH && st->rel_skip) return;
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            for (int i = 0; i < s.n; ++i) {
                T2<R> *xl = static_cast<T2<R> *>(s.x[i]);
                const T2<R> lv = xl[j];
                double2 hv = s.xhi[i][j];
                hv.x += double(lv.x);
                hv.y += double(lv.y);
                s.xhi[i][j] = hv;
                xl[j] = mk2<R>(R(0), R(0));
            }
        }
    } else if (op == BV_DEFER_APPLY) {
        if (!s.dlen) return;
        const DeferHist *h = s.hist;
        const int nv = h->nvalid;
        if (nv == 0) return;
        const T2<R> *ring = static_cast<const T2<R> *>(s.ring);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            T2<R> rr[kDefer];
#pragma unroll
            for (int m = 0; m < kDefer; ++m) rr[m] = m < nv ? ring[m * n + j] : mk2<R>(R(0), R(0));
            T2<R> acc;
            if (s.rat) acc = mk2<R>(R(s.out[j].x), R(s.out[j].y));
            for (int i = 0; i < s.n; ++i) {
                if (!h->act[i]) continue;
                T2<R> *pi = static_cast<T2<R> *>(s.p[i]);
                T2<R> pv = pi[j];
                if (s.rat) {   // weighted increments of every shift into out
                    defer_combine<T2<R>, R>(h, i, rr, acc, pv);
                } else {
                    T2<R> *xi = static_cast<T2<R> *>(s.x[i]);
                    T2<R> xv = xi[j];
                    defer_combine<T2<R>, R>(h, i, rr, xv, pv);
                    xi[j] = xv;
                }
                pi[j] = pv;
            }
            if (s.rat) s.out[j] = make_double2(double(acc.x), double(acc.y));
        }
    } else if (op == BV_DEMOTE) {
        if (st->rel_skip) return;
        T2<R> *r = rvec(it);
        for (int e = 0; e < 4; ++e) {
            const int64_t j = j0 + e * kWave;
            if (j >= n) break;
            const double2 h = s.rhi[j];
            r[j] = mk2<R>(R(h.x), R(h.y));
        }
    }
    if (reduce) {
        const double w = wave_sum(part);
        if (lane == 0 && chunk < s.nchunk_bl) s.part_bl[chunk] = w;
    }
}

hipError_t launch_bvec(bool dbl, BView v, int op, int max_blocks, hipStream_t s, int it) {
    if (v.nsys <= 0) return hipSuccess;
    const dim3 grid(max_blocks, v.nsys), blk(kBBlock);
    if (dbl) hipLaunchKernelGGL(kb_vec<double>, grid, blk, 0, s, v, op, it);
    else hipLaunchKernelGGL(kb_vec<float>, grid, blk, 0, s, v, op, it);
    return hipGetLastError();
}

// One wave per system (deferred systems only).
__global__ void __launch_bounds__(kWave) kb_defer_coef(BView v) {
    const BSys &s = v.sys[blockIdx.x];
    if (!s.dlen) return;
    defer_coef_step(s.n, s.hist, s.st->rat ? s.st->wgt : nullptr);
}

hipError_t launch_bdefer_coef(BView v, hipStream_t s) {
    if (v.nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_defer_coef, dim3(v.nsys), dim3(kWave), 0, s, v);
    return hipGetLastError();
}

// One workgroup per system: sum the partials in a fixed order, then apply
// the step of the shifted recursion.
constexpr int kBTailBlock = 256;
__global__ void __launch_bounds__(kBTailBlock) kb_tail(BView v, int kind, int idx) {
    __shared__ double red[kBTailBlock / kWave];
    const BSys &s = v.sys[blockIdx.x];
    MsState *st = s.st;
    if (kind == BT_TRUE_RESID) {
        if (s.rat || idx >= s.n) return;
        const double total = block_sum(part_sum<kBTailBlock>(s.part_ds, s.nchunk_ds), red);
        if (threadIdx.x == 0) st->resid_true[idx] = st->bnorm2 > 0.0 ? sqrt(total / st->bnorm2) : sqrt(total);
        return;
    }
    if (kind == BT_ALPHA) {
        if (threadIdx.x == 0) st->upd_valid = 0;  // retire the previous update
        if (st->done) return;
    }
    if (kind == BT_BETA && st->done) return;
    const bool use_ds = kind == BT_ALPHA;
    const double *part = use_ds ? s.part_ds : s.part_bl;
    const int np = use_ds ? s.nchunk_ds : s.nchunk_bl;
    const double total = block_sum(part_sum<kBTailBlock>(part, np), red);
    if (kind == BT_INIT) ms_init_step(st, total, total);   // zero start: r = b
    else if (kind == BT_ALPHA) ms_alpha_step(st, total);
    else ms_beta_step(st, total);
}

hipError_t launch_btail(BView v, int kind, hipStream_t s, int idx) {
    if (v.nsys <= 0) return hipSuccess;
    hipLaunchKernelGGL(kb_tail, dim3(v.nsys), dim3(kBTailBlock), 0, s, v, kind, idx);
    return hipGetLastError();
}

// flag[0] = 1 once every system of the batch has finished.  One wave.
__global__ void __launch_bounds__(kWave) kb_all_done(BView v, int *flag) {
    int notdone = 0;
    for (int k = threadIdx.x; k < v.nsys; k += kWave) notdone |= v.sys[k].st->done ? 0 : 1;
    const unsigned long long b = __ballot(notdone != 0);
    if (threadIdx.x == 0) flag[0] = b ? 0 : 1;
}

hipError_t launch_ball_done(BView v, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(kb_all_done, dim3(1), dim3(kWave), 0, s, v, flag);
    return hipGetLastError();
}

}  // namespace stag
