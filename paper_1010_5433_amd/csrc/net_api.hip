// Host side of the learned preconditioner: parameter handling, the forward
// application, gradients, one Adam training step, and the flexible CG that
// uses the network as its preconditioner.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "internal.h"
#include "net.h"
#include "solver.h"

namespace stag {

hipError_t net_launch_prep(const float2 *theta, NetDev *w, hipStream_t s);
hipError_t net_launch_forward(const NetArgs &a, int n_samples, int mix, hipStream_t s);
hipError_t net_launch_backward(const NetArgs &a, int n_samples, const float2 *gin, float2 *g2, float2 *partE,
                               float2 *partO, double2 *grad, hipStream_t s);
hipError_t net_launch_loss(const NetArgs &a, int n_samples, const float2 *xs, double *xnorm2, double *norm_part,
                           float2 *gout, double *loss_part, double *loss_rows, hipStream_t s);
hipError_t net_launch_adam(float2 *theta, float2 *m, float2 *v, const double2 *grad, int t, float lr, hipStream_t s);
int net_blocks_even_bwd(const Geom &g);
int net_blocks_odd_bwd(const Geom &g);
int net_part_e();
int net_part_o();
int net_loss_blocks(const Geom &g);

stag_status single_cg(stag_lattice *lat, double mass, double shift, const void *src, void *x, double tol,
                      int max_iter, stag_prec prec, stag_cg_stats *stats, hipStream_t s);

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Work buffers of the network for n samples of a lattice.
struct NetBufs {
    float2 *phi1, *phi2, *out, *g, *g2, *partE, *partO;
    double *xnorm2, *norm_part, *loss_part, *loss_rows;
    double2 *grad;
};

static stag_status net_work(stag_net *net, const stag_lattice *lat, int n, NetBufs *b) {
    const size_t vh = (size_t)lat->Vh;
    const size_t f24 = al(sizeof(float2) * vh * 24 * n), vec = al(sizeof(float2) * 3 * vh * n);
    const int nbe = net_blocks_even_bwd(lat->g), nbo = net_blocks_odd_bwd(lat->g), nbl = net_loss_blocks(lat->g);
    const size_t pe = al(sizeof(float2) * (size_t)nbe * n * net_part_e()), po = al(sizeof(float2) * (size_t)nbo * n * net_part_o());
    const size_t dn = al(sizeof(double) * n), dnl = al(sizeof(double) * (size_t)nbl * n);
    const size_t bytes = 3 * f24 + 2 * vec + pe + po + 2 * dn + 2 * dnl + al(sizeof(double2) * kNetNParam);
    if (net->work_bytes < bytes) {
        if (net->work) {
            STAG_HIP(hipDeviceSynchronize());
            STAG_HIP(hipFree(net->work));
            net->work = nullptr;
            net->work_bytes = 0;
        }
        STAG_HIP(hipMalloc(&net->work, bytes));
        net->work_bytes = bytes;
    }
    char *p = static_cast<char *>(net->work);
    auto take = [&](size_t n2) {
        char *q = p;
        p += n2;
        return q;
    };
    b->phi1 = reinterpret_cast<float2 *>(take(f24));
    b->phi2 = reinterpret_cast<float2 *>(take(f24));
    b->g2 = reinterpret_cast<float2 *>(take(f24));
    b->out = reinterpret_cast<float2 *>(take(vec));
    b->g = reinterpret_cast<float2 *>(take(vec));
    b->partE = reinterpret_cast<float2 *>(take(pe));
    b->partO = reinterpret_cast<float2 *>(take(po));
    b->xnorm2 = reinterpret_cast<double *>(take(dn));
    b->loss_rows = reinterpret_cast<double *>(take(dn));
    b->norm_part = reinterpret_cast<double *>(take(dnl));
    b->loss_part = reinterpret_cast<double *>(take(dnl));
    b->grad = reinterpret_cast<double2 *>(take(al(sizeof(double2) * kNetNParam)));
    return STAG_OK;
}

static NetArgs net_args(const stag_net *net, const stag_lattice *lat, const void *r, float2 *out, const NetBufs &b,
                        bool keep_phi2) {
    NetArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.links = lat->links32;
    a.nrow = lat->nrow;
    a.w = net->w;
    a.r = static_cast<const float2 *>(r);
    a.out = out;
    a.phi1 = b.phi1;
    a.phi2 = keep_phi2 ? b.phi2 : nullptr;
    a.vstride = 3 * lat->Vh;
    return a;
}

// ---------------------------------------------------------------- flexible CG
constexpr int kFcgBlock = 256;

__global__ void __launch_bounds__(kFcgBlock) k_fcg_sum(const double *part, int n, double *out) {
    __shared__ double red[kFcgBlock / kWave];
    double t = 0.0;
    for (int k = threadIdx.x; k < n; k += kFcgBlock) t += part[k];
    const double s = block_sum(t, red);
    if (threadIdx.x == 0) out[0] = s;
}

// x += alpha p; r_old = r; r -= alpha q; partial |r|^2
__global__ void __launch_bounds__(kFcgBlock) k_fcg_step(double2 *x, double2 *r, double2 *rold, const double2 *p,
                                                     const double2 *q, double alpha, int64_t n, double *part) {
    __shared__ double red[kFcgBlock / kWave];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const double2 pv = p[j], qv = q[j];
        double2 xv = x[j], rv = r[j];
        rold[j] = rv;
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        rv.x -= alpha * qv.x;
        rv.y -= alpha * qv.y;
        x[j] = xv;
        r[j] = rv;
        acc += rv.x * rv.x + rv.y * rv.y;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kFcgBlock) k_fcg_demote(const double2 *r, float2 *r32, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock)
        r32[j] = make_float2(float(r[j].x), float(r[j].y));
}

// z = (double) z32; partials of Re<z, r - r_old> and Re<r, z>
__global__ void __launch_bounds__(kFcgBlock) k_fcg_z(const float2 *z32, double2 *z, const double2 *r, const double2 *rold,
                                                  int64_t n, double *part_a, double *part_b) {
    __shared__ double red[kFcgBlock / kWave];
    double a = 0.0, b = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const double2 zv = make_double2(double(z32[j].x), double(z32[j].y));
        z[j] = zv;
        const double2 rv = r[j], ro = rold[j];
        a += zv.x * (rv.x - ro.x) + zv.y * (rv.y - ro.y);
        b += zv.x * rv.x + zv.y * rv.y;
    }
    const double sa = block_sum(a, red);
    const double sb = block_sum(b, red);
    if (threadIdx.x == 0) {
        part_a[blockIdx.x] = sa;
        part_b[blockIdx.x] = sb;
    }
}

// p = z + beta p
__global__ void __launch_bounds__(kFcgBlock) k_fcg_dir(double2 *p, const double2 *z, double beta, int64_t n) {
    for (int64_t j = (int64_t)blockIdx.x * kFcgBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kFcgBlock) {
        const double2 zv = z[j];
        double2 pv = p[j];
        pv.x = zv.x + beta * pv.x;
        pv.y = zv.y + beta * pv.y;
        p[j] = pv;
    }
}

stag_status fcg_solve(stag_lattice *lat, double mass, double shift, const void *src, void *sol, stag_net *net,
                      double tol, int max_iter, stag_cg_stats *stats, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    stag_cg_stats st;
    std::memset(&st, 0, sizeof(st));
    if (!net) {   // plain double precision CG
        STAG_TRY(single_cg(lat, mass, shift, src, sol, tol, max_iter, STAG_F64, &st, s));
        if (stats) *stats = st;
        return STAG_OK;
    }
    const int64_t ne = 3 * lat->Vh;
    const size_t vb = sizeof(double2) * ne;
    const int ds_grid = dslash_grid(lat->g, kDslashBlock);
    const int grid = (int)std::min<int64_t>((ne + kFcgBlock - 1) / kFcgBlock, 2048);
    const int nparts = std::max(ds_grid, grid);
    void *W = nullptr;
    const size_t bytes = 6 * al(vb) + al(sizeof(float2) * ne) * 2 + 3 * al(sizeof(double) * nparts) + 256;
    STAG_TRY(ws_get(lat, WS_E2, bytes, &W));
    char *cur = static_cast<char *>(W);
    auto take = [&](size_t n) {
        char *q = cur;
        cur += al(n);
        return q;
    };
    double2 *x = static_cast<double2 *>(sol), *b = static_cast<double2 *>(const_cast<void *>(src));
    double2 *r = reinterpret_cast<double2 *>(take(vb)), *rold = reinterpret_cast<double2 *>(take(vb));
    double2 *z = reinterpret_cast<double2 *>(take(vb)), *p = reinterpret_cast<double2 *>(take(vb));
    double2 *q = reinterpret_cast<double2 *>(take(vb)), *t = reinterpret_cast<double2 *>(take(vb));
    float2 *r32 = reinterpret_cast<float2 *>(take(sizeof(float2) * ne));
    float2 *z32 = reinterpret_cast<float2 *>(take(sizeof(float2) * ne));
    double *pa = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *pb = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *pc = reinterpret_cast<double *>(take(sizeof(double) * nparts));
    double *scal = reinterpret_cast<double *>(take(256));
    NetBufs nb;
    STAG_TRY(net_work(net, lat, 1, &nb));
    const double m2 = mass * mass;
    DslashArgs d;
    std::memset(&d, 0, sizeof(d));
    d.g = lat->g;
    d.links = lat->links64;

    auto reduce = [&](const double *part, int n, int slot) -> hipError_t {
        hipLaunchKernelGGL(k_fcg_sum, dim3(1), dim3(kFcgBlock), 0, s, part, n, scal + slot);
        return hipGetLastError();
    };
    auto fetch = [&](int nslots, double *h) -> stag_status {
        STAG_HIP(hipMemcpyAsync(h, scal, sizeof(double) * nslots, hipMemcpyDeviceToHost, s));
        STAG_HIP(hipStreamSynchronize(s));
        return STAG_OK;
    };
    // r = b - A x (double), partial |r|^2 -> slot 0; |b|^2 -> slot 1
    auto residual = [&]() -> stag_status {
        DslashArgs e = d;
        e.out_parity = 1;
        e.in = x;
        e.out = t;
        STAG_HIP(launch_dslash(true, lat->nrow, DS_PLAIN, e, s));
        e.out_parity = 0;
        e.in = t;
        e.out = r;
        e.aux = x;
        e.rhs = b;
        e.c = m2 + shift;
        e.partial = pa;
        STAG_HIP(launch_dslash(true, lat->nrow, DS_RESID, e, s));
        STAG_HIP(reduce(pa, ds_grid, 0));
        return STAG_OK;
    };
    auto precondition = [&]() -> stag_status {   // z = P(r); <z, r - r_old> -> slot 2, <r, z> -> slot 3
        hipLaunchKernelGGL(k_fcg_demote, dim3(grid), dim3(kFcgBlock), 0, s, (const double2 *)r, r32, ne);
        NetArgs a = net_args(net, lat, r32, z32, nb, false);
        STAG_HIP(net_launch_forward(a, 1, kMixBF16, s));
        hipLaunchKernelGGL(k_fcg_z, dim3(grid), dim3(kFcgBlock), 0, s, (const float2 *)z32, z, (const double2 *)r,
                           (const double2 *)rold, ne, pb, pc);
        STAG_HIP(hipGetLastError());
        STAG_HIP(reduce(pb, grid, 2));
        STAG_HIP(reduce(pc, grid, 3));
        return STAG_OK;
    };

    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    double h[4];
    // |b|^2
    STAG_HIP(launch_norm2(true, b, ne, pb, grid, s));
    STAG_HIP(reduce(pb, grid, 1));
    STAG_TRY(residual());
    STAG_TRY(fetch(2, h));
    const double bnorm = std::sqrt(h[1]);
    double rnorm = std::sqrt(h[0]);
    int it = 0;
    bool fallback = false, converged = bnorm == 0.0 || rnorm <= tol * bnorm;
    double best = rnorm;
    int since_best = 0;
    STAG_HIP(hipMemsetAsync(rold, 0, vb, s));
    if (!converged) {
        STAG_TRY(precondition());
        STAG_HIP(hipMemcpyAsync(p, z, vb, hipMemcpyDeviceToDevice, s));
        STAG_TRY(fetch(4, h));
        double rz = h[3];
        while (it < max_iter) {
            if (!(rz > 0.0) || !std::isfinite(rz)) {
                fallback = true;
                break;
            }
            DslashArgs e = d;
            e.out_parity = 1;
            e.in = p;
            e.out = t;
            STAG_HIP(launch_dslash(true, lat->nrow, DS_PLAIN, e, s));
            e.out_parity = 0;
            e.in = t;
            e.out = q;
            e.aux = p;
            e.c = m2 + shift;
            e.partial = pa;
            STAG_HIP(launch_dslash(true, lat->nrow, DS_NORMAL_DOT, e, s));
            STAG_HIP(reduce(pa, ds_grid, 0));
            STAG_TRY(fetch(1, h));
            const double pq = h[0];
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                fallback = true;
                break;
            }
            const double alpha = rz / pq;
            hipLaunchKernelGGL(k_fcg_step, dim3(grid), dim3(kFcgBlock), 0, s, x, r, rold, (const double2 *)p,
                               (const double2 *)q, alpha, ne, pa);
            STAG_HIP(hipGetLastError());
            STAG_HIP(reduce(pa, grid, 0));
            STAG_TRY(precondition());
            STAG_TRY(fetch(4, h));
            ++it;
            rnorm = std::sqrt(h[0]);
            if (rnorm <= tol * bnorm) {
                // the judge: the double precision true residual
                STAG_TRY(residual());
                STAG_TRY(fetch(1, h));
                rnorm = std::sqrt(h[0]);
                if (rnorm <= tol * bnorm) {
                    converged = true;
                    break;
                }
                STAG_TRY(precondition());   // restart from the true residual
                STAG_HIP(hipMemcpyAsync(p, z, vb, hipMemcpyDeviceToDevice, s));
                STAG_TRY(fetch(4, h));
                rz = h[3];
                continue;
            }
            if (rnorm < best) {
                best = rnorm;
                since_best = 0;
            } else if (++since_best >= 50) {
                fallback = true;   // stagnation
                break;
            }
            const double beta = h[2] / rz;   // Polak-Ribiere
            rz = h[3];
            hipLaunchKernelGGL(k_fcg_dir, dim3(grid), dim3(kFcgBlock), 0, s, p, (const double2 *)z, beta, ne);
            STAG_HIP(hipGetLastError());
        }
    }
    st.iters = it;
    if (fallback && it < max_iter) {
        stag_cg_stats cs;
        stag_status rc = single_cg(lat, mass, shift, src, sol, tol, max_iter - it, STAG_F64, &cs, s);
        if (rc < 0) return rc;
        st.iters += cs.iters;
        st.fallback_used = 1;
        st.resid_true[0] = cs.resid_true[0];
        converged = rc == STAG_OK;
    } else {
        STAG_TRY(residual());
        STAG_TRY(fetch(1, h));
        st.resid_true[0] = bnorm > 0 ? std::sqrt(h[0]) / bnorm : std::sqrt(h[0]);
        converged = st.resid_true[0] <= tol;
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

using namespace stag;

extern "C" {

stag_status stag_net_create(stag_net **out) {
    if (!out) return invalid("null argument");
    *out = nullptr;
    stag_net *net = new (std::nothrow) stag_net;
    if (!net) return STAG_ENOMEM;
    std::memset(net, 0, sizeof(*net));
    hipError_t e = hipGetDevice(&net->device);
    if (e == hipSuccess) e = hipMalloc(&net->theta, sizeof(float2) * kNetNParam * 3);
    if (e == hipSuccess) e = hipMalloc(&net->w, sizeof(NetDev));
    if (e != hipSuccess) {
        set_error(std::string("network set-up failed: ") + hipGetErrorString(e));
        (void)hipFree(net->theta);
        delete net;
        return STAG_EHIP;
    }
    net->adam_m = net->theta + kNetNParam;
    net->adam_v = net->theta + 2 * kNetNParam;
    e = hipMemset(net->theta, 0, sizeof(float2) * kNetNParam * 3);
    if (e != hipSuccess) {
        set_error("network set-up failed");
        return STAG_EHIP;
    }
    *out = net;
    return STAG_OK;
}

stag_status stag_net_destroy(stag_net *net) {
    if (!net) return STAG_OK;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(net->theta);
    (void)hipFree(net->w);
    (void)hipFree(net->work);
    delete net;
    return STAG_OK;
}

stag_status stag_net_set_params(stag_net *net, const double *theta) {
    if (!net || !theta) return invalid("null argument");
    std::vector<float2> h(kNetNParam);
    for (int j = 0; j < kNetNParam; ++j) h[j] = make_float2(float(theta[2 * j]), float(theta[2 * j + 1]));
    STAG_HIP(hipMemcpy(net->theta, h.data(), sizeof(float2) * kNetNParam, hipMemcpyHostToDevice));
    STAG_HIP(hipMemset(net->adam_m, 0, sizeof(float2) * kNetNParam * 2));
    net->adam_t = 0;
    return STAG_OK;
}

stag_status stag_net_get_params(const stag_net *net, double *theta) {
    if (!net || !theta) return invalid("null argument");
    std::vector<float2> h(kNetNParam);
    STAG_HIP(hipMemcpy(h.data(), net->theta, sizeof(float2) * kNetNParam, hipMemcpyDeviceToHost));
    for (int j = 0; j < kNetNParam; ++j) {
        theta[2 * j] = h[j].x;
        theta[2 * j + 1] = h[j].y;
    }
    return STAG_OK;
}

static stag_status check_net_lat(const stag_net *net, const stag_lattice *lat, int mode) {
    if (!net || !lat) return invalid("null handle");
    if (!lat->nrow) return invalid("links not set");
    if (mode != kMixBF16 && mode != kMixFP32) return invalid("mode must be 0 (BF16 matrix cores) or 1 (FP32)");
    return STAG_OK;
}

stag_status stag_net_apply(stag_net *net, stag_lattice *lat, const void *r, void *out, int mode, void *stream) {
    STAG_TRY(check_net_lat(net, lat, mode));
    if (!r || !out || r == out) return invalid("bad vector");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NetBufs b;
    STAG_TRY(net_work(net, lat, 1, &b));
    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    NetArgs a = net_args(net, lat, r, static_cast<float2 *>(out), b, false);
    STAG_HIP(net_launch_forward(a, 1, mode, s));
    return STAG_OK;
}

stag_status stag_net_grad(stag_net *net, stag_lattice *lat, const void *r, const void *g, double *grad, int mode,
                          void *stream) {
    STAG_TRY(check_net_lat(net, lat, mode));
    if (!r || !g || !grad) return invalid("null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NetBufs b;
    STAG_TRY(net_work(net, lat, 1, &b));
    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    NetArgs a = net_args(net, lat, r, b.out, b, true);
    STAG_HIP(net_launch_forward(a, 1, mode, s));
    STAG_HIP(net_launch_backward(a, 1, static_cast<const float2 *>(g), b.g2, b.partE, b.partO, b.grad, s));
    std::vector<double2> h(kNetNParam);
    STAG_HIP(hipMemcpyAsync(h.data(), b.grad, sizeof(double2) * kNetNParam, hipMemcpyDeviceToHost, s));
    STAG_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < kNetNParam; ++j) {
        grad[2 * j] = h[j].x;
        grad[2 * j + 1] = h[j].y;
    }
    return STAG_OK;
}

stag_status stag_net_train_step(stag_net *net, stag_lattice *lat, const void *b, const void *x, int n, double lr,
                                int mode, double *loss, void *stream) {
    STAG_TRY(check_net_lat(net, lat, mode));
    if (!b || !x || n < 1 || n > 1024) return invalid("bad batch");
    if (!(lr > 0) || !std::isfinite(lr)) return invalid("lr must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NetBufs w;
    STAG_TRY(net_work(net, lat, n, &w));
    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    NetArgs a = net_args(net, lat, b, w.out, w, true);
    STAG_HIP(net_launch_forward(a, n, mode, s));
    STAG_HIP(net_launch_loss(a, n, static_cast<const float2 *>(x), w.xnorm2, w.norm_part, w.g, w.loss_part,
                             w.loss_rows, s));
    STAG_HIP(net_launch_backward(a, n, w.g, w.g2, w.partE, w.partO, w.grad, s));
    net->adam_t += 1;
    STAG_HIP(net_launch_adam(net->theta, net->adam_m, net->adam_v, w.grad, net->adam_t, float(lr), s));
    if (loss) {
        STAG_HIP(hipMemcpyAsync(loss, w.loss_rows, sizeof(double), hipMemcpyDeviceToHost, s));
        STAG_HIP(hipStreamSynchronize(s));
    }
    return STAG_OK;
}

stag_status stag_fcg_solve(stag_lattice *lat, double mass, double shift, const void *src, void *sol, stag_net *net,
                           double tol, int max_iter, stag_cg_stats *stats, void *stream) {
    if (!lat || !lat->nrow) return invalid("lattice with links required");
    if (!src || !sol || src == sol) return invalid("bad vector");
    if (!(mass > 0) || !(shift >= 0) || !(tol > 0) || max_iter < 1) return invalid("bad solver parameter");
    return fcg_solve(lat, mass, shift, src, sol, net, tol, max_iter, stats, static_cast<hipStream_t>(stream));
}

}  // extern "C"
