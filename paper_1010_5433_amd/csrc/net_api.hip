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
#include "links.h"
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

stag_status fcg_solve(stag_lattice *lat, double mass, double shift, const void *src, void *sol, stag_net *net,
                      int mode, double tol, int max_iter, stag_cg_stats *stats, hipStream_t s);

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

stag_status net_work(stag_net *net, const stag_lattice *lat, int n, NetBufs *b) {
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

NetArgs net_args(const stag_net *net, const stag_lattice *lat, const void *r, float2 *out, const NetBufs &b,
                 bool keep_phi2) {
    NetArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = lat->g;
    a.links = lat->links32;
    a.nrow = nrow_single(lat->nrow);
    a.links16 = lat->links16;
    a.w = net->w;
    a.r = static_cast<const float2 *>(r);
    a.out = out;
    a.phi1 = b.phi1;
    a.phi2 = keep_phi2 ? b.phi2 : nullptr;
    a.vstride = 3 * lat->Vh;
    return a;
}

stag_status net_prepare_links(stag_lattice *lat, int mode, hipStream_t s) {
    if (mode != kMixFoldedBF16 || lat->links16) return STAG_OK;
    STAG_HIP(hipMalloc(&lat->links16, (size_t)8 * lat->Vh * LinkLayout<BF16Link, 2>::kBytesPerLink));
    const hipError_t e = launch_pack_links16(lat->g, lat->links32, lat->nrow, lat->links16, s);
    if (e != hipSuccess) {
        (void)hipFree(lat->links16);
        lat->links16 = nullptr;
        STAG_HIP(e);
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

static const char *kModeError = "mode must be 0 (BF16 matrix cores), 1 (FP32), 2 (folded) or 3 (folded, bfloat16 links)";

static stag_status check_net_lat(const stag_net *net, const stag_lattice *lat, int mode) {
    if (!net || !lat) return invalid("null handle");
    if (!lat->nrow) return invalid("links not set");
    if (!net_mode_ok(mode)) return invalid(kModeError);
    return STAG_OK;
}

stag_status stag_net_apply(stag_net *net, stag_lattice *lat, const void *r, void *out, int mode, void *stream) {
    STAG_TRY(check_net_lat(net, lat, mode));
    if (!r || !out) return invalid("bad vector");
    if (ranges_overlap({r, (size_t)vec_bytes(lat, false)}, {out, (size_t)vec_bytes(lat, false)}))
        return invalid("r and out must not overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    NetBufs b;
    STAG_TRY(net_work(net, lat, 1, &b));
    STAG_TRY(net_prepare_links(lat, mode, s));
    STAG_HIP(net_launch_prep(net->theta, net->w, s));
    NetArgs a = net_args(net, lat, r, static_cast<float2 *>(out), b, false);
    STAG_HIP(net_launch_forward(a, 1, mode, s));
    return STAG_OK;
}

stag_status stag_net_grad(stag_net *net, stag_lattice *lat, const void *r, const void *g, double *grad, int mode,
                          void *stream) {
    STAG_TRY(check_net_lat(net, lat, mode));
    if (net_mode_folded(mode)) return invalid("gradients need the layered form (mode 0 or 1)");
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
    if (net_mode_folded(mode)) return invalid("training needs the layered form (mode 0 or 1)");
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
                           int mode, double tol, int max_iter, stag_cg_stats *stats, void *stream) {
    if (!lat || !lat->nrow) return invalid("lattice with links required");
    if (!src || !sol) return invalid("bad vector");
    if (ranges_overlap({src, (size_t)vec_bytes(lat, true)}, {sol, (size_t)vec_bytes(lat, true)}))
        return invalid("sol overlaps the source");
    if (!(mass > 0) || !(shift >= 0) || !(tol > 0) || max_iter < 1) return invalid("bad solver parameter");
    if (net && !net_mode_ok(mode)) return invalid(kModeError);
    return fcg_solve(lat, mass, shift, src, sol, net, mode, tol, max_iter, stats, static_cast<hipStream_t>(stream));
}

}  // extern "C"
