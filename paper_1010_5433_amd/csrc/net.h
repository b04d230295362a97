// Learned gauge-equivariant preconditioner: parameter layout, device weight
// forms, kernel arguments and host entry points.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace stag {

constexpr int kNetC = 8;                 // channels
constexpr int kNetK = 72;                // layer-2 inputs per channel: self (8) + 8 hops x 8 channels
constexpr int kNetW1S = 0, kNetW1H = 8, kNetW2 = 72, kNetWout = 648, kNetNParam = 656;

// Evaluation modes: the layer-2 channel mixing in BF16 on the matrix cores,
// the same in FP32 on the vector ALU, the folded two-hop form (FP32), or the
// folded form reading bfloat16 links and storing its intermediate field in
// bfloat16 (FP32 arithmetic).
enum NetMix { kMixBF16 = 0, kMixFP32 = 1, kMixFolded = 2, kMixFoldedBF16 = 3 };
inline bool net_mode_ok(int m) { return m >= kMixBF16 && m <= kMixFoldedBF16; }
inline bool net_mode_folded(int m) { return m == kMixFolded || m == kMixFoldedBF16; }

// Weights in the forms the kernels read.
struct NetDev {
    float2 w1s[kNetC];
    float2 w1h[kNetC][8];          // [c][d]
    float2 W2[kNetC][kNetK];       // [c][k]
    float2 wout[kNetC];
    // folded form of the (linear) network: P r = fsig r + sum_d T_d psi_d with
    // psi_d = sum_d' fA[d][d'] T_d' r on odd sites
    float2 fsig;
    float2 fA[8][8];
    alignas(16) __hip_bfloat16 B[5 * 4 * 16 * 8];   // real form of W2 in matrix-core operand order
                                                     // [step][lane group][column][8 K values]
};

struct NetArgs {
    Geom g;
    const void *links;      // packed single precision links of the lattice
    int nrow;
    const void *links16;    // bfloat16 12-real copy (folded bfloat16 mode only)
    const NetDev *w;
    const float2 *r;        // input  (samples x [3][V/2]) even sites
    float2 *out;            // output (samples x [3][V/2]) even sites
    float2 *phi1;           // layer-1 field, odd sites: samples x [8][3][V/2] (24 planes)
    float2 *phi2;           // layer-2 field, even sites: samples x [8][3][V/2] (training only; may be null)
    int64_t vstride;        // complex entries between samples of r/out (3 V/2)
    const int *skip;        // if non-null and *skip != 0 the forward kernels return at once
};

// Work buffers of the network for n samples of a lattice (carved from the
// net handle's arena).
struct NetBufs {
    float2 *phi1, *phi2, *out, *g, *g2, *partE, *partO;
    double *xnorm2, *norm_part, *loss_part, *loss_rows;
    double2 *grad;
};

}  // namespace stag

struct stag_net;
namespace stag {
stag_status net_work(stag_net *net, const stag_lattice *lat, int n, NetBufs *b);
NetArgs net_args(const stag_net *net, const stag_lattice *lat, const void *r, float2 *out, const NetBufs &b,
                 bool keep_phi2);
hipError_t net_launch_prep(const float2 *theta, NetDev *w, hipStream_t s);
// Makes the bfloat16 link copy that mode kMixFoldedBF16 reads (once per link field).
stag_status net_prepare_links(stag_lattice *lat, int mode, hipStream_t s);
hipError_t net_launch_forward(const NetArgs &a, int n_samples, int mix, hipStream_t s);
}  // namespace stag

struct stag_net {
    int device;
    float2 *theta;          // FP32 master parameters (device, 656)
    float2 *adam_m, *adam_v;
    int adam_t;
    stag::NetDev *w;        // device weight forms
    void *work;             // work arena (grown on demand)
    size_t work_bytes;
};
