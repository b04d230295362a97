// Learned gauge-equivariant preconditioner: parameter layout, device weight
// forms, kernel arguments and host entry points.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace stag {

constexpr int kNetC = 8;                 // channels
constexpr int kNetK = 72;                // layer-2 inputs per channel: self (8) + 8 hops x 8 channels
constexpr int kNetKR = 160;              // real layer-2 inputs padded to 5 x 32 for the matrix cores
constexpr int kNetW1S = 0, kNetW1H = 8, kNetW2 = 72, kNetWout = 648, kNetNParam = 656;

enum NetMix { kMixBF16 = 0, kMixFP32 = 1 };

// Weights in the forms the kernels read.
struct NetDev {
    float2 w1s[kNetC];
    float2 w1h[kNetC][8];          // [c][d]
    float2 W2[kNetC][kNetK];       // [c][k]
    float2 wout[kNetC];
    __hip_bfloat16 B[16][kNetKR];  // real form of W2 for the matrix cores: B[n][kr]
};

struct NetArgs {
    Geom g;
    const void *links;      // packed single precision links of the lattice
    int nrow;
    const NetDev *w;
    const float2 *r;        // input  (samples x [3][V/2]) even sites
    float2 *out;            // output (samples x [3][V/2]) even sites
    float2 *phi1;           // layer-1 field, odd sites: samples x [V/2][8][3]
    float2 *phi2;           // layer-2 field, even sites: samples x [V/2][8][3] (training only; may be null)
    int64_t vstride;        // complex entries between samples of r/out (3 V/2)
};

// per-lattice work buffers of the network (owned by the net handle)
struct NetWork {
    void *buf;
    size_t bytes;
};

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
