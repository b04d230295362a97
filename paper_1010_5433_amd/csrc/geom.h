// Lattice geometry on the device: even/odd site decoding, neighbour indices,
// staggered phases and the antiperiodic time boundary.  The operator kernels
// and the table-export kernel use exactly these functions.
//
// dims L = (x,y,z,t), lex = x0 + L0*(x1 + L1*(x2 + L2*x3)),
// parity = (x0+x1+x2+x3) & 1, eo index i = lex >> 1 (L0 even), so
//   i = (x0 >> 1) + (L0/2) * (x1 + L1*(x2 + L2*x3)).
#pragma once

#include <stdint.h>

namespace stag {

struct Geom {
    int L[4];
    int Lh0;        // L0 / 2
    int Vh;         // sites per parity
    int s[4];       // eo-index stride of a unit step in x1, x2, x3 (s[0] unused)
    int antiperiodic;
};

inline Geom make_geom(const int dims[4], int antiperiodic) {
    Geom g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = dims[mu];
    g.Lh0 = dims[0] / 2;
    g.s[0] = 0;
    g.s[1] = g.Lh0;
    g.s[2] = g.Lh0 * dims[1];
    g.s[3] = g.Lh0 * dims[1] * dims[2];
    g.Vh = g.s[3] * dims[3];
    g.antiperiodic = antiperiodic ? 1 : 0;
    return g;
}

// Coordinates of the site with eo index i on parity p.
__device__ __forceinline__ void site_coords(const Geom &g, int p, int i, int x[4]) {
    unsigned r = (unsigned)i;
    const unsigned xh = r % (unsigned)g.Lh0;
    r /= (unsigned)g.Lh0;
    x[1] = (int)(r % (unsigned)g.L[1]);
    r /= (unsigned)g.L[1];
    x[2] = (int)(r % (unsigned)g.L[2]);
    x[3] = (int)(r / (unsigned)g.L[2]);
    x[0] = 2 * (int)xh + ((p + x[1] + x[2] + x[3]) & 1);
}

// eo index of x + dir * mu-hat (dir = +1 or -1), periodic.
__device__ __forceinline__ int site_nbr(const Geom &g, int i, const int x[4], int mu, int dir) {
    const int L = g.L[mu];
    int y = x[mu] + dir;
    y = (y < 0) ? L - 1 : ((y == L) ? 0 : y);
    if (mu == 0) return i - (x[0] >> 1) + (y >> 1);
    return i + (y - x[mu]) * g.s[mu];
}

// eta_mu(x) = (-1)^(x0 + ... + x_{mu-1}) as +-1.
__device__ __forceinline__ int eta_sign(const int x[4], int mu) {
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += x[nu];
    return 1 - 2 * (s & 1);
}

// Sign of the forward hop x -> x+mu (link U_mu(x)) and of the backward hop
// x -> x-mu (link U_mu(x-mu)), phases and boundary included.
__device__ __forceinline__ int fwd_sign(const Geom &g, const int x[4], int mu) {
    const int bc = (g.antiperiodic && mu == 3 && x[3] == g.L[3] - 1) ? -1 : 1;
    return eta_sign(x, mu) * bc;
}
__device__ __forceinline__ int bwd_sign(const Geom &g, const int x[4], int mu) {
    const int bc = (g.antiperiodic && mu == 3 && x[3] == 0) ? -1 : 1;
    return eta_sign(x, mu) * bc;
}

// Workgroup order that gives each of the 8 XCDs a contiguous range of
// tiles.  Workgroups are dispatched round robin over the XCDs (workgroup k
// runs on XCD k % 8), so without the remap neighbouring sites land on
// different L2 caches.  Bijective for any count n.
__device__ __forceinline__ int xcd_tile(int k, int n) {
    const int q = n >> 3, rem = n & 7;
    const int x = k & 7, j = k >> 3;
    return x * q + (x < rem ? x : rem) + j;
}

}  // namespace stag
