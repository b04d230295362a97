// Pseudo-fermion force of the RHMC from the multi-shift solutions (Section 2:
// the molecular dynamics integrates the force of the rational action, built
// from the same shifted solves as the heatbath and the Metropolis step).
//
// For S = sum_i alpha_i <phi, (M + sigma_i)^-1 phi>, X_i = (M + sigma_i)^-1 phi
// on even sites and Z_i = D_oe X_i on odd sites (M = m^2 - D_eo D_oe with
// D_oe = -D_eo^dag), a variation dU of the links changes S by
// Re sum tr(dU_mu(x) W_mu(x)) with
//   x even: W = sum_i alpha_i eta s          Z_i(x+mu) X_i(x)^dag
//   x odd : W = sum_i alpha_i (-eta s)       X_i(x+mu) Z_i(x)^dag
// (eta s = eta_mu(x) s_mu(x), the sign carried by the link U_mu(x)).  The
// force is F_mu(x) = TA(U_mu(x) W_mu(x)), the traceless anti-Hermitian part:
// moving U -> exp(i eps T) U changes S at the rate i tr(T F).
//
// One lane per lattice site, in lex order (even and odd sites alternate in a
// wave, so the force stores of one direction are contiguous).  The lane
// holds the four directions' W in registers: per shift it reads its own
// vector once and the vectors of its four forward neighbours, and each link
// once at the end.  The output goes to the (4, V, 3, 3) complex layout in
// which links are handed to the library.  Bandwidth-bound (about 70 flops
// per shift and link against 96 bytes read), so no matrix cores.
#include "internal.h"
#include "links.h"
#include "solver.h"

namespace stag {

constexpr int kForceBlock = 256;

struct ForceArgs {
    Geom g;
    int n;                        // shifts
    const void *links;            // packed double precision links
    const void *x[kMaxShifts];    // even-site solutions
    const void *z;                // odd-site Z_i = D_oe X_i, one vector after another
    double alpha[kMaxShifts];
    double2 *force;               // (4, V, 3, 3) complex
};

template <int NROW>
__global__ void __launch_bounds__(kForceBlock) k_force(ForceArgs a) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t lex = (int64_t)tile * kForceBlock + threadIdx.x;
    const int vh = a.g.Vh;
    const int64_t V = 2 * (int64_t)vh;
    if (lex >= V) return;
    int x[4];
    {
        int64_t r = lex;
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            x[nu] = (int)(r % a.g.L[nu]);
            r /= a.g.L[nu];
        }
    }
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int i = (int)(lex >> 1);
    int j[4];
    double es[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        j[mu] = site_nbr(a.g, i, x, mu, +1);
        es[mu] = p ? -double(fwd_sign(a.g, x, mu)) : double(fwd_sign(a.g, x, mu));
    }
    const int64_t zstride = 3 * (int64_t)vh;   // double2 entries per odd vector
    const double2 *zb = static_cast<const double2 *>(a.z);
    cplx<double> W[4][3][3];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) W[mu][r][c] = {0.0, 0.0};
#pragma unroll 1
    for (int s = 0; s < a.n; ++s) {
        // even x: W += Z(x+mu) X(x)^dag; odd x: W -= X(x+mu) Z(x)^dag (the sign is in es)
        const void *zs = zb + s * zstride;
        const vec3<double> o = load_vec<double>(p ? zs : a.x[s], vh, i);
        vec3<double> l[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) l[mu] = load_vec<double>(p ? a.x[s] : zs, vh, j[mu]);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const double k = a.alpha[s] * es[mu];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const cplx<double> kl = {k * l[mu].c[r].re, k * l[mu].c[r].im};
#pragma unroll
                for (int c = 0; c < 3; ++c) W[mu][r][c] = W[mu][r][c] + cmul(kl, conj(o.c[c]));
            }
        }
    }
    // fully unrolled, so W stays in registers (a dynamic index puts it in scratch)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const su3<double> u = LinkLayout<double, NROW>::load(a.links, vh, p * 4 + mu, i);
        cplx<double> A[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cplx<double> t = cmul(u.e[r][0], W[mu][0][c]);
                t = t + cmul(u.e[r][1], W[mu][1][c]);
                t = t + cmul(u.e[r][2], W[mu][2][c]);
                A[r][c] = t;
            }
        // TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6; tr(A - A^dag) = 2i Im tr A
        const double tr_im = (A[0][0].im + A[1][1].im + A[2][2].im) / 3.0;
        double2 *f = a.force + ((int64_t)mu * V + lex) * 9;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double re = 0.5 * (A[r][c].re - A[c][r].re);
                double im = 0.5 * (A[r][c].im + A[c][r].im);
                if (r == c) im -= tr_im;
                f[r * 3 + c] = make_double2(re, im);
            }
    }
}

template <int NROW>
static hipError_t launch_force_nrow(const ForceArgs &a, hipStream_t s) {
    const dim3 grid((2 * a.g.Vh + kForceBlock - 1) / kForceBlock), block(kForceBlock);
    hipLaunchKernelGGL((k_force<NROW>), grid, block, 0, s, a);
    return hipGetLastError();
}

static hipError_t launch_force(int nrow, const ForceArgs &a, hipStream_t s) {
    switch (nrow) {
        case 3: return launch_force_nrow<3>(a, s);
        case 2: return launch_force_nrow<2>(a, s);
        case 1: return launch_force_nrow<1>(a, s);
        case kHiLo + 2: return launch_force_nrow<kHiLo + 2>(a, s);
        case kHiLo + 3: return launch_force_nrow<kHiLo + 3>(a, s);
        default: return hipErrorInvalidValue;
    }
}

// Launch shape of the multi-right-hand-side D_oe that makes the Z_i.
constexpr int kZBlock = 128;
constexpr int kZRpt = 8;

// Z_i = D_oe X_i for every shift into a work buffer (eight vectors per
// launch), then the force launch.  The caller has validated the arguments.
stag_status fermion_force(stag_lattice *lat, int n, const double *alphas, const void *const *x, void *force,
                          hipStream_t s) {
    TraceRange tr("pseudo-fermion force");
    void *z = nullptr;
    const int64_t vb = vec_bytes(lat, true);
    STAG_TRY(ws_get(lat, WS_FORCE, (size_t)(n > 0 ? n : 1) * vb, &z));
    void *zs[kMaxShifts];
    for (int i = 0; i < n; ++i) zs[i] = static_cast<char *>(z) + i * vb;
    STAG_HIP(launch_dslash_oe_multi(lat, n, x, zs, kZBlock, kZRpt, s));
    ForceArgs a{};
    a.g = lat->g;
    a.n = n;
    a.links = lat->links64;
    a.z = z;
    a.force = static_cast<double2 *>(force);
    for (int i = 0; i < n; ++i) {
        a.x[i] = x[i];
        a.alpha[i] = alphas[i];
    }
    STAG_HIP(launch_force(lat->nrow, a, s));
    return STAG_OK;
}

}  // namespace stag
