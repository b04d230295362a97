// The RHMC trajectory on the device (Section 2 of the paper: RHMC with a
// multi-step second order minimum norm integrator that splits the action into
// its gauge and fermion parts, several pseudo-fermions, rational
// approximations for the heatbath, the molecular dynamics and the Metropolis
// step; Section 3: one thread per link in the gauge update; Section 4: the
// gauge update in single precision with a double precision reunitarisation,
// the molecular-dynamics inversions in single precision and the Metropolis
// inversions in double precision).
//
// The paper prints none of the formulas; the readings (textbook ones) are:
//   * Wilson plaquette action S_g = beta sum_{x, mu<nu} (1 - Re tr P_munu / 3);
//   * momenta P_mu(x) = sum_a p_a lambda_a / 2 (Gell-Mann lambda_a), kinetic
//     energy (1/2) sum p_a^2, equations of motion dU/dt = i P U;
//   * the force F of an action S on a link is fixed by dS/deps = i tr(T F)
//     for U -> exp(i eps T) U, and a kick moves p_a by h Im tr(lambda_a F) / 2;
//     for any Y, Im tr(lambda_a TA(Y)) = Im tr(lambda_a Y) (TA: traceless
//     anti-Hermitian part), so kicks project U A directly;
//   * gauge force -(beta/3) TA(U_mu(x) A_mu(x)), A the sum of the six staples;
//   * the integrator of Omelyan, Mryglod and Folk (lambda = 0.1931833275037836)
//     on two levels (Sexton and Weingarten): per outer step delta,
//       K_f(l d) G(d/2) K_f((1-2l) d) G(d/2) K_f(l d),
//     G(h): n_g steps of K_g(l e) U(e/2) K_g((1-2l) e) U(e/2) K_g(l e), e = h/n_g.
//     Kicks between two link updates act on the same links, so they are
//     summed and applied once (the fermion force is computed 2 n_md + 1
//     times per trajectory instead of 3 n_md).
//
// Links are the library's float-pair field (one device copy, Section 5): the
// double precision value of each entry is hi + lo with hi its single
// precision rounding.  A link update in single precision reads hi,
// multiplies by exp(i h P) in single precision, then reorthonormalises in
// double precision and stores the result as a new pair, so that the double
// precision inversions of the Metropolis step see an SU(3) field to double
// precision.  A double precision update (for checks against a double
// precision reference) reads hi + lo and computes in double.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "internal.h"
#include "links.h"
#include "solver.h"

namespace stag {

constexpr int kMdBlock = 256;
constexpr double kLambda2MN = 0.1931833275037836;

// ---------------------------------------------------------------- addressing
__device__ __forceinline__ void lex_coords(const Geom &g, int64_t lex, int x[4]) {
    int64_t r = lex;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        x[nu] = (int)(r % g.L[nu]);
        r /= g.L[nu];
    }
}
__device__ __forceinline__ int eo_of(const Geom &g, const int y[4]) {
    return (y[0] >> 1) + g.Lh0 * (y[1] + g.L[1] * (y[2] + g.L[2] * y[3]));
}
__device__ __forceinline__ int parity_of(const int y[4]) { return (y[0] + y[1] + y[2] + y[3]) & 1; }
__device__ __forceinline__ void move(const Geom &g, int y[4], int mu, int d) {
    y[mu] += d;
    if (y[mu] < 0) y[mu] += g.L[mu];
    else if (y[mu] >= g.L[mu]) y[mu] -= g.L[mu];
}
template <typename R, int NR>
__device__ __forceinline__ su3<R> link_at(const void *links, const Geom &g, const int y[4], int mu) {
    return LinkLayout<R, NR>::load(links, g.Vh, parity_of(y) * 4 + mu, eo_of(g, y));
}

// ---------------------------------------------------------------- 3x3 algebra
template <typename R> __device__ __forceinline__ su3<R> mm(const su3<R> &a, const su3<R> &b) {
    su3<R> c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cplx<R> t = cmul(a.e[r][0], b.e[0][k]);
            t = t + cmul(a.e[r][1], b.e[1][k]);
            t = t + cmul(a.e[r][2], b.e[2][k]);
            c.e[r][k] = t;
        }
    return c;
}
// a b^dag
template <typename R> __device__ __forceinline__ su3<R> mm_nd(const su3<R> &a, const su3<R> &b) {
    su3<R> c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cplx<R> t = cmul(a.e[r][0], conj(b.e[k][0]));
            t = t + cmul(a.e[r][1], conj(b.e[k][1]));
            t = t + cmul(a.e[r][2], conj(b.e[k][2]));
            c.e[r][k] = t;
        }
    return c;
}
// a^dag b
template <typename R> __device__ __forceinline__ su3<R> mm_dn(const su3<R> &a, const su3<R> &b) {
    su3<R> c;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cplx<R> t = cmulc(a.e[0][r], b.e[0][k]);
            t = t + cmulc(a.e[1][r], b.e[1][k]);
            t = t + cmulc(a.e[2][r], b.e[2][k]);
            c.e[r][k] = t;
        }
    return c;
}
template <typename R> __device__ __forceinline__ void acc(su3<R> &a, const su3<R> &b) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.e[r][k] = a.e[r][k] + b.e[r][k];
}

// q_a = Im tr(lambda_a Y) / 2 for a = 1..8 (q[0..7]).
template <typename R> __device__ __forceinline__ void algebra_proj(const su3<R> &y, R q[8]) {
    const R h = R(0.5);
    q[0] = h * (y.e[0][1].im + y.e[1][0].im);
    q[1] = h * (y.e[0][1].re - y.e[1][0].re);
    q[2] = h * (y.e[0][0].im - y.e[1][1].im);
    q[3] = h * (y.e[0][2].im + y.e[2][0].im);
    q[4] = h * (y.e[0][2].re - y.e[2][0].re);
    q[5] = h * (y.e[1][2].im + y.e[2][1].im);
    q[6] = h * (y.e[1][2].re - y.e[2][1].re);
    q[7] = R(0.28867513459481288225) * (y.e[0][0].im + y.e[1][1].im - R(2) * y.e[2][2].im);   // 1/(2 sqrt 3)
}

// P = sum_a p_a lambda_a / 2 (traceless Hermitian).
template <typename R> __device__ __forceinline__ su3<R> algebra_matrix(const R p[8]) {
    const R h = R(0.5), r3 = R(0.28867513459481288225);   // 1/(2 sqrt 3)
    su3<R> m;
    m.e[0][0] = {h * p[2] + r3 * p[7], R(0)};
    m.e[1][1] = {-h * p[2] + r3 * p[7], R(0)};
    m.e[2][2] = {R(-2) * r3 * p[7], R(0)};
    m.e[0][1] = {h * p[0], -h * p[1]};
    m.e[1][0] = {h * p[0], h * p[1]};
    m.e[0][2] = {h * p[3], -h * p[4]};
    m.e[2][0] = {h * p[3], h * p[4]};
    m.e[1][2] = {h * p[5], -h * p[6]};
    m.e[2][1] = {h * p[5], h * p[6]};
    return m;
}

// exp(i Q) of a Hermitian Q: scaling and squaring of the Taylor series.
// Q is halved until its Frobenius norm (a bound of the spectral norm) is at
// most 1/2; the series of exp(i Q / 2^s) is summed by Horner's rule to the
// order whose remainder, at most (1/2)^(K+1) / (K+1)!, is below the unit
// roundoff (K = 14 in double, 8 in single precision); then s squarings.
template <typename R> struct ExpOrder;
template <> struct ExpOrder<double> { static constexpr int K = 14; };
template <> struct ExpOrder<float> { static constexpr int K = 8; };
template <typename R> __device__ __forceinline__ su3<R> expi(const su3<R> &q) {
    R n2 = R(0);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) n2 += q.e[r][k].re * q.e[r][k].re + q.e[r][k].im * q.e[r][k].im;
    int s = 0;
    R scale = R(1);
    while (n2 > R(0.25) && s < 60) {   // |Q|_F > 1/2
        n2 *= R(0.25);
        scale *= R(0.5);
        ++s;
    }
    su3<R> a;   // i Q / 2^s
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.e[r][k] = {-scale * q.e[r][k].im, scale * q.e[r][k].re};
    su3<R> e;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) e.e[r][k] = {R(r == k), R(0)};
#pragma unroll
    for (int j = ExpOrder<R>::K; j >= 1; --j) {
        su3<R> t = mm(a, e);
        const R inv = R(1) / R(j);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) e.e[r][k] = {R(r == k) + inv * t.e[r][k].re, inv * t.e[r][k].im};
    }
    for (int j = 0; j < s; ++j) e = mm(e, e);
    return e;
}

// Closest SU(3) matrix in the Gram-Schmidt sense, in double precision: row 0
// normalised, row 1 orthogonalised against it and normalised, row 2 the
// complex conjugate of their cross product.
__device__ __forceinline__ su3<double> reunitarise(const su3<double> &u) {
    su3<double> w;
    double n0 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) n0 += u.e[0][k].re * u.e[0][k].re + u.e[0][k].im * u.e[0][k].im;
    const double i0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int k = 0; k < 3; ++k) w.e[0][k] = i0 * u.e[0][k];
    cplx<double> d = {0.0, 0.0};   // <r0, u1>
#pragma unroll
    for (int k = 0; k < 3; ++k) d = d + cmulc(w.e[0][k], u.e[1][k]);
    double n1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w.e[1][k] = u.e[1][k] - cmul(d, w.e[0][k]);
        n1 += w.e[1][k].re * w.e[1][k].re + w.e[1][k].im * w.e[1][k].im;
    }
    const double i1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int k = 0; k < 3; ++k) w.e[1][k] = i1 * w.e[1][k];
    su3_rebuild_row2(w);
    return w;
}

template <typename R> __device__ __forceinline__ su3<double> to_double(const su3<R> &u) {
    su3<double> d;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) d.e[r][k] = {double(u.e[r][k].re), double(u.e[r][k].im)};
    return d;
}

// ---------------------------------------------------------------- momenta
// Library layout: component a of the momentum of link (parity p, mu, eo i)
// at mom[((p * 4 + mu) * 8 + a) * V/2 + i], in the precision of the
// molecular dynamics.  Canonical layout: (4, V, 8) float64 [mu][lex][a].
template <typename R>
__global__ void __launch_bounds__(kMdBlock) k_mom_pack(Geom g, const double *canon, R *mom) {
    const int64_t vol = 2 * (int64_t)g.Vh;
    const int64_t k = (int64_t)blockIdx.x * kMdBlock + threadIdx.x;
    if (k >= 4 * vol) return;
    const int mu = (int)(k / vol);
    const int64_t lex = k - mu * vol;
    int x[4];
    lex_coords(g, lex, x);
    const int64_t base = (int64_t)(parity_of(x) * 4 + mu) * 8 * g.Vh + (lex >> 1);
#pragma unroll
    for (int a = 0; a < 8; ++a) mom[base + a * (int64_t)g.Vh] = R(canon[k * 8 + a]);
}
template <typename R>
__global__ void __launch_bounds__(kMdBlock) k_mom_unpack(Geom g, const R *mom, double *canon) {
    const int64_t vol = 2 * (int64_t)g.Vh;
    const int64_t k = (int64_t)blockIdx.x * kMdBlock + threadIdx.x;
    if (k >= 4 * vol) return;
    const int mu = (int)(k / vol);
    const int64_t lex = k - mu * vol;
    int x[4];
    lex_coords(g, lex, x);
    const int64_t base = (int64_t)(parity_of(x) * 4 + mu) * 8 * g.Vh + (lex >> 1);
#pragma unroll
    for (int a = 0; a < 8; ++a) canon[k * 8 + a] = double(mom[base + a * (int64_t)g.Vh]);
}

// ---------------------------------------------------------------- gauge force
// One lane per link U_mu(x), (parity, mu) from blockIdx.y.  Staples
//   A = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//                    + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu),
// Y = U_mu(x) A; the force is c TA(Y) with c = -beta/3.  force != null:
// write the force (canonical (4, V, 3, 3) complex128); else kick the momenta
// by h c q(Y).
template <typename R, int NR>
__global__ void __launch_bounds__(kMdBlock) k_gauge_force(Geom g, const void *links, R c, R h, R *mom,
                                                          double2 *force) {
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const int blk = blockIdx.y;   // parity * 4 + mu
    const int p = blk >> 2, mu = blk & 3;
    int x[4];
    site_coords(g, p, i, x);
    su3<R> A;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) A.e[r][k] = {R(0), R(0)};
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int y[4] = {x[0], x[1], x[2], x[3]};
        move(g, y, mu, +1);   // x + mu
        const su3<R> a1 = link_at<R, NR>(links, g, y, nu);
        int z[4] = {x[0], x[1], x[2], x[3]};
        move(g, z, nu, +1);   // x + nu
        const su3<R> a2 = link_at<R, NR>(links, g, z, mu);
        const su3<R> a3 = link_at<R, NR>(links, g, x, nu);
        acc(A, mm_nd(mm_nd(a1, a2), a3));
        move(g, y, nu, -1);   // x + mu - nu
        const su3<R> b1 = link_at<R, NR>(links, g, y, nu);
        int w[4] = {x[0], x[1], x[2], x[3]};
        move(g, w, nu, -1);   // x - nu
        const su3<R> b2 = link_at<R, NR>(links, g, w, mu);
        const su3<R> b3 = link_at<R, NR>(links, g, w, nu);
        // b1^dag b2^dag b3 = (b2 b1)^dag b3
        acc(A, mm_dn(mm(b2, b1), b3));
    }
    const su3<R> u = LinkLayout<R, NR>::load(links, g.Vh, blk, i);
    const su3<R> y = mm(u, A);
    if (force) {
        const R tr = (y.e[0][0].im + y.e[1][1].im + y.e[2][2].im) / R(3);
        const int64_t lex = 2 * (int64_t)i + (x[0] & 1);
        double2 *f = force + ((int64_t)mu * 2 * g.Vh + lex) * 9;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                R re = R(0.5) * (y.e[r][k].re - y.e[k][r].re);
                R im = R(0.5) * (y.e[r][k].im + y.e[k][r].im);
                if (r == k) im -= tr;
                f[r * 3 + k] = make_double2(double(c * re), double(c * im));
            }
    } else {
        R q[8];
        algebra_proj(y, q);
        R *m = mom + (int64_t)blk * 8 * g.Vh + i;
#pragma unroll
        for (int a = 0; a < 8; ++a) m[a * (int64_t)g.Vh] += (h * c) * q[a];
    }
}

// Momentum kick from a force in the canonical (4, V, 3, 3) complex128 layout
// (the pseudo-fermion force): p_a += h Im tr(lambda_a F) / 2.
template <typename R>
__global__ void __launch_bounds__(kMdBlock) k_force_kick(Geom g, const double2 *force, R h, R *mom) {
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const int blk = blockIdx.y;
    const int p = blk >> 2, mu = blk & 3;
    int x[4];
    site_coords(g, p, i, x);
    const int64_t lex = 2 * (int64_t)i + (x[0] & 1);
    const double2 *f = force + ((int64_t)mu * 2 * g.Vh + lex) * 9;
    su3<R> y;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double2 v = f[e];
        y.e[e / 3][e % 3] = {R(v.x), R(v.y)};
    }
    R q[8];
    algebra_proj(y, q);
    R *m = mom + (int64_t)blk * 8 * g.Vh + i;
#pragma unroll
    for (int a = 0; a < 8; ++a) m[a * (int64_t)g.Vh] += h * q[a];
}

// ---------------------------------------------------------------- link update
// U <- exp(i h P) U in precision R, then reorthonormalised in double
// precision and stored as a float pair (NP = kHiLo + 2 or kHiLo + 3).
template <typename R, int NP>
__global__ void __launch_bounds__(kMdBlock) k_link_update(Geom g, void *links, const R *mom, R h) {
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    if (i >= g.Vh) return;
    const int blk = blockIdx.y;
    R pa[8];
    const R *m = mom + (int64_t)blk * 8 * g.Vh + i;
#pragma unroll
    for (int a = 0; a < 8; ++a) pa[a] = h * m[a * (int64_t)g.Vh];
    const su3<R> e = expi(algebra_matrix(pa));
    su3<double> un;
    if constexpr (sizeof(R) == sizeof(double)) {
        const su3<double> u = LinkLayout<double, NP>::load(links, g.Vh, blk, i);
        un = reunitarise(mm(e, u));
    } else {
        const su3<float> u = LinkLayout<float, NP - kHiLo>::load(links, g.Vh, blk, i);
        un = reunitarise(to_double(mm(e, u)));
    }
    LinkLayout<double, NP>::store(links, g.Vh, blk, i, un);
}

// ---------------------------------------------------------------- energies
// Sum over the six plaquettes of site x of Re tr P_munu(x), one partial per block.
template <int NR>
__global__ void __launch_bounds__(kMdBlock) k_plaquette(Geom g, const void *links, double *partial) {
    __shared__ double red[kMdBlock / kWave];
    const int64_t lex = (int64_t)blockIdx.x * kMdBlock + threadIdx.x;
    double s = 0.0;
    if (lex < 2 * (int64_t)g.Vh) {
        int x[4];
        lex_coords(g, lex, x);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            const su3<double> umu = link_at<double, NR>(links, g, x, mu);
            int y[4] = {x[0], x[1], x[2], x[3]};
            move(g, y, mu, +1);
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu) {
                const su3<double> a = mm(umu, link_at<double, NR>(links, g, y, nu));
                int z[4] = {x[0], x[1], x[2], x[3]};
                move(g, z, nu, +1);
                const su3<double> b = mm_nd(a, link_at<double, NR>(links, g, z, mu));
                const su3<double> c = mm_nd(b, link_at<double, NR>(links, g, x, nu));
                s += c.e[0][0].re + c.e[1][1].re + c.e[2][2].re;
            }
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// sum_a p_a^2 over the library momenta, one partial per block.
template <typename R>
__global__ void __launch_bounds__(kMdBlock) k_mom_norm2(const R *mom, int64_t n, double *partial) {
    __shared__ double red[kMdBlock / kWave];
    double s = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kMdBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kMdBlock) {
        const double v = double(mom[k]);
        s += v * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------- host side
static bool pair_format(int nrow) { return nrow == kHiLo + 2 || nrow == kHiLo + 3; }

template <typename R, int NR>
static hipError_t gauge_force_nr(const stag_lattice *lat, const void *links, double c, double h, void *mom,
                                 double2 *force, hipStream_t s) {
    const dim3 grid((lat->Vh + kMdBlock - 1) / kMdBlock, 8), block(kMdBlock);
    hipLaunchKernelGGL((k_gauge_force<R, NR>), grid, block, 0, s, lat->g, links, R(c), R(h), static_cast<R *>(mom),
                       force);
    return hipGetLastError();
}

// Gauge force (force != null) or gauge kick (mom != null) in precision dbl.
static hipError_t launch_gauge_force(const stag_lattice *lat, bool dbl, double beta, double h, void *mom,
                                     double2 *force, hipStream_t s) {
    const double c = -beta / 3.0;
    const int nrow = lat->nrow;
    if (dbl) {
        const void *l = lat->links64;
        switch (nrow) {
            case 1: return gauge_force_nr<double, 1>(lat, l, c, h, mom, force, s);
            case 2: return gauge_force_nr<double, 2>(lat, l, c, h, mom, force, s);
            case 3: return gauge_force_nr<double, 3>(lat, l, c, h, mom, force, s);
            case kHiLo + 2: return gauge_force_nr<double, kHiLo + 2>(lat, l, c, h, mom, force, s);
            case kHiLo + 3: return gauge_force_nr<double, kHiLo + 3>(lat, l, c, h, mom, force, s);
            default: return hipErrorInvalidValue;
        }
    }
    const void *l = lat->links32;
    switch (nrow_single(nrow)) {
        case 1: return gauge_force_nr<float, 1>(lat, l, c, h, mom, force, s);
        case 2: return gauge_force_nr<float, 2>(lat, l, c, h, mom, force, s);
        case 3: return gauge_force_nr<float, 3>(lat, l, c, h, mom, force, s);
        default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_link_update(stag_lattice *lat, bool dbl, const void *mom, double h, hipStream_t s) {
    const dim3 grid((lat->Vh + kMdBlock - 1) / kMdBlock, 8), block(kMdBlock);
    if (lat->nrow == kHiLo + 3) {
        if (dbl)
            hipLaunchKernelGGL((k_link_update<double, kHiLo + 3>), grid, block, 0, s, lat->g, lat->links64,
                               static_cast<const double *>(mom), h);
        else
            hipLaunchKernelGGL((k_link_update<float, kHiLo + 3>), grid, block, 0, s, lat->g, lat->links64,
                               static_cast<const float *>(mom), float(h));
    } else if (lat->nrow == kHiLo + 2) {
        if (dbl)
            hipLaunchKernelGGL((k_link_update<double, kHiLo + 2>), grid, block, 0, s, lat->g, lat->links64,
                               static_cast<const double *>(mom), h);
        else
            hipLaunchKernelGGL((k_link_update<float, kHiLo + 2>), grid, block, 0, s, lat->g, lat->links64,
                               static_cast<const float *>(mom), float(h));
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t launch_force_kick(const stag_lattice *lat, bool dbl, const void *force, double h, void *mom,
                                    hipStream_t s) {
    const dim3 grid((lat->Vh + kMdBlock - 1) / kMdBlock, 8), block(kMdBlock);
    if (dbl)
        hipLaunchKernelGGL((k_force_kick<double>), grid, block, 0, s, lat->g, static_cast<const double2 *>(force), h,
                           static_cast<double *>(mom));
    else
        hipLaunchKernelGGL((k_force_kick<float>), grid, block, 0, s, lat->g, static_cast<const double2 *>(force),
                           float(h), static_cast<float *>(mom));
    return hipGetLastError();
}

static int mom_grid(const stag_lattice *lat) { return (int)((8 * lat->V + kMdBlock - 1) / kMdBlock); }

static hipError_t launch_mom_pack(const stag_lattice *lat, bool dbl, const double *canon, void *mom, hipStream_t s) {
    const int64_t n = 4 * lat->V;
    const dim3 grid((unsigned)((n + kMdBlock - 1) / kMdBlock)), block(kMdBlock);
    if (dbl) hipLaunchKernelGGL((k_mom_pack<double>), grid, block, 0, s, lat->g, canon, static_cast<double *>(mom));
    else hipLaunchKernelGGL((k_mom_pack<float>), grid, block, 0, s, lat->g, canon, static_cast<float *>(mom));
    return hipGetLastError();
}
static hipError_t launch_mom_unpack(const stag_lattice *lat, bool dbl, const void *mom, double *canon, hipStream_t s) {
    const int64_t n = 4 * lat->V;
    const dim3 grid((unsigned)((n + kMdBlock - 1) / kMdBlock)), block(kMdBlock);
    if (dbl)
        hipLaunchKernelGGL((k_mom_unpack<double>), grid, block, 0, s, lat->g, static_cast<const double *>(mom), canon);
    else
        hipLaunchKernelGGL((k_mom_unpack<float>), grid, block, 0, s, lat->g, static_cast<const float *>(mom), canon);
    return hipGetLastError();
}

// Deterministic host sum of device partials (fixed order).
static stag_status sum_partials(const double *part, int n, hipStream_t s, double *out) {
    std::vector<double> h(n);
    STAG_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    STAG_HIP(hipStreamSynchronize(s));
    double t = 0.0;
    for (double v : h) t += v;
    *out = t;
    return STAG_OK;
}

stag_status gauge_action(stag_lattice *lat, double beta, double *out, hipStream_t s) {
    const int nb = (int)((lat->V + kMdBlock - 1) / kMdBlock);
    void *part = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_PART, sizeof(double) * nb, &part));
    const dim3 grid(nb), block(kMdBlock);
    double *pp = static_cast<double *>(part);
    switch (lat->nrow) {
        case 1: hipLaunchKernelGGL((k_plaquette<1>), grid, block, 0, s, lat->g, lat->links64, pp); break;
        case 2: hipLaunchKernelGGL((k_plaquette<2>), grid, block, 0, s, lat->g, lat->links64, pp); break;
        case 3: hipLaunchKernelGGL((k_plaquette<3>), grid, block, 0, s, lat->g, lat->links64, pp); break;
        case kHiLo + 2: hipLaunchKernelGGL((k_plaquette<kHiLo + 2>), grid, block, 0, s, lat->g, lat->links64, pp); break;
        case kHiLo + 3: hipLaunchKernelGGL((k_plaquette<kHiLo + 3>), grid, block, 0, s, lat->g, lat->links64, pp); break;
        default: return invalid("unknown link format");
    }
    STAG_HIP(hipGetLastError());
    double tr = 0.0;
    STAG_TRY(sum_partials(pp, nb, s, &tr));
    *out = beta * (6.0 * (double)lat->V - tr / 3.0);
    return STAG_OK;
}

// |v|^2 of a double precision library vector, summed in a fixed order.
static stag_status vec_norm2(stag_lattice *lat, const void *v, double *out, hipStream_t s) {
    const int64_t ne = 3 * (int64_t)lat->Vh;
    const int grid = blas_grid(ne);
    void *part = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_PART, sizeof(double) * grid, &part));
    STAG_HIP(launch_norm2(true, v, ne, static_cast<double *>(part), grid, s));
    return sum_partials(static_cast<double *>(part), grid, s, out);
}

static stag_status kinetic_energy(stag_lattice *lat, bool dbl, const void *mom, double *out, hipStream_t s) {
    const int nb = 1024;
    void *part = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_PART, sizeof(double) * nb, &part));
    const int64_t n = 32 * lat->V;
    if (dbl)
        hipLaunchKernelGGL((k_mom_norm2<double>), dim3(nb), dim3(kMdBlock), 0, s, static_cast<const double *>(mom), n,
                           static_cast<double *>(part));
    else
        hipLaunchKernelGGL((k_mom_norm2<float>), dim3(nb), dim3(kMdBlock), 0, s, static_cast<const float *>(mom), n,
                           static_cast<double *>(part));
    STAG_HIP(hipGetLastError());
    double t = 0.0;
    STAG_TRY(sum_partials(static_cast<double *>(part), nb, s, &t));
    *out = 0.5 * t;
    return STAG_OK;
}

stag_status multishift_cg(stag_lattice *lat, double mass, const double *shifts, int n, const void *src,
                          void *const *sols, double tol, int max_iter, stag_prec prec, stag_cg_stats *stats,
                          hipStream_t s);
stag_status fermion_force(stag_lattice *lat, int n, const double *alphas, const void *const *x, void *force,
                          hipStream_t s);
stag_status rational_apply(stag_lattice *lat, double mass, double alpha0, const double *alphas, const double *shifts,
                           int n, const void *src, void *out, double tol, int max_iter, double *dot,
                           stag_cg_stats *stats, hipStream_t s);

// The molecular dynamics from the library momenta `mom` (precision dbl).
static stag_status md_run(stag_lattice *lat, const stag_rhmc_params *prm, void *mom, bool dbl, int n_pf,
                          const void *const *phis, stag_rhmc_info *info, hipStream_t s) {
    const int nr = prm->rat_md.n;
    const int64_t vb = vec_bytes(lat, true);
    // several pseudo-fermion fields: their solves in one batched call and one
    // force over all their solutions (the force is linear in them), while
    // the solutions fit the force's limit of shifts
    const bool batch = n_pf > 1 && n_pf * nr <= kMaxShifts;
    const int nsol = batch ? n_pf * nr : nr;
    void *sols_buf = nullptr, *force = nullptr;
    if (n_pf > 0) {
        STAG_TRY(ws_get(lat, WS_MD_SOLS, (size_t)(nsol > 0 ? nsol : 1) * vb, &sols_buf));
        STAG_TRY(ws_get(lat, WS_MD_FORCE, (size_t)576 * lat->V, &force));
    }
    std::vector<void *> sols(nsol > 0 ? nsol : 1);
    for (int k = 0; k < nsol; ++k) sols[k] = static_cast<char *>(sols_buf) + k * vb;
    std::vector<double> alphas_all;
    for (int k = 0; batch && k < n_pf; ++k)
        alphas_all.insert(alphas_all.end(), prm->rat_md.alpha, prm->rat_md.alpha + nr);
    const stag_prec solve_prec = dbl ? STAG_F64 : STAG_F32;
    double pend_g = 0.0, pend_f = 0.0;
    auto flush = [&]() -> stag_status {
        if (pend_f != 0.0 && batch) {
            std::vector<BSpec> spec(n_pf);
            for (int k = 0; k < n_pf; ++k)
                spec[k] = {lat, prm->mass, nr, prm->rat_md.shift, phis[k], sols.data() + k * nr, false};
            BOptions opt{};
            opt.tol = prm->tol_md;
            opt.max_iter = prm->max_iter;
            opt.dbl = dbl;
            opt.reliable_every = 0;
            std::vector<stag_cg_stats> st(n_pf);
            const stag_status rc = batched_solve(spec.data(), n_pf, opt, false, st.data(), s);
            for (int k = 0; k < n_pf; ++k) info->md_iters += st[k].iters;
            if (rc != STAG_OK) return rc;
            STAG_TRY(fermion_force(lat, nsol, alphas_all.data(), sols.data(), force, s));
            STAG_HIP(launch_force_kick(lat, dbl, force, pend_f, mom, s));
            info->fermion_forces += 1;
        } else if (pend_f != 0.0 && n_pf > 0) {
            for (int k = 0; k < n_pf; ++k) {
                stag_cg_stats st;
                std::memset(&st, 0, sizeof(st));
                const stag_status rc = multishift_cg(lat, prm->mass, prm->rat_md.shift, nr, phis[k], sols.data(),
                                                     prm->tol_md, prm->max_iter, solve_prec, &st, s);
                info->md_iters += st.iters;
                if (rc != STAG_OK) return rc;
                STAG_TRY(fermion_force(lat, nr, prm->rat_md.alpha, sols.data(), force, s));
                STAG_HIP(launch_force_kick(lat, dbl, force, pend_f, mom, s));
            }
            info->fermion_forces += 1;
        }
        if (pend_g != 0.0) {
            STAG_HIP(launch_gauge_force(lat, dbl, prm->beta, pend_g, mom, nullptr, s));
            info->gauge_forces += 1;
        }
        pend_g = pend_f = 0.0;
        return STAG_OK;
    };
    auto kick_g = [&](double h) { pend_g += h; };
    auto kick_f = [&](double h) { pend_f += h; };
    auto drift = [&](double h) -> stag_status {
        STAG_TRY(flush());
        STAG_HIP(launch_link_update(lat, dbl, mom, h, s));
        return STAG_OK;
    };
    const double lam = kLambda2MN;
    const double delta = prm->tau / prm->n_md;
    auto gauge_part = [&](double h) -> stag_status {
        const double d = h / prm->n_g;
        for (int j = 0; j < prm->n_g; ++j) {
            kick_g(lam * d);
            STAG_TRY(drift(0.5 * d));
            kick_g((1.0 - 2.0 * lam) * d);
            STAG_TRY(drift(0.5 * d));
            kick_g(lam * d);
        }
        return STAG_OK;
    };
    for (int k = 0; k < prm->n_md; ++k) {
        kick_f(lam * delta);
        STAG_TRY(gauge_part(0.5 * delta));
        kick_f((1.0 - 2.0 * lam) * delta);
        STAG_TRY(gauge_part(0.5 * delta));
        kick_f(lam * delta);
    }
    return flush();
}

static stag_status check_rational(const stag_rational &r, const char *what) {
    if (r.n < 1 || r.n > STAG_MAX_SHIFTS) return invalid(std::string(what) + ": n must be in [1, 64]");
    if (!std::isfinite(r.alpha0)) return invalid(std::string(what) + ": alpha0 must be finite");
    for (int i = 0; i < r.n; ++i)
        if (!(r.shift[i] >= 0) || !std::isfinite(r.shift[i]) || !std::isfinite(r.alpha[i]))
            return invalid(std::string(what) + ": shifts must be >= 0 and weights finite");
    return STAG_OK;
}

stag_status check_md_params(const stag_lattice *lat, const stag_rhmc_params *prm, int n_pf, bool trajectory) {
    if (!prm) return invalid("null parameters");
    if (!pair_format(lat->nrow))
        return invalid("the molecular dynamics updates the links in place: set them as STAG_LINK18_PAIRS or "
                       "STAG_LINK12_PAIRS");
    if (!(prm->beta >= 0) || !std::isfinite(prm->beta)) return invalid("beta must be >= 0 and finite");
    if (!(prm->mass > 0) || !std::isfinite(prm->mass)) return invalid("mass must be > 0");
    if (!(prm->tau > 0) || !std::isfinite(prm->tau)) return invalid("tau must be > 0");
    if (prm->n_md < 1 || prm->n_g < 1) return invalid("n_md and n_g must be >= 1");
    if (prm->md_prec != STAG_F64 && prm->md_prec != STAG_F32) return invalid("md_prec must be STAG_F64 or STAG_F32");
    if (n_pf < 0 || n_pf > STAG_MAX_PSEUDOFERMIONS) return invalid("n_pf must be in [0, 16]");
    if (n_pf > 0) {
        if (!(prm->tol_md > 0) || !std::isfinite(prm->tol_md)) return invalid("tol_md must be > 0");
        if (prm->max_iter < 1) return invalid("max_iter must be >= 1");
        STAG_TRY(check_rational(prm->rat_md, "rat_md"));
    }
    if (trajectory && n_pf > 0) {
        if (!(prm->tol_act > 0) || !std::isfinite(prm->tol_act)) return invalid("tol_act must be > 0");
        STAG_TRY(check_rational(prm->rat_hb, "rat_hb"));
        STAG_TRY(check_rational(prm->rat_act, "rat_act"));
    }
    return STAG_OK;
}

stag_status md_integrate(stag_lattice *lat, const stag_rhmc_params *prm, double *mom_canon, int n_pf,
                         const void *const *phis, stag_rhmc_info *info, hipStream_t s) {
    TraceRange tr("molecular dynamics");
    const auto t0 = std::chrono::steady_clock::now();
    const bool dbl = prm->md_prec == STAG_F64;
    void *mom = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_MOM, (size_t)32 * lat->V * (dbl ? 8 : 4), &mom));
    STAG_HIP(launch_mom_pack(lat, dbl, mom_canon, mom, s));
    STAG_TRY(md_run(lat, prm, mom, dbl, n_pf, phis, info, s));
    STAG_HIP(launch_mom_unpack(lat, dbl, mom, mom_canon, s));
    STAG_HIP(hipStreamSynchronize(s));
    info->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return STAG_OK;
}

stag_status rhmc_trajectory(stag_lattice *lat, const stag_rhmc_params *prm, double *mom_canon, int n_pf,
                            const void *const *xis, double u, stag_rhmc_info *info, hipStream_t s) {
    TraceRange tr("RHMC trajectory");
    const auto t0 = std::chrono::steady_clock::now();
    const bool dbl = prm->md_prec == STAG_F64;
    const int64_t vb = vec_bytes(lat, true);
    const size_t lb = (size_t)link_field_bytes(true, lat->nrow, lat->Vh);
    void *bak = nullptr, *phi_buf = nullptr, *mom = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_LINKS, lb, &bak));
    STAG_TRY(ws_get(lat, WS_MD_MOM, (size_t)32 * lat->V * (dbl ? 8 : 4), &mom));
    if (n_pf > 0) STAG_TRY(ws_get(lat, WS_MD_PHI, (size_t)n_pf * vb, &phi_buf));
    STAG_HIP(hipMemcpyAsync(bak, lat->links64, lb, hipMemcpyDeviceToDevice, s));
    // heatbath: phi_k = r_hb(M) xi_k; the fermion action at the start is |xi_k|^2
    // (several fields: one batched application of the rational function to
    // all of them, every link read once per up to eight fields)
    std::vector<const void *> phis(n_pf > 0 ? n_pf : 1);
    std::vector<void *> phi_out(n_pf > 0 ? n_pf : 1);
    for (int k = 0; k < n_pf; ++k) phis[k] = phi_out[k] = static_cast<char *>(phi_buf) + k * vb;
    std::vector<stag_cg_stats> rst(n_pf > 0 ? n_pf : 1);
    double sf0 = 0.0;
    if (n_pf > 1) {
        TraceRange trk("heatbath");
        STAG_TRY(rational_apply_multi(lat, prm->mass, prm->rat_hb.alpha0, prm->rat_hb.alpha, prm->rat_hb.shift,
                                      prm->rat_hb.n, xis, phi_out.data(), n_pf, prm->tol_act, prm->max_iter, nullptr,
                                      rst.data(), s));
        for (int k = 0; k < n_pf; ++k) info->action_iters += rst[k].iters;
    }
    for (int k = 0; k < n_pf; ++k) {
        if (n_pf == 1) {
            TraceRange trk("heatbath");
            double dot = 0.0;
            std::memset(&rst[0], 0, sizeof(rst[0]));
            STAG_TRY(rational_apply(lat, prm->mass, prm->rat_hb.alpha0, prm->rat_hb.alpha, prm->rat_hb.shift,
                                    prm->rat_hb.n, xis[k], phi_out[k], prm->tol_act, prm->max_iter, &dot, &rst[0], s));
            info->action_iters += rst[0].iters;
        }
        double x2 = 0.0;
        STAG_TRY(vec_norm2(lat, xis[k], &x2, s));
        sf0 += x2;
    }
    STAG_HIP(launch_mom_pack(lat, dbl, mom_canon, mom, s));
    double k0 = 0.0, sg0 = 0.0;
    STAG_TRY(kinetic_energy(lat, dbl, mom, &k0, s));
    STAG_TRY(gauge_action(lat, prm->beta, &sg0, s));
    {
        TraceRange trm("molecular dynamics");
        STAG_TRY(md_run(lat, prm, mom, dbl, n_pf, phis.data(), info, s));
    }
    double k1 = 0.0, sg1 = 0.0, sf1 = 0.0;
    STAG_TRY(kinetic_energy(lat, dbl, mom, &k1, s));
    STAG_TRY(gauge_action(lat, prm->beta, &sg1, s));
    void *scratch_out = nullptr;
    if (n_pf > 0) STAG_TRY(ws_get(lat, WS_MD_OUT, (size_t)n_pf * vb, &scratch_out));
    if (n_pf > 1) {
        TraceRange trk("Metropolis action");
        std::vector<void *> outs(n_pf);
        for (int k = 0; k < n_pf; ++k) outs[k] = static_cast<char *>(scratch_out) + k * vb;
        std::vector<double> dots(n_pf, 0.0);
        STAG_TRY(rational_apply_multi(lat, prm->mass, prm->rat_act.alpha0, prm->rat_act.alpha, prm->rat_act.shift,
                                      prm->rat_act.n, phis.data(), outs.data(), n_pf, prm->tol_act, prm->max_iter,
                                      dots.data(), rst.data(), s));
        for (int k = 0; k < n_pf; ++k) {
            info->action_iters += rst[k].iters;
            sf1 += dots[k];
        }
    } else if (n_pf == 1) {
        TraceRange trk("Metropolis action");
        double dot = 0.0;
        std::memset(&rst[0], 0, sizeof(rst[0]));
        STAG_TRY(rational_apply(lat, prm->mass, prm->rat_act.alpha0, prm->rat_act.alpha, prm->rat_act.shift,
                                prm->rat_act.n, phis[0], scratch_out, prm->tol_act, prm->max_iter, &dot, &rst[0], s));
        info->action_iters += rst[0].iters;
        sf1 += dot;
    }
    STAG_HIP(launch_mom_unpack(lat, dbl, mom, mom_canon, s));
    info->H0[0] = k0;
    info->H0[1] = sg0;
    info->H0[2] = sf0;
    info->H1[0] = k1;
    info->H1[1] = sg1;
    info->H1[2] = sf1;
    info->dH = (k1 + sg1 + sf1) - (k0 + sg0 + sf0);
    info->accepted = (u < 0.0 || u < std::exp(-info->dH)) ? 1 : 0;
    if (!info->accepted) STAG_HIP(hipMemcpyAsync(lat->links64, bak, lb, hipMemcpyDeviceToDevice, s));
    STAG_HIP(hipStreamSynchronize(s));
    info->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stag_log(1, "rhmc_trajectory: dH %.6g (K %.6g, S_g %.6g, S_f %.6g -> %.6g, %.6g, %.6g), %s, %d fermion forces, "
             "%d MD iterations, %.4f s", info->dH, k0, sg0, sf0, k1, sg1, sf1, info->accepted ? "accepted" : "rejected",
             info->fermion_forces, info->md_iters, info->seconds);
    return STAG_OK;
}

// ---------------------------------------------------------------- single steps (checks, tools)
stag_status gauge_force_out(stag_lattice *lat, double beta, void *force, bool dbl, hipStream_t s) {
    STAG_HIP(launch_gauge_force(lat, dbl, beta, 0.0, nullptr, static_cast<double2 *>(force), s));
    return STAG_OK;
}

stag_status mom_step(stag_lattice *lat, double *mom_canon, int kind, double beta, const void *force, double h,
                     bool dbl, hipStream_t s) {
    void *mom = nullptr;
    STAG_TRY(ws_get(lat, WS_MD_MOM, (size_t)32 * lat->V * (dbl ? 8 : 4), &mom));
    STAG_HIP(launch_mom_pack(lat, dbl, mom_canon, mom, s));
    if (kind == 0) STAG_HIP(launch_gauge_force(lat, dbl, beta, h, mom, nullptr, s));
    else if (kind == 1) STAG_HIP(launch_force_kick(lat, dbl, force, h, mom, s));
    else STAG_HIP(launch_link_update(lat, dbl, mom, h, s));
    if (kind != 2) STAG_HIP(launch_mom_unpack(lat, dbl, mom, mom_canon, s));
    return STAG_OK;
}

}  // namespace stag
