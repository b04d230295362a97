// Zolotarev's optimal rational approximation of x^(-1/2) (and, through
// x^(1/2) = x * x^(-1/2), of x^(1/2)) in partial fractions, for the rational
// functions of the RHMC (Section 2 of the paper: rational approximations for
// the Metropolis step and the molecular dynamics).  Host code.
//
// On [1, B] the best type (n-1, n) approximation of y^(-1/2) in the relative
// sense is
//   R(y) = M prod_{l=1}^{n-1} (y + c_{2l}) / prod_{l=1}^{n} (y + c_{2l-1}),
//   c_l = sn^2(u_l; k') / cn^2(u_l; k'),  u_l = l K(k') / (2n),  k'^2 = 1 - 1/B,
// with sn, cn Jacobi elliptic functions and K the complete elliptic integral
// (Zolotarev; Akhiezer's "Elements of the theory of elliptic functions").
// M is fixed here numerically so that the relative error sqrt(y) R(y) - 1
// takes its extreme values +delta and -delta; the error then alternates
// 2n + 1 times, which certifies optimality.  K uses the arithmetic-geometric
// mean, sn and cn the descending Landen (AGM) method of Abramowitz and
// Stegun, 16.4.
#include <cmath>
#include <vector>

#include "internal.h"

namespace stag {

namespace {

// The elliptic functions run in long double (64-bit significand on x86-64):
// for k'^2 = 1 - 1/B close to 1 the AGM recursion of sn loses a few digits
// where cn is small, and the high-degree approximations resolve errors of
// order 1e-13.

// K(m) for parameter m = k^2, given m1 = 1 - m exactly.
long double ellip_k(long double m1) {
    long double a = 1.0L, b = std::sqrt(m1);
    for (int it = 0; it < 64 && std::fabs(a - b) > 1e-19L * a; ++it) {
        const long double an = 0.5L * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return 3.14159265358979323846264338327950288L / (2.0L * a);
}

// sn(u | m), cn(u | m) by the AGM scale (m1 = 1 - m).
void ellip_sncn(long double u, long double m, long double m1, long double *sn, long double *cn) {
    long double a[64], c[64];
    a[0] = 1.0L;
    long double b = std::sqrt(m1);
    c[0] = std::sqrt(m);
    int N = 0;
    while (N < 62 && std::fabs(c[N]) > 1e-21L) {
        a[N + 1] = 0.5L * (a[N] + b);
        c[N + 1] = 0.5L * (a[N] - b);
        b = std::sqrt(a[N] * b);
        ++N;
    }
    long double phi = std::ldexp(a[N] * u, N);
    for (int i = N; i >= 1; --i) phi = 0.5L * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
    *sn = std::sin(phi);
    *cn = std::cos(phi);
}

// sqrt(y) prod (y + num) / prod (y + den), written as a product of O(1) factors
double zolo_g(double y, const std::vector<double> &num, const std::vector<double> &den) {
    double g = std::sqrt(y) / (y + den.back());
    for (size_t l = 0; l < num.size(); ++l) g *= (y + num[l]) / (y + den[l]);
    return g;
}

}  // namespace

stag_status zolotarev(int power, double lo, double hi, int n, double *alpha0, double *alphas, double *shifts,
                      double *delta_out) {
    const long double B = (long double)hi / (long double)lo;
    const long double m1 = 1.0L / B, m = 1.0L - m1;
    const long double Kp = ellip_k(m1);
    std::vector<double> c(2 * n);   // c[l], l = 1 .. 2n-1
    for (int l = 1; l < 2 * n; ++l) {
        long double sn, cn;
        ellip_sncn(l * Kp / (2.0L * n), m, m1, &sn, &cn);
        c[l] = (double)((sn * sn) / (cn * cn));
    }
    std::vector<double> num, den;
    for (int l = 1; l <= n - 1; ++l) num.push_back(c[2 * l]);
    for (int l = 1; l <= n; ++l) den.push_back(c[2 * l - 1]);

    // extreme values of g over [1, B]: endpoints and interior local extrema
    // (grid in t = ln y, each bracket refined by golden-section search)
    const int ng = 64 * (2 * n + 1);
    const double T = std::log((double)B);
    auto gt = [&](double t) { return zolo_g(std::exp(t), num, den); };
    std::vector<double> gv(ng + 1);
    for (int k = 0; k <= ng; ++k) gv[k] = gt(T * k / ng);
    double gmax = std::max(gv[0], gv[ng]), gmin = std::min(gv[0], gv[ng]);
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int k = 1; k < ng; ++k) {
        const bool is_max = gv[k] >= gv[k - 1] && gv[k] >= gv[k + 1];
        const bool is_min = gv[k] <= gv[k - 1] && gv[k] <= gv[k + 1];
        if (!is_max && !is_min) continue;
        const double sg = is_max ? 1.0 : -1.0;   // maximise sg * g
        double a = T * (k - 1) / ng, b = T * (k + 1) / ng;
        double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        double f1 = sg * gt(x1), f2 = sg * gt(x2);
        for (int it = 0; it < 200 && b - a > 1e-14 * (1.0 + T); ++it) {
            if (f1 > f2) {
                b = x2;
                x2 = x1;
                f2 = f1;
                x1 = b - gr * (b - a);
                f1 = sg * gt(x1);
            } else {
                a = x1;
                x1 = x2;
                f1 = f2;
                x2 = a + gr * (b - a);
                f2 = sg * gt(x2);
            }
        }
        const double v = sg * std::max(f1, f2);
        gmax = std::max(gmax, v);
        gmin = std::min(gmin, v);
    }
    const double M = 2.0 / (gmax + gmin);
    const double delta = (gmax - gmin) / (gmax + gmin);

    // partial fractions R(y) = sum_l res_l / (y + den_l), then x = lo y
    const double sl = std::sqrt(lo);
    double a0 = 0.0;
    for (int l = 0; l < n; ++l) {
        double res = M;
        for (int k = 0; k < n - 1; ++k) res *= num[k] - den[l];
        for (int k = 0; k < n; ++k)
            if (k != l) res /= den[k] - den[l];
        const double al = res * sl, sh = lo * den[l];
        if (power < 0) {
            alphas[l] = al;
        } else {   // x^(1/2) = x * x^(-1/2): al x / (x + sh) = al - al sh / (x + sh)
            a0 += al;
            alphas[l] = -al * sh;
        }
        shifts[l] = sh;
    }
    *alpha0 = a0;
    if (delta_out) *delta_out = delta;
    return STAG_OK;
}

}  // namespace stag
