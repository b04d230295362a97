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

// ---------------------------------------------------------------- other powers
// Best relative approximation of y^(-p), 0 < p < 1, on [1, B] of type
// (n-1, n), R(y) = sum_i a_i / (y + c_i), by Remez's exchange algorithm with
// Newton steps on the 2n + 1 equations R(y_j) y_j^p - 1 = s_j E at reference
// points y_j of alternating sign s_j (unknowns a_i, ln c_i, E), continued in
// p from Zolotarev's solution at p = 1/2 in steps of at most 0.02.  Long
// double throughout.
namespace {

typedef long double ld;

struct RatFn {
    std::vector<ld> a, lc;   // residues, log of the pole offsets
};

ld rel_err(ld y, ld p, const RatFn &r) {
    ld acc = 0.0L;
    for (size_t i = 0; i < r.a.size(); ++i) acc += r.a[i] / (y + std::exp(r.lc[i]));
    return acc * std::pow(y, p) - 1.0L;
}

// Local extrema of the error on a grid in t = ln y, refined by golden-section
// search, reduced to an alternating sequence (largest |e| per sign run).
std::vector<ld> alternating_extrema(ld p, ld B, const RatFn &r, int ngrid, std::vector<ld> *vals) {
    const ld T = std::log(B);
    std::vector<ld> t(ngrid + 1), e(ngrid + 1);
    for (int k = 0; k <= ngrid; ++k) {
        t[k] = T * k / ngrid;
        e[k] = rel_err(std::exp(t[k]), p, r);
    }
    std::vector<ld> pos, val;
    auto push = [&](ld tt, ld ee) {
        if (!val.empty() && ((ee > 0) == (val.back() > 0))) {
            if (std::fabs(ee) > std::fabs(val.back())) {
                pos.back() = tt;
                val.back() = ee;
            }
        } else {
            pos.push_back(tt);
            val.push_back(ee);
        }
    };
    push(t[0], e[0]);
    const ld gr = 0.5L * (std::sqrt(5.0L) - 1.0L);
    for (int k = 1; k < ngrid; ++k) {
        const bool mx = e[k] >= e[k - 1] && e[k] >= e[k + 1];
        const bool mn = e[k] <= e[k - 1] && e[k] <= e[k + 1];
        if (!mx && !mn) continue;
        const ld sg = mx ? 1.0L : -1.0L;
        ld a = t[k - 1], b = t[k + 1];
        ld x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        ld f1 = sg * rel_err(std::exp(x1), p, r), f2 = sg * rel_err(std::exp(x2), p, r);
        for (int it = 0; it < 80 && b - a > 1e-15L * (1.0L + T); ++it) {
            if (f1 > f2) {
                b = x2;
                x2 = x1;
                f2 = f1;
                x1 = b - gr * (b - a);
                f1 = sg * rel_err(std::exp(x1), p, r);
            } else {
                a = x1;
                x1 = x2;
                f1 = f2;
                x2 = a + gr * (b - a);
                f2 = sg * rel_err(std::exp(x2), p, r);
            }
        }
        push(f1 > f2 ? x1 : x2, sg * std::max(f1, f2));
    }
    push(t[ngrid], e[ngrid]);
    if (vals) *vals = val;
    return pos;
}

// Below this relative error the coefficients, stored in double precision,
// cannot be improved further.
constexpr ld kRoundingFloor = 1e-12L;

// Newton steps on the reference equations; false if the system is singular.
bool remez_newton(ld p, const std::vector<ld> &y, const std::vector<ld> &sg, RatFn &r, ld &E) {
    const int n = (int)r.a.size(), m = 2 * n + 1;
    std::vector<ld> F(m), J((size_t)m * m), du(m);
    auto residual = [&](const RatFn &q, ld e, std::vector<ld> &out) {
        ld worst = 0.0L;
        for (int j = 0; j < m; ++j) {
            out[j] = rel_err(y[j], p, q) - sg[j] * e;
            worst = std::max(worst, std::fabs(out[j]));
        }
        return worst;
    };
    ld f0 = residual(r, E, F);
    for (int it = 0; it < 40 && f0 > 1e-18L; ++it) {
        for (int j = 0; j < m; ++j) {
            const ld w = std::pow(y[j], p);
            for (int i = 0; i < n; ++i) {
                const ld c = std::exp(r.lc[i]), d = y[j] + c;
                J[(size_t)j * m + i] = w / d;
                J[(size_t)j * m + n + i] = -w * r.a[i] * c / (d * d);
            }
            J[(size_t)j * m + 2 * n] = -sg[j];
            du[j] = -F[j];
        }
        // Gaussian elimination with partial pivoting
        for (int c = 0; c < m; ++c) {
            int piv = c;
            for (int k = c + 1; k < m; ++k)
                if (std::fabs(J[(size_t)k * m + c]) > std::fabs(J[(size_t)piv * m + c])) piv = k;
            if (!(std::fabs(J[(size_t)piv * m + c]) > 0.0L)) return false;
            if (piv != c) {
                for (int k = 0; k < m; ++k) std::swap(J[(size_t)c * m + k], J[(size_t)piv * m + k]);
                std::swap(du[c], du[piv]);
            }
            for (int k = c + 1; k < m; ++k) {
                const ld f = J[(size_t)k * m + c] / J[(size_t)c * m + c];
                if (f == 0.0L) continue;
                for (int q = c; q < m; ++q) J[(size_t)k * m + q] -= f * J[(size_t)c * m + q];
                du[k] -= f * du[c];
            }
        }
        for (int c = m - 1; c >= 0; --c) {
            ld acc = du[c];
            for (int q = c + 1; q < m; ++q) acc -= J[(size_t)c * m + q] * du[q];
            du[c] = acc / J[(size_t)c * m + c];
        }
        // damped update
        ld lam = 1.0L;
        RatFn trial = r;
        ld Et = E, f1 = 0.0L;
        std::vector<ld> Ft(m);
        for (;;) {
            for (int i = 0; i < n; ++i) {
                trial.a[i] = r.a[i] + lam * du[i];
                trial.lc[i] = r.lc[i] + lam * du[n + i];
            }
            Et = E + lam * du[2 * n];
            f1 = residual(trial, Et, Ft);
            if ((std::isfinite((double)f1) && f1 < f0) || lam < 1e-4L) break;
            lam *= 0.5L;
        }
        if (!std::isfinite((double)f1)) return false;
        r = trial;
        E = Et;
        F = Ft;
        f0 = f1;
    }
    return true;
}

}  // namespace

stag_status rational_power(double power, double lo, double hi, int n, double *alpha0, double *alphas, double *shifts,
                           double *delta_out) {
    if (power == -0.5 || power == 0.5) return zolotarev(power < 0 ? -1 : 1, lo, hi, n, alpha0, alphas, shifts, delta_out);
    const ld B = (ld)hi / (ld)lo;
    const ld p_target = power < 0 ? -(ld)power : 1.0L - (ld)power;   // approximate y^(-p)
    // start: Zolotarev's y^(-1/2) on [1, B]
    std::vector<double> za(n), zs(n);
    double z0 = 0.0, zd = 0.0;
    STAG_TRY(zolotarev(-1, 1.0, (double)B, n, &z0, za.data(), zs.data(), &zd));
    RatFn r;
    r.a.assign(za.begin(), za.end());
    for (int i = 0; i < n; ++i) r.lc.push_back(std::log((ld)zs[i]));
    const int m = 2 * n + 1, ngrid = 300 * m;
    std::vector<ld> vals;
    std::vector<ld> pos = alternating_extrema(0.5L, B, r, ngrid, &vals);
    if ((int)pos.size() < m) return invalid("approximation of this degree is below double precision; use fewer poles");
    while ((int)pos.size() > m) {
        if (std::fabs(vals.front()) < std::fabs(vals.back())) {
            pos.erase(pos.begin());
            vals.erase(vals.begin());
        } else {
            pos.pop_back();
            vals.pop_back();
        }
    }
    std::vector<ld> y(m), sg(m);
    for (int j = 0; j < m; ++j) {
        y[j] = std::exp(pos[j]);
        sg[j] = vals[j] > 0 ? 1.0L : -1.0L;
    }
    ld E = std::fabs(vals[0]);
    const int nsteps = std::max(1, (int)std::ceil(std::fabs((double)(p_target - 0.5L)) / 0.02));
    ld emax = 0.0L;
    for (int step = 1; step <= nsteps; ++step) {
        const ld p = 0.5L + (p_target - 0.5L) * step / nsteps;
        bool ok = false;
        for (int it = 0; it < 30; ++it) {
            if (!remez_newton(p, y, sg, r, E)) break;
            pos = alternating_extrema(p, B, r, ngrid, &vals);
            ld vall = 0.0L;
            for (ld v : vals) vall = std::max(vall, std::fabs(v));
            if (vall < kRoundingFloor) {
                // the error is at the level of double precision rounding of
                // the coefficients: no alternation left to resolve
                emax = vall;
                ok = true;
                break;
            }
            while ((int)pos.size() > m) {
                if (std::fabs(vals.front()) < std::fabs(vals.back())) {
                    pos.erase(pos.begin());
                    vals.erase(vals.begin());
                } else {
                    pos.pop_back();
                    vals.pop_back();
                }
            }
            if ((int)pos.size() < m) break;
            ld vmin = 1e300L, vmax = 0.0L;
            for (int j = 0; j < m; ++j) {
                y[j] = std::exp(pos[j]);
                sg[j] = vals[j] > 0 ? 1.0L : -1.0L;
                vmin = std::min(vmin, std::fabs(vals[j]));
                vmax = std::max(vmax, std::fabs(vals[j]));
            }
            emax = vmax;
            if (vmin > (1.0L - 1e-5L) * vmax) {
                ok = true;
                break;
            }
        }
        if (!ok) return invalid("Remez iteration did not converge; use fewer poles or a narrower range");
    }
    // back to x = lo y: x^(-p) = lo^(-p) y^(-p) ~ sum a_i lo^(1-p) / (x + lo c_i)
    const ld scale = std::pow((ld)lo, 1.0L - p_target);
    ld a0 = 0.0L;
    for (int i = 0; i < n; ++i) {
        const ld al = r.a[i] * scale, sh = (ld)lo * std::exp(r.lc[i]);
        if (power < 0) {
            alphas[i] = (double)al;
        } else {   // x^(1-p) = x * x^(-p)
            a0 += al;
            alphas[i] = (double)(-al * sh);
        }
        shifts[i] = (double)sh;
    }
    *alpha0 = (double)a0;
    if (delta_out) *delta_out = (double)emax;
    return STAG_OK;
}

}  // namespace stag
