/*
 * FP64 CPU oracle for the even/odd-preconditioned unimproved staggered
 * operator and the multi-shift conjugate gradient of
 *   C. Bonati, G. Cossu, M. D'Elia, A. Di Giacomo,
 *   "Staggered fermions simulations on GPUs" (Lattice 2010).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP path, and the HIP path never loads
 * it.  It is deliberately plain: loops over lexicographic sites, C99
 * complex arithmetic in double precision, no blocking, no fusion.
 *
 * Conventions (the paper names the method -- unimproved staggered fermions
 * with even/odd preconditioning, Section 2, solved by CG and by Krylov
 * solvers for shifted systems, Section 6 -- but prints no formula; these
 * are the textbook Kogut-Susskind definitions):
 *   dims L = (L0,L1,L2,L3) = (x,y,z,t), every L_mu even and >= 2.
 *   lex(x) = x0 + L0*(x1 + L1*(x2 + L2*x3)); parity = (x0+x1+x2+x3) mod 2;
 *   eo(x)  = lex(x) / 2 (one index per parity; needs L0 even).
 *   eta_mu(x) = (-1)^(x0+...+x_{mu-1}), so eta_0 = 1.
 *   s_mu(x) = -1 if mu = 3, x3 = L3-1 and the time direction is
 *             antiperiodic (fermion boundary condition), else +1.
 *   (D psi)(x) = 1/2 sum_mu eta_mu(x) [ s_mu(x) U_mu(x) psi(x+mu)
 *                                      - s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   D_eo = D from odd sites to even sites, D_oe from even to odd.
 *   M = m^2 - D_eo D_oe on even sites (Hermitian, positive definite).
 * Gauge links U_mu(x) are stored as links[((mu*V + lex)*3 + row)*3 + col].
 * Colour vectors on one parity are vec[eo*3 + colour].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int L[4];
    int64_t V, Vh;
    int antiperiodic_t;
} geo;

static int geo_init(geo *g, const int *dims, int antiperiodic_t)
{
    g->V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || (dims[mu] & 1)) return -1;
        g->L[mu] = dims[mu];
        g->V *= dims[mu];
    }
    g->Vh = g->V / 2;
    g->antiperiodic_t = antiperiodic_t;
    return 0;
}

static void lex_to_coord(const geo *g, int64_t lex, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(lex % g->L[mu]);
        lex /= g->L[mu];
    }
}

static int64_t coord_to_lex(const geo *g, const int x[4])
{
    return x[0] + (int64_t)g->L[0] * (x[1] + (int64_t)g->L[1] * (x[2] + (int64_t)g->L[2] * x[3]));
}

static int site_parity(const int x[4]) { return (x[0] + x[1] + x[2] + x[3]) & 1; }

static double eta(int mu, const int x[4])
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += x[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* Sign carried by the link U_mu(x): the antiperiodic time boundary. */
static double bc_sign(const geo *g, int mu, const int x[4])
{
    return (g->antiperiodic_t && mu == 3 && x[3] == g->L[3] - 1) ? -1.0 : 1.0;
}

/* y = x + dir * mu-hat, periodic wrap. */
static void hop(const geo *g, const int x[4], int mu, int dir, int y[4])
{
    for (int nu = 0; nu < 4; ++nu) y[nu] = x[nu];
    y[mu] = (x[mu] + dir + g->L[mu]) % g->L[mu];
}

static const cplx *link_at(const geo *g, const cplx *U, int mu, int64_t lex)
{
    return U + ((int64_t)mu * g->V + lex) * 9;
}

/* acc += c * U v */
static void add_mul(cplx acc[3], double c, const cplx *U, const cplx *v)
{
    for (int a = 0; a < 3; ++a) {
        cplx s = 0;
        for (int b = 0; b < 3; ++b) s += U[a * 3 + b] * v[b];
        acc[a] += c * s;
    }
}

/* acc += c * U^dag v */
static void add_mul_dag(cplx acc[3], double c, const cplx *U, const cplx *v)
{
    for (int a = 0; a < 3; ++a) {
        cplx s = 0;
        for (int b = 0; b < 3; ++b) s += conj(U[b * 3 + a]) * v[b];
        acc[a] += c * s;
    }
}

/* One site of the hopping term; fetch(lex) returns the colour vector at lex. */
static void dhop_site(const geo *g, const cplx *U, const int x[4],
                      const cplx *in, int eo_in, cplx out[3])
{
    cplx acc[3] = {0, 0, 0};
    for (int mu = 0; mu < 4; ++mu) {
        int y[4], z[4];
        double e = eta(mu, x);
        hop(g, x, mu, +1, y);
        hop(g, x, mu, -1, z);
        int64_t ly = coord_to_lex(g, y), lz = coord_to_lex(g, z);
        const cplx *vy = in + (eo_in ? (ly >> 1) : ly) * 3;
        const cplx *vz = in + (eo_in ? (lz >> 1) : lz) * 3;
        add_mul(acc, e * bc_sign(g, mu, x), link_at(g, U, mu, coord_to_lex(g, x)), vy);
        add_mul_dag(acc, -e * bc_sign(g, mu, z), link_at(g, U, mu, lz), vz);
    }
    for (int a = 0; a < 3; ++a) out[a] = 0.5 * acc[a];
}

/* Full-lattice hopping term D on (V,3) lexicographic vectors. */
int orc_dhop_full(const int *dims, int antiperiodic_t, const cplx *U,
                  const cplx *in, cplx *out)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int x[4];
        lex_to_coord(&g, lex, x);
        dhop_site(&g, U, x, in, 0, out + lex * 3);
    }
    return 0;
}

/* Half hopping term: out on parity out_parity (eo-indexed, (V/2,3)),
 * in on the opposite parity.  out_parity = 0 gives D_eo, 1 gives D_oe. */
int orc_dslash_eo(const int *dims, int antiperiodic_t, const cplx *U,
                  int out_parity, const cplx *in, cplx *out)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t) || (out_parity & ~1)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int x[4];
        lex_to_coord(&g, lex, x);
        if (site_parity(x) != out_parity) continue;
        dhop_site(&g, U, x, in, 1, out + (lex >> 1) * 3);
    }
    return 0;
}

/* out = (m^2 + shift) in - D_eo D_oe in, on even sites. */
int orc_normal_op(const int *dims, int antiperiodic_t, const cplx *U,
                  double mass, double shift, const cplx *in, cplx *out)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t)) return -1;
    int64_t n = g.Vh * 3;
    cplx *t = malloc(sizeof(cplx) * n);
    cplx *s = malloc(sizeof(cplx) * n);
    if (!t || !s) { free(t); free(s); return -2; }
    orc_dslash_eo(dims, antiperiodic_t, U, 1, in, t);
    orc_dslash_eo(dims, antiperiodic_t, U, 0, t, s);
    double c = mass * mass + shift;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = c * in[k] - s[k];
    free(t);
    free(s);
    return 0;
}

/* Neighbour, coordinate and sign tables of one lattice.
 *   nbr[(p*8 + d)*Vh + i]  : eo index of neighbour d of site (p, i);
 *                            d = 0..3 is x + mu-hat, d = 4..7 is x - mu-hat.
 *   coord[(p*Vh + i)*4 + mu] : coordinates of site (p, i).
 *   sign[(p*8 + d)*Vh + i] : the +-1 that multiplies hop d at site (p, i):
 *                            eta_mu(x) s_mu(x) forward, eta_mu(x) s_mu(x-mu)
 *                            backward (the 1/2 and the minus of the backward
 *                            hop are not included). */
int orc_tables(const int *dims, int antiperiodic_t, int32_t *nbr,
               int32_t *coord, int32_t *sign)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t)) return -1;
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int x[4];
        lex_to_coord(&g, lex, x);
        int p = site_parity(x);
        int64_t i = lex >> 1;
        for (int mu = 0; mu < 4; ++mu) {
            int y[4], z[4];
            hop(&g, x, mu, +1, y);
            hop(&g, x, mu, -1, z);
            nbr[(p * 8 + mu) * g.Vh + i] = (int32_t)(coord_to_lex(&g, y) >> 1);
            nbr[(p * 8 + 4 + mu) * g.Vh + i] = (int32_t)(coord_to_lex(&g, z) >> 1);
            sign[(p * 8 + mu) * g.Vh + i] = (int32_t)(eta(mu, x) * bc_sign(&g, mu, x));
            sign[(p * 8 + 4 + mu) * g.Vh + i] = (int32_t)(eta(mu, x) * bc_sign(&g, mu, z));
            coord[(p * g.Vh + i) * 4 + mu] = x[mu];
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- BLAS-1 */
/* Serial sums keep the oracle's results independent of the thread count. */

static double re_dot(const cplx *a, const cplx *b, int64_t n)
{
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += creal(conj(a[k]) * b[k]);
    return s;
}

static double norm2(const cplx *a, int64_t n) { return re_dot(a, a, n); }

/* ||b - (M + shift) x|| / ||b|| */
double orc_true_residual(const int *dims, int antiperiodic_t, const cplx *U,
                         double mass, double shift, const cplx *b, const cplx *x)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t)) return -1.0;
    int64_t n = g.Vh * 3;
    cplx *ax = malloc(sizeof(cplx) * n);
    if (!ax) return -1.0;
    orc_normal_op(dims, antiperiodic_t, U, mass, shift, x, ax);
    double r2 = 0.0, b2 = norm2(b, n);
    for (int64_t k = 0; k < n; ++k) {
        cplx d = b[k] - ax[k];
        r2 += creal(conj(d) * d);
    }
    free(ax);
    return b2 > 0 ? sqrt(r2 / b2) : sqrt(r2);
}

/* Return codes shared by the solvers below. */
enum { ORC_OK = 0, ORC_NOCONV = 1, ORC_BREAKDOWN = 2, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

/* Conjugate gradient for (M + shift) x = b starting from the x passed in
 * (Section 6: CG is the Krylov solver of choice for staggered fermions).
 * Stops when the iterated residual satisfies ||r|| <= tol ||b||. */
int orc_cg(const int *dims, int antiperiodic_t, const cplx *U, double mass,
           double shift, const cplx *b, cplx *x, double tol, int max_iter,
           int *iters, double *resid_iter, double *resid_true)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t) || !(mass > 0) || !(shift >= 0) || !(tol > 0))
        return ORC_EINVAL;
    int64_t n = g.Vh * 3;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    if (!r || !p || !q) { free(r); free(p); free(q); return ORC_ENOMEM; }
    int status = ORC_NOCONV, k = 0;
    double bnorm = sqrt(norm2(b, n));
    orc_normal_op(dims, antiperiodic_t, U, mass, shift, x, q);
    for (int64_t j = 0; j < n; ++j) { r[j] = b[j] - q[j]; p[j] = r[j]; }
    double rho = norm2(r, n);
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        status = ORC_OK;
    } else if (sqrt(rho) <= tol * bnorm) {
        status = ORC_OK;
    } else {
        for (k = 0; k < max_iter;) {
            orc_normal_op(dims, antiperiodic_t, U, mass, shift, p, q);
            double pq = re_dot(p, q, n);
            if (!(pq > 0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
            double alpha = rho / pq;
            for (int64_t j = 0; j < n; ++j) { x[j] += alpha * p[j]; r[j] -= alpha * q[j]; }
            double rho_new = norm2(r, n);
            ++k;
            if (sqrt(rho_new) <= tol * bnorm) { rho = rho_new; status = ORC_OK; break; }
            double beta = rho_new / rho;
            for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
            rho = rho_new;
        }
    }
    if (iters) *iters = k;
    if (resid_iter) *resid_iter = bnorm > 0 ? sqrt(rho) / bnorm : 0.0;
    if (resid_true) *resid_true = orc_true_residual(dims, antiperiodic_t, U, mass, shift, b, x);
    free(r); free(p); free(q);
    return status;
}

/* Multi-shift CG (Jegerlehner, hep-lat/9612014; cited in Section 6 as the
 * Krylov solver for shifted systems, which must start from x = 0).
 * Solves (M + shifts[i]) x_i = b for every i with one Krylov space built on
 * the smallest shift sigma_0.  With s_i = shifts[i] - sigma_0, alpha_{-1} = 1,
 * beta_{-1} = 0 and zeta_i^{-1} = zeta_i^0 = 1, iteration k performs
 *   q = (M + sigma_0) p,  alpha_k = rho_k / Re<p,q>
 *   zeta_i^{k+1} = zeta_i^k zeta_i^{k-1} alpha_{k-1} /
 *        [ alpha_k beta_{k-1} (zeta_i^{k-1} - zeta_i^k)
 *          + zeta_i^{k-1} alpha_{k-1} (1 + s_i alpha_k) ]
 *   r -= alpha_k q,  rho_{k+1} = <r,r>,  beta_k = rho_{k+1} / rho_k
 *   alpha_k^i = alpha_k zeta_i^{k+1}/zeta_i^k,  beta_k^i = beta_k (zeta_i^{k+1}/zeta_i^k)^2
 *   x_i += alpha_k^i p_i,  p_i = zeta_i^{k+1} r + beta_k^i p_i
 * and shift i is frozen once |zeta_i^{k+1}| sqrt(rho_{k+1}) <= tol ||b||.
 * The shifted residuals are r_i = zeta_i r.  x is (n_shifts, V/2, 3). */
int orc_multishift_cg(const int *dims, int antiperiodic_t, const cplx *U,
                      double mass, int n_shifts, const double *shifts,
                      const cplx *b, cplx *x, double tol, int max_iter,
                      int *iters, int *iters_shift, double *resid_iter,
                      double *resid_true)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t) || !(mass > 0) || !(tol > 0) || n_shifts < 1)
        return ORC_EINVAL;
    int base = 0;
    for (int i = 0; i < n_shifts; ++i) {
        if (!(shifts[i] >= 0)) return ORC_EINVAL;
        if (shifts[i] < shifts[base]) base = i;
    }
    int64_t n = g.Vh * 3;
    cplx *r = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    cplx *ps = malloc(sizeof(cplx) * n * n_shifts);
    double *z = malloc(sizeof(double) * 3 * n_shifts);
    int *active = malloc(sizeof(int) * n_shifts);
    if (!r || !q || !ps || !z || !active) {
        free(r); free(q); free(ps); free(z); free(active);
        return ORC_ENOMEM;
    }
    double *zeta = z, *zeta_prev = z + n_shifts, *zeta_next = z + 2 * n_shifts;
    double sigma0 = shifts[base];

    memset(x, 0, sizeof(cplx) * n * n_shifts);
    memcpy(r, b, sizeof(cplx) * n);
    for (int i = 0; i < n_shifts; ++i) {
        memcpy(ps + i * n, b, sizeof(cplx) * n);
        zeta[i] = zeta_prev[i] = 1.0;
        active[i] = 1;
        if (iters_shift) iters_shift[i] = 0;
        if (resid_iter) resid_iter[i] = 1.0;
    }
    double rho = norm2(r, n), bnorm = sqrt(rho);
    double alpha_prev = 1.0, beta_prev = 0.0;
    int status = ORC_NOCONV, k = 0;
    cplx *p = ps + base * n; /* the base direction is p_base (zeta = 1) */

    if (bnorm == 0.0) {
        status = ORC_OK;
        for (int i = 0; i < n_shifts; ++i) if (resid_iter) resid_iter[i] = 0.0;
    } else {
        for (k = 0; k < max_iter;) {
            orc_normal_op(dims, antiperiodic_t, U, mass, sigma0, p, q);
            double pq = re_dot(p, q, n);
            if (!(pq > 0) || !isfinite(pq)) { status = ORC_BREAKDOWN; break; }
            double alpha = rho / pq;
            for (int i = 0; i < n_shifts; ++i) {
                if (!active[i]) continue;
                double s = shifts[i] - sigma0;
                double den = alpha * beta_prev * (zeta_prev[i] - zeta[i])
                           + zeta_prev[i] * alpha_prev * (1.0 + s * alpha);
                zeta_next[i] = zeta[i] * zeta_prev[i] * alpha_prev / den;
            }
            for (int64_t j = 0; j < n; ++j) r[j] -= alpha * q[j];
            double rho_new = norm2(r, n);
            double beta = rho_new / rho;
            ++k;
            int any_active = 0;
            for (int i = 0; i < n_shifts; ++i) {
                if (!active[i]) continue;
                double ratio = zeta_next[i] / zeta[i];
                double ai = alpha * ratio, bi = beta * ratio * ratio;
                cplx *xi = x + i * n, *pi = ps + i * n;
                for (int64_t j = 0; j < n; ++j) {
                    xi[j] += ai * pi[j];
                    pi[j] = zeta_next[i] * r[j] + bi * pi[j];
                }
                double res = fabs(zeta_next[i]) * sqrt(rho_new) / bnorm;
                if (resid_iter) resid_iter[i] = res;
                if (res <= tol) {
                    active[i] = 0;
                    if (iters_shift) iters_shift[i] = k;
                } else {
                    any_active = 1;
                }
            }
            /* Other shifts still running need the base direction even if
             * the base system itself is frozen. */
            if (any_active && !active[base]) {
                for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
            }
            for (int i = 0; i < n_shifts; ++i) {
                zeta_prev[i] = zeta[i];
                zeta[i] = zeta_next[i];
            }
            alpha_prev = alpha;
            beta_prev = beta;
            rho = rho_new;
            if (!any_active) { status = ORC_OK; break; }
        }
    }
    for (int i = 0; i < n_shifts; ++i) {
        if (iters_shift && active[i]) iters_shift[i] = k;
        if (resid_true)
            resid_true[i] = orc_true_residual(dims, antiperiodic_t, U, mass, shifts[i], b, x + i * n);
    }
    if (iters) *iters = k;
    free(r); free(q); free(ps); free(z); free(active);
    return status;
}

/* Pseudo-fermion force of the RHMC (Section 2: the molecular dynamics needs
 * the derivative of the fermion action, built from the multi-shift
 * solutions; Section 4 runs it in single precision).  The paper prints no
 * formula; this is the derivative written out from the operator above.
 *
 * For the action S = sum_i alpha_i <phi, (M + sigma_i)^-1 phi> with
 * X_i = (M + sigma_i)^-1 phi (even sites) and M = m^2 + D_eo D_eo^dag
 * (D_oe = -D_eo^dag), a variation dU of the links changes S by
 *   dS = -sum_i alpha_i 2 Re <X_i, dD_eo Y_i>,   Y_i = D_eo^dag X_i = -D_oe X_i.
 * Link U_mu(x) enters D_eo forward at an even x, with X_i(x) and
 * Y_i(x+mu), and backward (as U^dag) at an odd x, with X_i(x+mu) and
 * Y_i(x).  Collecting dS = Re sum tr(dU_mu(x) W_mu(x)):
 *   x even: W = sum_i (-2 alpha_i) (1/2) eta s  Y_i(x+mu) X_i(x)^dag
 *   x odd : W = sum_i (-2 alpha_i) (-1/2) eta s X_i(x+mu) Y_i(x)^dag
 * with eta s = eta_mu(x) s_mu(x), the sign the link carries.  For a move
 * U -> exp(i eps T) U with T Hermitian and traceless, dS/deps = i tr(T F)
 * where F_mu(x) = TA(U_mu(x) W_mu(x)), TA(A) = (A - A^dag)/2 - tr(A - A^dag)/6.
 *
 * x: n_shifts even vectors (V/2,3) one after another; force: (4,V,3,3)
 * in the layout of the links.  Returns 0, or -1 for bad dims. */
int orc_fermion_force(const int *dims, int antiperiodic_t, const cplx *U, int n_shifts,
                      const double *alphas, const cplx *x, cplx *force)
{
    geo g;
    if (geo_init(&g, dims, antiperiodic_t) || n_shifts < 0) return -1;
    const int64_t n = g.Vh * 3;
    cplx *y = malloc(sizeof(cplx) * (n_shifts > 0 ? n_shifts : 1) * n);
    if (!y) return -2;
    for (int i = 0; i < n_shifts; ++i) {
        orc_dslash_eo(dims, antiperiodic_t, U, 1, x + i * n, y + i * n);
        for (int64_t k = 0; k < n; ++k) y[i * n + k] = -y[i * n + k];
    }
#pragma omp parallel for schedule(static)
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int c[4];
        lex_to_coord(&g, lex, c);
        const int odd = site_parity(c);
        for (int mu = 0; mu < 4; ++mu) {
            int up[4];
            hop(&g, c, mu, +1, up);
            const int64_t here = lex >> 1, there = coord_to_lex(&g, up) >> 1;
            const double es = eta(mu, c) * bc_sign(&g, mu, c);
            cplx W[9] = {0};
            for (int i = 0; i < n_shifts; ++i) {
                const cplx *xi = x + i * n, *yi = y + i * n;
                /* even x: W += k Y(x+mu) X(x)^dag; odd x: W += k X(x+mu) Y(x)^dag */
                const cplx *left = odd ? xi + there * 3 : yi + there * 3;
                const cplx *right = odd ? yi + here * 3 : xi + here * 3;
                const double k = -2.0 * alphas[i] * (odd ? -0.5 : 0.5) * es;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) W[a * 3 + b] += k * left[a] * conj(right[b]);
            }
            const cplx *u = link_at(&g, U, mu, lex);
            cplx A[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    cplx s = 0;
                    for (int e = 0; e < 3; ++e) s += u[a * 3 + e] * W[e * 3 + b];
                    A[a * 3 + b] = s;
                }
            cplx tr = 0;
            for (int a = 0; a < 3; ++a) tr += A[a * 4] - conj(A[a * 4]);
            cplx *f = force + ((int64_t)mu * g.V + lex) * 9;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    f[a * 3 + b] = 0.5 * (A[a * 3 + b] - conj(A[b * 3 + a])) - (a == b ? tr / 6.0 : 0);
        }
    }
    free(y);
    return 0;
}
