/*
 * FP64 oracle of the learned gauge-equivariant preconditioner P(r).
 *
 * TEST INFRASTRUCTURE (see orc.c).  Plain loops over lexicographic sites,
 * C99 complex arithmetic in double precision, written from the definition
 * below; no code is shared with the HIP network kernels.
 *
 * Network (8 channels, two parallel-transport hopping layers, a projection):
 *   hops      (T_{+mu} psi)(x) = eta_mu(x) s_mu(x)      U_mu(x)        psi(x+mu)
 *             (T_{-mu} psi)(x) = eta_mu(x) s_mu(x-mu)   U_mu(x-mu)^dag psi(x-mu)
 *             hop index d = mu (forward) or 4 + mu (backward); T_d^dag = T_{d+4 mod 8}.
 *   input     r on even sites (one channel).
 *   layer 1   phi1[c](x) = w1s[c] r(x)                               x even
 *             phi1[c](y) = sum_d w1h[c][d] (T_d r)(y)                y odd
 *   layer 2   f_k(x), x even, k = 0..71: f_c' = phi1[c'](x) (c' < 8),
 *             f_{8+8d+c'} = (T_d phi1[c'])(x);
 *             phi2[c](x) = sum_k W2[c][k] f_k(x)
 *   output    P(r)(x) = sum_c wout[c] phi2[c](x), x even.
 * The maps commute with gauge transformations (weights do not touch
 * colour), and P is linear in r.
 *
 * Parameters are one complex array theta of NET_NPARAM entries:
 *   [0, 8)       w1s[c]
 *   [8, 72)      w1h[c][d]      at 8 + 8c + d
 *   [72, 648)    W2[c][k]       at 72 + 72c + k
 *   [648, 656)   wout[c]        at 648 + c
 *
 * Gradients: for a real objective L = Re sum_x <g(x), P(r)(x)> the oracle
 * returns grad[j] = dL/dRe(theta_j) + i dL/dIm(theta_j).  The loss
 * L = ||P(b) - x||^2 corresponds to g = 2 (P(b) - x).
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { NC = 8, NK = 72, NET_W1S = 0, NET_W1H = 8, NET_W2 = 72, NET_WOUT = 648, NET_NPARAM = 656 };

typedef struct {
    int L[4];
    int64_t V, Vh;
    int ap;
} ngeo;

static int ngeo_init(ngeo *g, const int *dims, int ap)
{
    g->V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || (dims[mu] & 1)) return -1;
        g->L[mu] = dims[mu];
        g->V *= dims[mu];
    }
    g->Vh = g->V / 2;
    g->ap = ap;
    return 0;
}

static void ncoord(const ngeo *g, int64_t lex, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(lex % g->L[mu]);
        lex /= g->L[mu];
    }
}

static int64_t nlex(const ngeo *g, const int x[4])
{
    return x[0] + (int64_t)g->L[0] * (x[1] + (int64_t)g->L[1] * (x[2] + (int64_t)g->L[2] * x[3]));
}

static double neta(int mu, const int x[4])
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += x[nu];
    return (s & 1) ? -1.0 : 1.0;
}

static double nbc(const ngeo *g, int mu, const int x[4])
{
    return (g->ap && mu == 3 && x[3] == g->L[3] - 1) ? -1.0 : 1.0;
}

/* out = (T_d psi)(x) for one site x; psi is indexed by lex and holds nch
 * channels of 3 colours: psi[(lex*nch + ch)*3 + a]. */
static void hop_site(const ngeo *g, const cplx *U, const int x[4], int d, const cplx *psi, int nch, int ch,
                     cplx out[3])
{
    const int mu = d & 3;
    int y[4];
    memcpy(y, x, sizeof(y));
    if (d < 4) {
        y[mu] = (x[mu] + 1) % g->L[mu];
        const double s = neta(mu, x) * nbc(g, mu, x);
        const cplx *u = U + ((int64_t)mu * g->V + nlex(g, x)) * 9;
        const cplx *v = psi + (nlex(g, y) * nch + ch) * 3;
        for (int a = 0; a < 3; ++a) out[a] = s * (u[a * 3 + 0] * v[0] + u[a * 3 + 1] * v[1] + u[a * 3 + 2] * v[2]);
    } else {
        y[mu] = (x[mu] - 1 + g->L[mu]) % g->L[mu];
        const double s = neta(mu, x) * nbc(g, mu, y);
        const cplx *u = U + ((int64_t)mu * g->V + nlex(g, y)) * 9;
        const cplx *v = psi + (nlex(g, y) * nch + ch) * 3;
        for (int a = 0; a < 3; ++a)
            out[a] = s * (conj(u[0 * 3 + a]) * v[0] + conj(u[1 * 3 + a]) * v[1] + conj(u[2 * 3 + a]) * v[2]);
    }
}

/* Full-lattice fields used by forward and backward (lex-indexed). */
typedef struct {
    cplx *r;     /* V x 1 x 3 (zero on odd sites) */
    cplx *phi1;  /* V x 8 x 3 */
    cplx *f;     /* V x 72 x 3 (even sites only) */
    cplx *phi2;  /* V x 8 x 3 (even sites only) */
} nfields;

static void nfields_free(nfields *F)
{
    free(F->r);
    free(F->phi1);
    free(F->f);
    free(F->phi2);
}

static int forward_fields(const ngeo *g, const cplx *U, const cplx *th, const cplx *r_eo, nfields *F)
{
    F->r = calloc((size_t)g->V * 3, sizeof(cplx));
    F->phi1 = calloc((size_t)g->V * NC * 3, sizeof(cplx));
    F->f = calloc((size_t)g->V * NK * 3, sizeof(cplx));
    F->phi2 = calloc((size_t)g->V * NC * 3, sizeof(cplx));
    if (!F->r || !F->phi1 || !F->f || !F->phi2) return -2;
    for (int64_t lex = 0; lex < g->V; ++lex) {
        int x[4];
        ncoord(g, lex, x);
        if (((x[0] + x[1] + x[2] + x[3]) & 1) == 0)
            for (int a = 0; a < 3; ++a) F->r[lex * 3 + a] = r_eo[(lex >> 1) * 3 + a];
    }
    /* layer 1 */
#pragma omp parallel for schedule(static)
    for (int64_t lex = 0; lex < g->V; ++lex) {
        int x[4];
        ncoord(g, lex, x);
        cplx *o = F->phi1 + lex * NC * 3;
        if (((x[0] + x[1] + x[2] + x[3]) & 1) == 0) {
            for (int c = 0; c < NC; ++c)
                for (int a = 0; a < 3; ++a) o[c * 3 + a] = th[NET_W1S + c] * F->r[lex * 3 + a];
        } else {
            for (int d = 0; d < 8; ++d) {
                cplx h[3];
                hop_site(g, U, x, d, F->r, 1, 0, h);
                for (int c = 0; c < NC; ++c)
                    for (int a = 0; a < 3; ++a) o[c * 3 + a] += th[NET_W1H + 8 * c + d] * h[a];
            }
        }
    }
    /* layer 2 and its inputs f, even sites */
#pragma omp parallel for schedule(static)
    for (int64_t lex = 0; lex < g->V; ++lex) {
        int x[4];
        ncoord(g, lex, x);
        if ((x[0] + x[1] + x[2] + x[3]) & 1) continue;
        cplx *f = F->f + lex * NK * 3;
        for (int c = 0; c < NC; ++c)
            for (int a = 0; a < 3; ++a) f[c * 3 + a] = F->phi1[(lex * NC + c) * 3 + a];
        for (int d = 0; d < 8; ++d)
            for (int c = 0; c < NC; ++c) hop_site(g, U, x, d, F->phi1, NC, c, f + (8 + 8 * d + c) * 3);
        cplx *o = F->phi2 + lex * NC * 3;
        for (int c = 0; c < NC; ++c)
            for (int a = 0; a < 3; ++a) {
                cplx s = 0;
                for (int k = 0; k < NK; ++k) s += th[NET_W2 + NK * c + k] * f[k * 3 + a];
                o[c * 3 + a] = s;
            }
    }
    return 0;
}

/* P(r) on even sites; r and out are (V/2, 3) eo-indexed. */
int orc_net_forward(const int *dims, int antiperiodic_t, const cplx *U, const cplx *theta, const cplx *r,
                    cplx *out)
{
    ngeo g;
    if (ngeo_init(&g, dims, antiperiodic_t)) return -1;
    nfields F;
    int rc = forward_fields(&g, U, theta, r, &F);
    if (rc == 0) {
        for (int64_t lex = 0; lex < g.V; ++lex) {
            int x[4];
            ncoord(&g, lex, x);
            if ((x[0] + x[1] + x[2] + x[3]) & 1) continue;
            for (int a = 0; a < 3; ++a) {
                cplx s = 0;
                for (int c = 0; c < NC; ++c) s += theta[NET_WOUT + c] * F.phi2[(lex * NC + c) * 3 + a];
                out[(lex >> 1) * 3 + a] = s;
            }
        }
    }
    nfields_free(&F);
    return rc;
}

/* Intermediate layer-1 field on odd sites, (V/2, 8, 3) eo-indexed: a hook
 * for checking the device's first layer on its own. */
int orc_net_layer1_odd(const int *dims, int antiperiodic_t, const cplx *U, const cplx *theta, const cplx *r,
                       cplx *phi1_odd)
{
    ngeo g;
    if (ngeo_init(&g, dims, antiperiodic_t)) return -1;
    nfields F;
    int rc = forward_fields(&g, U, theta, r, &F);
    if (rc == 0)
        for (int64_t lex = 0; lex < g.V; ++lex) {
            int x[4];
            ncoord(&g, lex, x);
            if (((x[0] + x[1] + x[2] + x[3]) & 1) == 0) continue;
            memcpy(phi1_odd + (lex >> 1) * NC * 3, F.phi1 + lex * NC * 3, sizeof(cplx) * NC * 3);
        }
    nfields_free(&F);
    return rc;
}

/* grad[j] = dL/dRe theta_j + i dL/dIm theta_j for L = Re sum_x <g(x), P(r)(x)>.
 * g is (V/2, 3) on even sites.  grad has NET_NPARAM entries (overwritten). */
int orc_net_backward(const int *dims, int antiperiodic_t, const cplx *U, const cplx *theta, const cplx *r,
                     const cplx *gout, cplx *grad)
{
    ngeo g;
    if (ngeo_init(&g, dims, antiperiodic_t)) return -1;
    nfields F;
    int rc = forward_fields(&g, U, theta, r, &F);
    cplx *gf = calloc((size_t)g.V * NK * 3, sizeof(cplx));   /* adjoint of f, even sites */
    cplx *gphi1 = calloc((size_t)g.V * NC * 3, sizeof(cplx));/* adjoint of phi1, odd sites */
    if (rc || !gf || !gphi1) {
        nfields_free(&F);
        free(gf);
        free(gphi1);
        return rc ? rc : -2;
    }
    memset(grad, 0, sizeof(cplx) * NET_NPARAM);
    /* output projection and layer 2 */
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int x[4];
        ncoord(&g, lex, x);
        if ((x[0] + x[1] + x[2] + x[3]) & 1) continue;
        const cplx *gx = gout + (lex >> 1) * 3;
        for (int c = 0; c < NC; ++c) {
            for (int a = 0; a < 3; ++a) {
                const cplx g2 = conj(theta[NET_WOUT + c]) * gx[a];       /* adjoint of phi2[c] */
                grad[NET_WOUT + c] += gx[a] * conj(F.phi2[(lex * NC + c) * 3 + a]);
                for (int k = 0; k < NK; ++k) {
                    grad[NET_W2 + NK * c + k] += g2 * conj(F.f[(lex * NK + k) * 3 + a]);
                    gf[(lex * NK + k) * 3 + a] += conj(theta[NET_W2 + NK * c + k]) * g2;
                }
            }
        }
        /* self part of layer 1 */
        for (int c = 0; c < NC; ++c)
            for (int a = 0; a < 3; ++a) grad[NET_W1S + c] += gf[(lex * NK + c) * 3 + a] * conj(F.r[lex * 3 + a]);
    }
    /* adjoint of the layer-2 hops: the hop T_d taken at even x reads phi1 at
     * x +- mu; its adjoint is T_{d'} with d' the opposite direction, applied
     * to the adjoint field gf_d living on even sites. */
    cplx *tmp = calloc((size_t)g.V * 3, sizeof(cplx));
    if (!tmp) {
        nfields_free(&F);
        free(gf);
        free(gphi1);
        return -2;
    }
    for (int d = 0; d < 8; ++d) {
        const int dbar = (d + 4) & 7;
        for (int c = 0; c < NC; ++c) {
            memset(tmp, 0, sizeof(cplx) * g.V * 3);
            for (int64_t lex = 0; lex < g.V; ++lex)
                for (int a = 0; a < 3; ++a) tmp[lex * 3 + a] = gf[(lex * NK + 8 + 8 * d + c) * 3 + a];
#pragma omp parallel for schedule(static)
            for (int64_t lex = 0; lex < g.V; ++lex) {
                int y[4];
                ncoord(&g, lex, y);
                if (((y[0] + y[1] + y[2] + y[3]) & 1) == 0) continue;
                cplx h[3];
                hop_site(&g, U, y, dbar, tmp, 1, 0, h);
                for (int a = 0; a < 3; ++a) gphi1[(lex * NC + c) * 3 + a] += h[a];
            }
        }
    }
    free(tmp);
    /* layer-1 hop weights */
    for (int64_t lex = 0; lex < g.V; ++lex) {
        int y[4];
        ncoord(&g, lex, y);
        if (((y[0] + y[1] + y[2] + y[3]) & 1) == 0) continue;
        for (int d = 0; d < 8; ++d) {
            cplx h[3];
            hop_site(&g, U, y, d, F.r, 1, 0, h);
            for (int c = 0; c < NC; ++c)
                for (int a = 0; a < 3; ++a) grad[NET_W1H + 8 * c + d] += gphi1[(lex * NC + c) * 3 + a] * conj(h[a]);
        }
    }
    nfields_free(&F);
    free(gf);
    free(gphi1);
    return 0;
}

int orc_net_nparam(void) { return NET_NPARAM; }
