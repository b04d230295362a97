"""FP64 oracle of the RHMC trajectory around the multi-shift solver.

TEST INFRASTRUCTURE.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark use this module; the library package never imports it.

Plain NumPy in double precision, vectorised over links only, following the
algorithm of Section 2 of the paper (RHMC with a multi-step, second order
minimum norm integrator that splits the action into its gauge and fermion
parts, several pseudo-fermions, and separate rational approximations for
the Metropolis step and the molecular dynamics) and Section 4 (the
Metropolis step in double precision; gauge update followed by
reunitarisation).  The paper prints none of the formulas; the readings
used are the textbook ones:

  Gauge action (Wilson plaquette):
      S_g = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3),
      P_munu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
  Momenta: one traceless Hermitian P_mu(x) = sum_a p_a lambda_a / 2 per
      link (lambda_a the Gell-Mann matrices), stored as the 8 reals p_a;
      the heatbath draws p_a ~ N(0, 1), the kinetic energy is
      K = (1/2) sum p_a^2 = sum tr P^2.
  Equations of motion: dU/dt = i P U; the force F on a link is defined
      by dS/deps = i tr(T F) for U -> exp(i eps T) U, and then
      dp_a/dt = Im tr(lambda_a F) / 2 conserves K + S.
  Gauge force: F_g = -(beta / 3) TA(U_mu(x) A_mu(x)) with A the sum of the
      six staples and TA(X) = (X - X^dag)/2 - tr(X - X^dag)/6.
  Fermion action of n_pf pseudo-fermions phi_k with a rational function
      r(M) = alpha0 + sum_i alpha_i (M + sigma_i)^-1:
      S_f = sum_k <phi_k, r(M) phi_k>; its force from the C oracle.
  Integrator: the second order minimum norm scheme of Omelyan, Mryglod and
      Folk (lambda = 0.1931833275037836) on two levels (Sexton and
      Weingarten's multiple time scales): per outer step delta = tau / n_md
          kick_f(lambda delta) G(delta/2) kick_f((1-2 lambda) delta)
          G(delta/2) kick_f(lambda delta),
      where G(h) runs n_g inner steps of size d = h / n_g,
          kick_g(lambda d) U(d/2) kick_g((1-2 lambda) d) U(d/2) kick_g(lambda d),
      and U(h): U <- exp(i h P) U, then reunitarisation.
  Trajectory: phi_k = r_hb(M) xi_k from Gaussian xi_k (heatbath),
      H0 = K + S_g + sum_k |xi_k|^2, integrate, H1 = K + S_g + S_f with the
      Metropolis approximation r_act, accept when u < exp(-(H1 - H0)).
"""
from __future__ import annotations

import numpy as np

LAMBDA_2MN = 0.1931833275037836


# ---------------------------------------------------------------- geometry
def volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


def coords(dims):
    """(V, 4) coordinates of lex = x0 + L0 (x1 + L1 (x2 + L2 x3))."""
    V = volume(dims)
    lex = np.arange(V)
    out = np.empty((V, 4), np.int64)
    rest = lex
    for mu in range(4):
        out[:, mu] = rest % dims[mu]
        rest = rest // dims[mu]
    return out


def lex_of(dims, c):
    return c[:, 0] + dims[0] * (c[:, 1] + dims[1] * (c[:, 2] + dims[2] * c[:, 3]))


def shifted(dims, mu, step):
    """lex of x + step * mu-hat (periodic) for every lex x."""
    c = coords(dims)
    c[:, mu] = (c[:, mu] + step) % dims[mu]
    return lex_of(dims, c)


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def gell_mann():
    g = np.zeros((8, 3, 3), np.complex128)
    g[0, 0, 1] = g[0, 1, 0] = 1
    g[1, 0, 1], g[1, 1, 0] = -1j, 1j
    g[2, 0, 0], g[2, 1, 1] = 1, -1
    g[3, 0, 2] = g[3, 2, 0] = 1
    g[4, 0, 2], g[4, 2, 0] = -1j, 1j
    g[5, 1, 2] = g[5, 2, 1] = 1
    g[6, 1, 2], g[6, 2, 1] = -1j, 1j
    g[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return g


# ---------------------------------------------------------------- gauge action and force
def plaquette(dims, U, mu, nu):
    """P_munu(x) for every x, shape (V, 3, 3)."""
    xpm, xpn = shifted(dims, mu, +1), shifted(dims, nu, +1)
    return U[mu] @ U[nu][xpm] @ dag(U[mu][xpn]) @ dag(U[nu])


def gauge_action(dims, U, beta):
    """Wilson plaquette action beta sum_{x, mu<nu} (1 - Re tr P_munu / 3)."""
    s = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            tr = np.trace(plaquette(dims, U, mu, nu), axis1=1, axis2=2).real
            s += np.sum(1.0 - tr / 3.0)
    return beta * s


def staples(dims, U, mu):
    """A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                                + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)],
    so that the action depends on U_mu(x) through -beta/3 Re tr(U_mu(x) A_mu(x))."""
    V = volume(dims)
    A = np.zeros((V, 3, 3), np.complex128)
    xpm = shifted(dims, mu, +1)
    for nu in range(4):
        if nu == mu:
            continue
        xpn, xmn = shifted(dims, nu, +1), shifted(dims, nu, -1)
        xpm_mn = shifted(dims, nu, -1)[xpm]
        A += U[nu][xpm] @ dag(U[mu][xpn]) @ dag(U[nu])
        A += dag(U[nu][xpm_mn]) @ dag(U[mu][xmn]) @ U[nu][xmn]
    return A


def traceless_antihermitian(X):
    Y = 0.5 * (X - dag(X))
    tr = np.trace(Y, axis1=-2, axis2=-1)
    return Y - (tr / 3.0)[..., None, None] * np.eye(3)


def gauge_force(dims, U, beta):
    """F_mu(x) = -(beta / 3) TA(U_mu(x) A_mu(x)), shape (4, V, 3, 3)."""
    return np.stack([-(beta / 3.0) * traceless_antihermitian(U[mu] @ staples(dims, U, mu))
                     for mu in range(4)])


# ---------------------------------------------------------------- momenta and link update
def momentum_matrix(p):
    """P = sum_a p_a lambda_a / 2 from the (..., 8) algebra coordinates."""
    return np.einsum("...a,aij->...ij", p, gell_mann() / 2)


def kinetic_energy(p):
    return 0.5 * float(np.sum(p * p))


def momentum_update(p, F, eps):
    """p_a += eps Im tr(lambda_a F) / 2: the momentum step dp/dt = -dS/dq
    for a force F in the convention dS/deps = i tr(T F)."""
    return p + eps * np.einsum("aij,...ji->...a", gell_mann() / 2, F).imag


def expi(Q):
    """exp(i Q) of Hermitian matrices Q (..., 3, 3) from their eigen-decomposition."""
    w, v = np.linalg.eigh(Q)
    return (v * np.exp(1j * w)[..., None, :]) @ dag(v)


def reunitarize(U):
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1) (SU(3))."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def link_update(U, p, eps):
    """U <- exp(i eps P) U for every link, then reunitarisation (Section 4)."""
    return reunitarize(expi(eps * momentum_matrix(p)) @ U)


# ---------------------------------------------------------------- fermion part
def fermion_force(orc, dims, U, mass, rat, phis, tol, antiperiodic_t=True):
    """Force of S_f = sum_k <phi_k, r(M) phi_k>: the multi-shift solutions of
    every pseudo-fermion, then the C oracle's force."""
    alpha0, alphas, shifts = rat
    F = np.zeros(U.shape, np.complex128)
    iters = 0
    for phi in phis:
        x, rc, info = orc.multishift_cg(dims, U, mass, shifts, phi, tol=tol, antiperiodic_t=antiperiodic_t)
        if rc != 0:
            raise RuntimeError(f"oracle multi-shift solve failed ({rc})")
        iters += info["iters"]
        F += orc.fermion_force(dims, U, alphas, x, antiperiodic_t)
    return F, iters


def fermion_action(orc, dims, U, mass, rat, phis, tol, antiperiodic_t=True):
    alpha0, alphas, shifts = rat
    s = 0.0
    for phi in phis:
        _, rc, info = orc.rational_apply(dims, U, mass, alpha0, alphas, shifts, phi, tol=tol,
                                         antiperiodic_t=antiperiodic_t)
        if rc != 0:
            raise RuntimeError(f"oracle rational apply failed ({rc})")
        s += info["dot"]
    return s


# ---------------------------------------------------------------- integrator
def integrate_2mn(kick_f, kick_g, drift, tau, n_md, n_g, lam=LAMBDA_2MN):
    """The two-level second order minimum norm scheme on abstract steps:
    kick_f(h), kick_g(h) advance the momenta by the fermion / gauge force
    for a time h, drift(h) the links."""
    delta = tau / n_md

    def gauge_part(h):
        d = h / n_g
        for _ in range(n_g):
            kick_g(lam * d)
            drift(0.5 * d)
            kick_g((1.0 - 2.0 * lam) * d)
            drift(0.5 * d)
            kick_g(lam * d)

    for _ in range(n_md):
        kick_f(lam * delta)
        gauge_part(0.5 * delta)
        kick_f((1.0 - 2.0 * lam) * delta)
        gauge_part(0.5 * delta)
        kick_f(lam * delta)


def md_integrate(orc, dims, U, p, phis, prm, antiperiodic_t=True):
    """Molecular dynamics for a time prm['tau'] from (U, p) with the
    pseudo-fermions phis fixed.  prm: beta, mass, tau, n_md, n_g, rat_md
    (alpha0, alphas, shifts), tol_md.  Returns (U, p, info)."""
    st = {"U": np.array(U, np.complex128), "p": np.array(p, np.float64), "iters": 0, "forces": 0}
    beta, mass = prm["beta"], prm["mass"]

    def kick_f(h):
        if not phis:
            return
        F, it = fermion_force(orc, dims, st["U"], mass, prm["rat_md"], phis, prm["tol_md"], antiperiodic_t)
        st["iters"] += it
        st["forces"] += 1
        st["p"] = momentum_update(st["p"], F, h)

    def kick_g(h):
        st["p"] = momentum_update(st["p"], gauge_force(dims, st["U"], beta), h)

    def drift(h):
        st["U"] = link_update(st["U"], st["p"], h)

    integrate_2mn(kick_f, kick_g, drift, prm["tau"], prm["n_md"], prm["n_g"])
    return st["U"], st["p"], {"iters": st["iters"], "fermion_forces": st["forces"]}


def hamiltonian(orc, dims, U, p, phis, prm, antiperiodic_t=True):
    """(K, S_g, S_f) with the Metropolis approximation prm['rat_act'] and
    tolerance prm['tol_act']."""
    K = kinetic_energy(p)
    Sg = gauge_action(dims, U, prm["beta"])
    Sf = fermion_action(orc, dims, U, prm["mass"], prm["rat_act"], phis, prm["tol_act"], antiperiodic_t)
    return K, Sg, Sf


def trajectory(orc, dims, U, p, xis, prm, u, antiperiodic_t=True):
    """One RHMC trajectory: heatbath of the pseudo-fermions from the Gaussian
    fields xis with prm['rat_hb'] (tolerance prm['tol_act']), the
    molecular dynamics, and the Metropolis test against the uniform number u
    (u < 0: accept regardless).  Returns (U_out, p_out, info); U_out is the
    initial field when the proposal is rejected."""
    a0, al, sh = prm["rat_hb"]
    phis = []
    for xi in xis:
        phi, rc, _ = orc.rational_apply(dims, U, prm["mass"], a0, al, sh, xi, tol=prm["tol_act"],
                                        antiperiodic_t=antiperiodic_t)
        if rc != 0:
            raise RuntimeError(f"oracle heatbath failed ({rc})")
        phis.append(phi)
    K0 = kinetic_energy(p)
    Sg0 = gauge_action(dims, U, prm["beta"])
    Sf0 = float(sum(np.vdot(xi, xi).real for xi in xis))
    U1, p1, info = md_integrate(orc, dims, U, p, phis, prm, antiperiodic_t)
    K1, Sg1, Sf1 = hamiltonian(orc, dims, U1, p1, phis, prm, antiperiodic_t)
    dH = (K1 + Sg1 + Sf1) - (K0 + Sg0 + Sf0)
    accept = bool(u < 0 or u < np.exp(-dH))
    info = dict(info, dH=dH, accepted=accept, H0=(K0, Sg0, Sf0), H1=(K1, Sg1, Sf1), phis=phis)
    return (U1 if accept else np.array(U)), p1, info
