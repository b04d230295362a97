"""Pins of the RHMC trajectory oracle (oracle/rhmc.py) against what the
mathematics fixes, independent of the oracle's own formulas:

  * gauge action: zero on the unit field; a closed form for an abelian field
    of constant field strength; invariance under random gauge transforms;
  * gauge force: central differences of the action along exp(i eps T);
    covariance under gauge transforms;
  * generators and kinetic energy: tr(T_a T_b) = delta_ab / 2, K = sum tr P^2;
  * exp(i Q): SciPy's matrix exponential;
  * reunitarisation: fixes SU(3), maps near-SU(3) matrices into SU(3);
  * integrator: on a harmonic oscillator it is symmetric, second order and
    far more accurate than leapfrog at the same number of force evaluations
    (the minimum norm property); with no pseudo-fermions the two-level
    scheme equals the one-level scheme with the same inner steps;
  * molecular dynamics with fermions: energy violation falls as delta^2,
    the integration is reversible, the Metropolis step follows its rule.
A few planted mistakes (wrong sign, factor, staple, step) must each fail
one of these checks.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import rhmc
import stag_synth as syn


def random_su3(n, seed):
    return syn.haar_su3(n, np.random.default_rng(seed))


def random_hermitian_traceless(n, rng):
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    h = 0.5 * (z + np.conj(np.swapaxes(z, -1, -2)))
    return h - (np.trace(h, axis1=1, axis2=2) / 3)[:, None, None] * np.eye(3)


def gauge_transform(dims, U, omega):
    out = np.empty_like(U)
    for mu in range(4):
        xp = rhmc.shifted(dims, mu, +1)
        out[mu] = omega @ U[mu] @ rhmc.dag(omega[xp])
    return out


# ---------------------------------------------------------------- gauge action
def test_gauge_action_unit_field_is_zero():
    dims = (4, 2, 4, 2)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, rhmc.volume(dims), 3, 3)).copy()
    assert abs(rhmc.gauge_action(dims, U, 5.6)) < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_gauge_action_abelian_closed_form(n):
    """U_1(x) = diag(e^{i q x0}, e^{-i q x0}, 1) with q = 2 pi n / L0, all
    other links 1: only the (0,1) plaquettes differ from 1, each equal to
    diag(e^{iq}, e^{-iq}, 1), so S_g = beta V (2/3)(1 - cos q)."""
    dims = (6, 4, 2, 4)
    V = rhmc.volume(dims)
    q = 2 * np.pi * n / dims[0]
    x0 = rhmc.coords(dims)[:, 0]
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    U[1, :, 0, 0] = np.exp(1j * q * x0)
    U[1, :, 1, 1] = np.exp(-1j * q * x0)
    beta = 5.3
    want = beta * V * (2.0 / 3.0) * (1 - np.cos(q))
    assert abs(rhmc.gauge_action(dims, U, beta) - want) <= 1e-12 * want


def test_gauge_action_and_force_gauge_covariant():
    dims = (4, 4, 2, 2)
    V = rhmc.volume(dims)
    U = syn.smooth_links(dims, 0.7, 11)
    omega = random_su3(V, 12)
    Ut = gauge_transform(dims, U, omega)
    s, st = rhmc.gauge_action(dims, U, 5.0), rhmc.gauge_action(dims, Ut, 5.0)
    assert abs(s - st) <= 1e-12 * abs(s)
    F, Ft = rhmc.gauge_force(dims, U, 5.0), rhmc.gauge_force(dims, Ut, 5.0)
    for mu in range(4):
        assert np.max(np.abs(Ft[mu] - omega @ F[mu] @ rhmc.dag(omega))) <= 1e-12


@pytest.mark.parametrize("dims,kind", [((4, 4, 4, 4), "smooth"), ((2, 4, 2, 4), "haar"), ((4, 2, 6, 2), "smooth")])
def test_gauge_force_finite_differences(dims, kind):
    """dS/deps along U_mu(x) -> exp(i eps T) U_mu(x) equals i tr(T F_mu(x)),
    for random links, directions and Hermitian traceless T."""
    V = rhmc.volume(dims)
    U = syn.haar_links(dims, 21) if kind == "haar" else syn.smooth_links(dims, 0.6, 21)
    beta = 5.7
    F = rhmc.gauge_force(dims, U, beta)
    rng = np.random.default_rng(22)
    eps = 1e-5
    for _ in range(8):
        mu, x = int(rng.integers(4)), int(rng.integers(V))
        T = random_hermitian_traceless(1, rng)[0]
        want = (1j * np.trace(T @ F[mu, x])).real
        vals = []
        for e in (eps, -eps):
            Up = U.copy()
            Up[mu, x] = scipy.linalg.expm(1j * e * T) @ U[mu, x]
            vals.append(rhmc.gauge_action(dims, Up, beta))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - want) <= 1e-6 * max(1.0, abs(want)), (mu, x, fd, want)
    # the force is traceless and anti-Hermitian
    assert np.max(np.abs(F + rhmc.dag(F))) <= 1e-13
    assert np.max(np.abs(np.trace(F, axis1=-2, axis2=-1))) <= 1e-13


# ---------------------------------------------------------------- momenta, exp, reunitarisation
def test_generators_and_kinetic_energy():
    T = rhmc.gell_mann() / 2
    gram = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(gram, 0.5 * np.eye(8), atol=1e-15)
    for t in T:
        assert np.allclose(t, rhmc.dag(t)) and abs(np.trace(t)) < 1e-15
    p = np.random.default_rng(3).standard_normal((4, 16, 8))
    P = rhmc.momentum_matrix(p)
    assert abs(rhmc.kinetic_energy(p) - np.trace(P @ P, axis1=-2, axis2=-1).real.sum()) <= 1e-12 * rhmc.kinetic_energy(p)


def test_expi_matches_scipy_expm():
    rng = np.random.default_rng(4)
    Q = random_hermitian_traceless(20, rng) * 1.7
    E = rhmc.expi(Q)
    for q, e in zip(Q, E):
        assert np.max(np.abs(e - scipy.linalg.expm(1j * q))) <= 1e-13


def test_reunitarize():
    U = random_su3(50, 5)
    assert np.max(np.abs(rhmc.reunitarize(U) - U)) <= 1e-14
    rng = np.random.default_rng(6)
    W = U + 1e-4 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    R = rhmc.reunitarize(W)
    assert np.max(np.abs(R @ rhmc.dag(R) - np.eye(3))) <= 1e-14
    assert np.max(np.abs(np.linalg.det(R) - 1)) <= 1e-14
    assert np.max(np.abs(R - U)) <= 1e-3
    # row 0 keeps its direction
    r0 = W[:, 0, :] / np.linalg.norm(W[:, 0, :], axis=1, keepdims=True)
    assert np.max(np.abs(R[:, 0, :] - r0)) <= 1e-15


def test_link_update_inverse_and_group():
    dims = (2, 2, 2, 2)
    U = syn.smooth_links(dims, 0.5, 7)
    p = np.random.default_rng(8).standard_normal((4, rhmc.volume(dims), 8))
    U1 = rhmc.link_update(U, p, 0.3)
    assert np.max(np.abs(rhmc.link_update(U1, p, -0.3) - U)) <= 1e-13
    assert np.max(np.abs(rhmc.link_update(rhmc.link_update(U, p, 0.1), p, 0.2) - U1)) <= 1e-13


# ---------------------------------------------------------------- integrator on a toy system
def _oscillator(lam, h, T=10.0):
    st = {"p": 1.0, "q": 0.3}

    def kick(hh):
        st["p"] -= hh * st["q"]

    def drift(hh):
        st["q"] += hh * st["p"]

    H0 = 0.5 * (st["p"] ** 2 + st["q"] ** 2)
    err = 0.0
    for _ in range(int(round(T / h))):
        rhmc.integrate_2mn(lambda x: None, kick, drift, h, 1, 1, lam)
        err = max(err, abs(0.5 * (st["p"] ** 2 + st["q"] ** 2) - H0))
    return err, st


def test_integrator_second_order_and_minimum_norm():
    e1, _ = _oscillator(rhmc.LAMBDA_2MN, 0.2)
    e2, _ = _oscillator(rhmc.LAMBDA_2MN, 0.1)
    assert 3.5 < e1 / e2 < 4.5
    # leapfrog with half the step uses the same number of force evaluations
    # (lambda = 1/4 is two leapfrog steps of h/2)
    lf, _ = _oscillator(0.25, 0.2)
    assert e1 < lf / 10


def test_integrator_reversible_toy():
    st = {"p": 0.7, "q": -0.4}

    def kick(h):
        st["p"] -= h * (st["q"] + st["q"] ** 3)

    def drift(h):
        st["q"] += h * st["p"]

    rhmc.integrate_2mn(lambda h: kick(0.5 * h), lambda h: kick(0.5 * h), drift, 1.3, 5, 3)
    st["p"] = -st["p"]
    rhmc.integrate_2mn(lambda h: kick(0.5 * h), lambda h: kick(0.5 * h), drift, 1.3, 5, 3)
    assert abs(st["q"] + 0.4) < 1e-13 and abs(-st["p"] - 0.7) < 1e-13


def test_two_levels_without_fermions_equal_one_level(orc):
    dims = (4, 2, 2, 4)
    U = syn.smooth_links(dims, 0.5, 9)
    p = np.random.default_rng(10).standard_normal((4, rhmc.volume(dims), 8))
    prm = dict(beta=5.5, mass=0.1, tau=0.6, n_md=3, n_g=2, rat_md=None, tol_md=1e-12)
    Ua, pa, _ = rhmc.md_integrate(orc, dims, U, p, [], prm)
    Ub, pb, _ = rhmc.md_integrate(orc, dims, U, p, [], dict(prm, n_md=6, n_g=1))
    assert np.array_equal(Ua, Ub) and np.array_equal(pa, pb)


# ---------------------------------------------------------------- full molecular dynamics
def _rational():
    # a positive partial fraction (any such r(M) defines a valid action)
    return (0.3, np.array([0.05, 0.2, 0.6, 1.1]), np.array([0.01, 0.1, 0.7, 3.0]))


def _md_setup(dims=(4, 4, 2, 4), seed=30):
    U = syn.smooth_links(dims, 0.5, seed)
    p = np.random.default_rng(seed + 1).standard_normal((4, rhmc.volume(dims), 8))
    phis = [syn.gaussian_source(dims, seed + 2), syn.gaussian_source(dims, seed + 3)]
    rat = _rational()
    prm = dict(beta=5.6, mass=0.1, tau=0.5, n_md=4, n_g=3, rat_md=rat, rat_act=rat,
               tol_md=1e-13, tol_act=1e-13)
    return U, p, phis, prm


def _dH(orc, dims, U, p, phis, prm):
    H0 = sum(rhmc.hamiltonian(orc, dims, U, p, phis, prm))
    U1, p1, _ = rhmc.md_integrate(orc, dims, U, p, phis, prm)
    return sum(rhmc.hamiltonian(orc, dims, U1, p1, phis, prm)) - H0


def test_md_energy_violation_second_order(orc):
    dims = (4, 4, 2, 4)
    U, p, phis, prm = _md_setup(dims)
    d1 = _dH(orc, dims, U, p, phis, prm)
    d2 = _dH(orc, dims, U, p, phis, dict(prm, n_md=8, n_g=3))
    assert abs(d1) < 0.05
    assert 3.0 < d1 / d2 < 5.0, (d1, d2)


def test_md_reversible(orc):
    dims = (4, 4, 2, 4)
    U, p, phis, prm = _md_setup(dims)
    U1, p1, info = rhmc.md_integrate(orc, dims, U, p, phis, prm)
    assert info["fermion_forces"] == 3 * prm["n_md"]
    U2, p2, _ = rhmc.md_integrate(orc, dims, U1, -p1, phis, prm)
    assert np.max(np.abs(U2 - U)) <= 1e-10
    assert np.max(np.abs(-p2 - p)) <= 1e-10


def test_trajectory_metropolis_rule(orc):
    dims = (4, 4, 2, 4)
    U, p, _, prm = _md_setup(dims)
    rat_hb = (0.8, np.array([0.02, 0.1]), np.array([0.05, 0.5]))
    prm = dict(prm, rat_hb=rat_hb)
    xis = [syn.gaussian_source(dims, 40)]
    Ua, _, ia = rhmc.trajectory(orc, dims, U, p, xis, prm, u=-1.0)
    assert ia["accepted"]
    # u just above exp(-dH) rejects and returns the initial links
    u = min(np.exp(-ia["dH"]) * (1 + 1e-9), 1 - 1e-12) if ia["dH"] > -1e-9 else None
    if u is not None and u < 1:
        Ur, _, ir = rhmc.trajectory(orc, dims, U, p, xis, prm, u=u)
        assert not ir["accepted"] and np.array_equal(Ur, U)
    Uc, _, ic = rhmc.trajectory(orc, dims, U, p, xis, prm, u=0.0)
    assert ic["accepted"] and np.array_equal(Uc, Ua)
    # the heatbath's phi reproduces |xi|^2 when r_act is the inverse square of r_hb ... not
    # required here; H0's fermion part is |xi|^2 by construction
    assert abs(ia["H0"][2] - np.vdot(xis[0], xis[0]).real) <= 1e-12 * ia["H0"][2]


# ---------------------------------------------------------------- planted mistakes
def _mutant_fails(monkeypatch, orc, name, fn, check):
    monkeypatch.setattr(rhmc, name, fn)
    with pytest.raises(AssertionError):
        check(orc)


def test_planted_mistakes_fail_a_pin(monkeypatch, orc):
    orig_update = rhmc.momentum_update
    orig_staples = rhmc.staples
    orig_kin = rhmc.kinetic_energy
    orig_link = rhmc.link_update

    def fd_check(_orc):
        test_gauge_force_finite_differences((4, 4, 4, 4), "smooth")

    def md_check(_orc):
        test_md_energy_violation_second_order(_orc)

    mutants = [
        ("momentum_update", lambda p, F, e: orig_update(p, F, -e), md_check),          # kick sign
        ("kinetic_energy", lambda p: 2 * orig_kin(p), md_check),                       # K = sum p^2
        ("link_update", lambda U, p, e: orig_link(U, p, -e), md_check),                # exp(-i eps P)
        ("staples", lambda dims, U, mu: 2 * orig_staples(dims, U, mu), fd_check),      # force factor
    ]

    def upper_only(dims, U, mu):
        V = rhmc.volume(dims)
        A = np.zeros((V, 3, 3), np.complex128)
        xpm = rhmc.shifted(dims, mu, +1)
        for nu in range(4):
            if nu != mu:
                A += U[nu][xpm] @ rhmc.dag(U[mu][rhmc.shifted(dims, nu, +1)]) @ rhmc.dag(U[nu])
        return A
    mutants.append(("staples", upper_only, fd_check))                                 # lower staple lost
    for name, fn, check in mutants:
        with monkeypatch.context() as m:
            _mutant_fails(m, orc, name, fn, check)
    # a wrong integrator weight fails the minimum norm check
    with monkeypatch.context() as m:
        m.setattr(rhmc, "LAMBDA_2MN", 1.0 / 6.0)
        m.setattr(rhmc.integrate_2mn, "__defaults__", (1.0 / 6.0,))
        with pytest.raises(AssertionError):
            test_integrator_second_order_and_minimum_norm()
