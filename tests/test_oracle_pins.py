"""Pins of the FP64 oracle against facts the mathematics fixes.

Each pin is chosen so that a plausible slip in the oracle (a dropped hop, a
wrong sign or eta phase, a transposed or misplaced link, a wrong boundary
sign, a wrong neighbour index, a wrong shifted-CG coefficient) fails at
least one of them:

  * free field: plane waves are eigenvectors of M with eigenvalue
    m^2 + sum_mu sin^2 p_mu (antiperiodic p_3), and the full even-site
    spectrum is that multiset           -> normalisation, eta, BC, indexing
  * anti-Hermiticity D^dag = -D         -> relative sign, dagger on back hop
  * parity mapping                      -> D_eo is D restricted odd->even
  * gauge covariance                    -> which link sits on which hop
  * translation by two sites            -> neighbour wrap-around
  * multi-shift CG: closed-form solves of plane-wave sources, dense direct
    solves, single-shift CG, iterated vs true residual  -> zeta recursion
"""
import numpy as np
import pytest

import stag_synth as syn
from tests import lattice_np as ln

LATTICES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 4), (2, 4, 6, 2), (6, 4, 2, 8)]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("antiperiodic", [True, False])
def test_free_field_plane_wave_eigen(orc, dims, antiperiodic):
    rng = np.random.default_rng(7)
    U = ln.free_links(dims)
    m = 0.3
    for trial in range(4):
        n = [int(rng.integers(0, d)) for d in dims]
        colour = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        full, p = ln.plane_wave(dims, n, colour, antiperiodic)
        psi = ln.restrict(dims, 0, full)
        lam = m * m + np.sum(np.sin(p) ** 2)
        out = orc.normal_op(dims, U, m, 0.0, psi, antiperiodic)
        assert rel(out, lam * psi) < 1e-13
        # shifted operator adds the shift to the eigenvalue
        out = orc.normal_op(dims, U, m, 0.25, psi, antiperiodic)
        assert rel(out, (lam + 0.25) * psi) < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 2, 4), (2, 2, 4, 6)])
def test_free_field_spectrum(orc, dims):
    U = ln.free_links(dims)
    m = 0.2
    V = int(np.prod(dims))
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, m, 0.0, v), 3 * V // 2)
    ev = np.sort(np.linalg.eigvalsh((M + M.conj().T) / 2))
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    L = np.array(dims, float)
    ps = [2 * np.pi * g.ravel() / L[mu] for mu, g in enumerate(grids)]
    ps[3] = 2 * np.pi * (grids[3].ravel() + 0.5) / L[3]
    lam = m * m + sum(np.sin(p) ** 2 for p in ps)
    # momenta p and p + (pi,pi,pi,pi) coincide on even sites: every value twice
    expect = np.sort(np.repeat(lam, 3))[::2]
    assert np.max(np.abs(ev - expect)) < 1e-13
    assert np.max(np.abs(M - M.conj().T)) < 1e-14


def test_two_site_lattice_every_eigenvalue(orc):
    # On 2^4 with antiperiodic time, sin^2 p = 0 in x,y,z and 1 in t.
    dims = (2, 2, 2, 2)
    U = ln.free_links(dims)
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, 0.5, 0.0, v), 24)
    assert np.allclose(np.linalg.eigvalsh(M), 0.25 + 1.0, atol=1e-14)


@pytest.mark.parametrize("dims", LATTICES)
def test_anti_hermitian(orc, dims):
    rng = np.random.default_rng(11)
    U = syn.haar_links(dims, 5)
    V = int(np.prod(dims))
    a = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    b = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    lhs = np.vdot(a, orc.dhop_full(dims, U, b))
    rhs = -np.vdot(orc.dhop_full(dims, U, a), b)
    assert abs(lhs - rhs) < 1e-13 * np.linalg.norm(a) * np.linalg.norm(b)
    # even/odd blocks: <a_e, D_eo b_o> = -<D_oe a_e, b_o>
    ae, bo = a[: V // 2], b[: V // 2]
    lhs = np.vdot(ae, orc.dslash_eo(dims, U, 0, bo))
    rhs = -np.vdot(orc.dslash_eo(dims, U, 1, ae), bo)
    assert abs(lhs - rhs) < 1e-13 * np.linalg.norm(ae) * np.linalg.norm(bo)


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("p_in", [0, 1])
def test_parity_mapping(orc, dims, p_in):
    rng = np.random.default_rng(3)
    U = syn.haar_links(dims, 9)
    V = int(np.prod(dims))
    v = rng.standard_normal((V // 2, 3)) + 1j * rng.standard_normal((V // 2, 3))
    full = orc.dhop_full(dims, U, ln.embed(dims, p_in, v))
    assert np.max(np.abs(ln.restrict(dims, p_in, full))) == 0.0
    half = orc.dslash_eo(dims, U, 1 - p_in, v)
    assert rel(ln.restrict(dims, 1 - p_in, full), half) < 1e-15


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 2), (6, 4, 2, 8)])
def test_gauge_covariance(orc, dims):
    rng = np.random.default_rng(5)
    V = int(np.prod(dims))
    U = syn.haar_links(dims, 21)
    omega = syn.haar_su3(V, rng)
    Ug = ln.gauge_transform(dims, U, omega)
    psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    lhs = orc.dhop_full(dims, Ug, np.einsum("nij,nj->ni", omega, psi))
    rhs = np.einsum("nij,nj->ni", omega, orc.dhop_full(dims, U, psi))
    assert rel(lhs, rhs) < 1e-14
    # even/odd operator and the normal operator transform the same way
    ev = ln.sites_of_parity(dims, 0)
    od = ln.sites_of_parity(dims, 1)
    vo = psi[od]
    lhs = orc.dslash_eo(dims, Ug, 0, np.einsum("nij,nj->ni", omega[od], vo))
    rhs = np.einsum("nij,nj->ni", omega[ev], orc.dslash_eo(dims, U, 0, vo))
    assert rel(lhs, rhs) < 1e-14
    ve = psi[ev]
    lhs = orc.normal_op(dims, Ug, 0.1, 0.0, np.einsum("nij,nj->ni", omega[ev], ve))
    rhs = np.einsum("nij,nj->ni", omega[ev], orc.normal_op(dims, U, 0.1, 0.0, ve))
    assert rel(lhs, rhs) < 1e-14


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
@pytest.mark.parametrize("nu", [0, 1, 2, 3])
def test_translation_by_two(orc, dims, nu):
    antiperiodic = nu != 3  # a shift in t moves the antiperiodic boundary
    rng = np.random.default_rng(13)
    V = int(np.prod(dims))
    U = syn.haar_links(dims, 33)
    back = ln.shifted_lex(dims, nu, -2)  # T psi (x) = psi(x - 2 nu)
    UT = U[:, back]
    psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    lhs = orc.dhop_full(dims, UT, psi[back], antiperiodic)
    rhs = orc.dhop_full(dims, U, psi, antiperiodic)[back]
    assert rel(lhs, rhs) < 1e-15


def test_translation_by_one_is_not_a_symmetry(orc):
    # eta phases break single-site translations: guards against eta == 1.
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(1)
    V = int(np.prod(dims))
    U = syn.haar_links(dims, 3)
    back = ln.shifted_lex(dims, 0, -1)
    psi = rng.standard_normal((V, 3)) + 1j * rng.standard_normal((V, 3))
    lhs = orc.dhop_full(dims, U[:, back], psi[back])
    rhs = orc.dhop_full(dims, U, psi)[back]
    assert rel(lhs, rhs) > 0.1


def test_normal_op_hermitian_positive(orc):
    dims = (4, 4, 4, 4)
    rng = np.random.default_rng(2)
    U = syn.haar_links(dims, 8)
    m = 0.1
    n = 3 * 128
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, m, 0.0, v), n)
    assert np.max(np.abs(M - M.conj().T)) < 1e-14
    ev = np.linalg.eigvalsh(M)
    assert ev.min() >= m * m - 1e-12
    # ||D|| <= 1/2 * 8 unitary hops = 4, so lambda_max <= m^2 + 16; a Haar
    # field sits well above the free-field maximum m^2 + 4.
    assert 4.0 < ev.max() <= m * m + 16.0 + 1e-12


# ---------------------------------------------------------------- solvers

def _free_superposition(dims, ns, m, rng):
    waves, lams = [], []
    for n in ns:
        colour = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        full, p = ln.plane_wave(dims, n, colour)
        waves.append(ln.restrict(dims, 0, full))
        lams.append(m * m + np.sum(np.sin(p) ** 2))
    return waves, np.array(lams)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_multishift_free_field_closed_form(orc, dims):
    """Plane-wave sources with K distinct eigenvalues: CG ends after K steps
    and x_i = sum_k psi_k / (lambda_k + sigma_i) exactly."""
    rng = np.random.default_rng(17)
    m = 0.1
    # four momenta with pairwise distinct eigenvalues on this lattice
    ns, seen = [], []
    while len(ns) < 4:
        n = tuple(int(rng.integers(0, d)) for d in dims)
        _, p = ln.plane_wave(dims, n, np.ones(3))
        lam = np.sum(np.sin(p) ** 2)
        if all(abs(lam - l) > 1e-3 for l in seen):
            ns.append(n)
            seen.append(lam)
    waves, lams = _free_superposition(dims, ns, m, rng)
    b = sum(waves)
    shifts = np.array([0.0, 1e-3, 0.05, 0.7, 3.0])
    U = ln.free_links(dims)
    x, rc, info = orc.multishift_cg(dims, U, m, shifts, b, tol=1e-12)
    assert rc == 0
    assert info["iters"] <= len(ns) + 1
    for i, s in enumerate(shifts):
        exact = sum(w / (l + s) for w, l in zip(waves, lams))
        assert rel(x[i], exact) < 1e-12


@pytest.mark.parametrize("dims,seed", [((2, 2, 2, 2), 1), ((4, 4, 4, 4), 101), ((4, 2, 2, 4), 7)])
def test_multishift_dense_solve(orc, dims, seed):
    rng = np.random.default_rng(seed)
    U = syn.haar_links(dims, seed)
    m = 0.1
    shifts = syn.logspace_shifts(1e-4, 1.0, 8)
    vh = int(np.prod(dims)) // 2
    b = syn.gaussian_source(dims, seed + 1)
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, m, 0.0, v), 3 * vh)
    x, rc, info = orc.multishift_cg(dims, U, m, shifts, b, tol=1e-10)
    assert rc == 0
    bb = b.ravel()
    for i, s in enumerate(shifts):
        A = M + s * np.eye(3 * vh)
        xd = np.linalg.solve(A, bb)
        r = np.linalg.norm(bb - A @ x[i].ravel()) / np.linalg.norm(bb)
        assert r <= 1.5e-10, (i, r)
        ev = np.linalg.eigvalsh(A)
        kappa = ev[-1] / ev[0]
        assert rel(x[i].ravel(), xd) <= 2 * kappa * 1e-10
        # the oracle's own true residual agrees with the dense one
        assert abs(info["resid_true"][i] - r) <= 1e-3 * r + 1e-16
    # iterated residual of each frozen shift is below tol
    assert np.all(info["resid_iter"] <= 1e-10)


def test_multishift_matches_single_shift_cg(orc):
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 101)
    b = syn.gaussian_source(dims, 102)
    m = 0.1
    shifts = np.array([0.0, 0.01, 0.5])
    x, rc, info = orc.multishift_cg(dims, U, m, shifts, b, tol=1e-11)
    assert rc == 0
    for i, s in enumerate(shifts):
        xs, rc1, info1 = orc.cg(dims, U, m, s, b, tol=1e-11)
        assert rc1 == 0
        assert info1["resid_true"] < 2e-11
        assert rel(x[i], xs) < 1e-8
    # a single shift is plain CG: same iteration count
    x1, rc, info1 = orc.multishift_cg(dims, U, m, [0.01], b, tol=1e-11)
    xs, _, infos = orc.cg(dims, U, m, 0.01, b, tol=1e-11)
    assert info1["iters"] == infos["iters"]
    assert rel(x1[0], xs) < 1e-13


def test_multishift_iterated_equals_true_residual_early(orc):
    """Before rounding noise dominates, the shifted residual zeta_i r equals
    the true residual of x_i; a wrong zeta recursion breaks this."""
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 41)
    b = syn.gaussian_source(dims, 42)
    shifts = np.array([0.0, 0.003, 0.1, 2.0])
    for kmax in (3, 10, 25):
        x, rc, info = orc.multishift_cg(dims, U, 0.1, shifts, b, tol=1e-14, max_iter=kmax)
        assert rc == 1 and info["iters"] == kmax
        active = info["resid_iter"] > 1e-14
        ri, rt = info["resid_iter"][active], info["resid_true"][active]
        # rounding floor ~1e-16 ||b|| once a shift is nearly converged
        assert np.all(np.abs(ri - rt) <= 1e-8 * rt + 1e-15), (kmax, ri, rt)


def test_multishift_shift_order_and_duplicates(orc):
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 61)
    b = syn.gaussian_source(dims, 62)
    shifts = np.array([0.5, 1e-3, 0.5, 0.02])  # unsorted, with a duplicate
    x, rc, info = orc.multishift_cg(dims, U, 0.1, shifts, b, tol=1e-10)
    assert rc == 0
    assert np.all(info["resid_true"] < 1.5e-10)
    assert rel(x[0], x[2]) < 1e-14


def test_multishift_zero_source_and_errors(orc):
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 1)
    b = np.zeros((128, 3), np.complex128)
    x, rc, info = orc.multishift_cg(dims, U, 0.1, [0.0, 0.1], b)
    assert rc == 0 and info["iters"] == 0 and not np.any(x)
    b = syn.gaussian_source(dims, 2)
    with pytest.raises(ValueError):
        orc.multishift_cg(dims, U, 0.0, [0.0], b)      # m <= 0
    with pytest.raises(ValueError):
        orc.multishift_cg(dims, U, 0.1, [-1.0], b)     # negative shift
    with pytest.raises(ValueError):
        orc.dslash_eo((3, 4, 4, 4), U, 0, b)           # odd extent
    x, rc, info = orc.multishift_cg(dims, U, 0.1, [0.0], b, max_iter=5)
    assert rc == 1 and info["iters"] == 5


def test_config1_end_to_end(orc):
    """The small workload (4^4 Haar, m=0.1, 8 shifts in [1e-4,1]) runs in seconds."""
    c = syn.config("c1_4x4x4x4_haar")
    U = syn.make_links(c["links"], c["dims"])
    b = syn.gaussian_source(c["dims"], c["source_seed"])
    shifts = syn.logspace_shifts(*c["shifts"])
    x, rc, info = orc.multishift_cg(c["dims"], U, c["mass"], shifts, b, tol=c["tol"])
    assert rc == 0
    assert np.all(info["resid_true"] <= 1e-10 * 1.5)
    assert 100 < info["iters"] < 1000


# ---------------------------------------------------------------- inputs

def test_haar_statistics():
    rng = np.random.default_rng(0)
    u = syn.haar_su3(200000, rng)
    tr = np.trace(u, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.01
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.02
    uu = u @ np.conj(np.swapaxes(u, 1, 2))
    assert np.max(np.abs(uu - np.eye(3))) < 1e-13
    assert np.max(np.abs(np.linalg.det(u) - 1)) < 1e-13


def test_smooth_links_su3():
    u = syn.smooth_links((4, 4, 4, 4), 0.5, 3).reshape(-1, 3, 3)
    uu = u @ np.conj(np.swapaxes(u, 1, 2))
    assert np.max(np.abs(uu - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(u) - 1)) < 1e-14
    # eps -> 0 approaches the identity; eps = 0.5 stays close to it
    assert np.real(np.trace(u, axis1=1, axis2=2)).mean() / 3 > 0.8
    u0 = syn.smooth_links((2, 2, 2, 2), 0.0, 3)
    assert np.max(np.abs(u0 - np.eye(3))) < 1e-14


def test_inputs_are_seeded():
    a = syn.smooth_links((2, 2, 2, 4), 0.5, 9)
    b = syn.smooth_links((2, 2, 2, 4), 0.5, 9)
    assert np.array_equal(a, b)
    assert np.array_equal(syn.gaussian_source((4, 4, 4, 4), 3), syn.gaussian_source((4, 4, 4, 4), 3))
    s = syn.gaussian_source((8, 8, 8, 8), 1)
    assert abs(np.mean(np.abs(s) ** 2) - 1.0) < 0.02


def test_float_pair_split_bound():
    """Section 5's storage of a double as two floats, b = RN_float(a) and
    c = RN_float(a - b): |a - (b + c)| <= 2^-48 |a| (the remainder is
    rounded once more, so the pair is not exact), and b alone is the single
    precision value.  Checked on link-like entries (|a| <= 1) and on a wide
    range of magnitudes."""
    rng = np.random.default_rng(41)
    a = np.concatenate([rng.uniform(-1, 1, 200000),
                        rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))])
    b = a.astype(np.float32)
    c = (a - b.astype(np.float64)).astype(np.float32)
    err = np.abs(a - (b.astype(np.float64) + c.astype(np.float64)))
    assert np.all(err <= 2.0 ** -48 * np.abs(a))
    assert np.max(err / np.abs(a)) > 2.0 ** -52      # not exact in general
    assert np.array_equal(b, a.astype(np.float32))
