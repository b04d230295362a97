"""The RHMC trajectory on the GPU against the oracle (oracle/rhmc.py), one
component at a time and then whole molecular dynamics and trajectories:

  * gauge force and action, every link format, double and single precision;
  * momentum kicks from the gauge force and from a given force;
  * the link update exp(i h P) U with the double precision reunitarisation;
  * molecular dynamics without and with pseudo-fermions (double precision
    arithmetic, compared entry by entry with the oracle's);
  * the trajectory: the energies H0, H1, dH and the Metropolis decision,
    rejection restoring the links;
  * second order energy violation, reversibility in double and in single
    precision (the paper reports about 5e-6 per degree of freedom for its
    single precision gauge update);
  * argument checks.

Tolerances of the single precision steps are derived from the arithmetic: a
force entry is a sum of 6 staples of entries at most 1, each the result of
at most 64 roundings, times beta/3; eps32 = 2^-24.
"""
import numpy as np
import pytest

import stag_synth as syn
from oracle import rhmc
from tests.gpu_common import lattice_with_links, links_np, log, pack, to_dev

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5433_amd  # noqa: F401


def _momenta(dims, seed):
    return np.random.default_rng(seed).standard_normal((4, rhmc.volume(dims), 8))


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _force_tol(beta, eps):
    return 64 * eps * (beta / 3.0) * 6


def _rational():
    return (0.3, np.array([0.05, 0.2, 0.6, 1.1]), np.array([0.01, 0.1, 0.7, 3.0]))


def _params(prec="f64", **kw):
    import paper_1010_5433_amd as stag
    rat = _rational()
    base = dict(beta=5.6, mass=0.1, tau=0.5, n_md=4, n_g=3, prec=prec, tol_md=1e-13, tol_act=1e-13,
                rat_md=rat, rat_act=rat, rat_hb=(0.8, np.array([0.02, 0.1]), np.array([0.05, 0.5])))
    base.update(kw)
    return stag.rhmc_params(**base)


def _oracle_prm(**kw):
    rat = _rational()
    prm = dict(beta=5.6, mass=0.1, tau=0.5, n_md=4, n_g=3, rat_md=rat, rat_act=rat, tol_md=1e-13,
               tol_act=1e-13, rat_hb=(0.8, np.array([0.02, 0.1]), np.array([0.05, 0.5])))
    prm.update(kw)
    return prm


# ---------------------------------------------------------------- single steps
@pytest.mark.parametrize("fmt", ["18", "12", "8", "18p", "12p"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_gauge_force_and_action(dims, fmt):
    log(f"gauge force dims={dims} fmt={fmt}")
    U0 = links_np(dims, "smooth", 0.5, 41)
    lat = lattice_with_links(dims, U0, fmt)
    U = _host(lat.links_get())        # the field as stored (compressed forms rebuilt)
    if fmt == "18":
        assert np.array_equal(U, U0)
    beta = 5.7
    ref = rhmc.gauge_force(dims, U, beta)
    F = _host(lat.gauge_force(beta, "f64"))
    assert np.abs(F - ref).max() <= _force_tol(beta, EPS64)
    F32 = _host(lat.gauge_force(beta, "f32"))
    assert np.abs(F32 - ref).max() <= _force_tol(beta, EPS32)
    S = lat.gauge_action(beta)
    Sref = rhmc.gauge_action(dims, U, beta)
    assert abs(S - Sref) <= 1e-12 * abs(Sref), (S, Sref)
    lat.close()


def test_links_get_pairs_round_trip():
    dims = (4, 4, 2, 6)
    U0 = links_np(dims, "haar", 0.5, 42)
    for fmt, tol in (("18p", 2.0 ** -47), ("12p", 1e-14)):
        lat = lattice_with_links(dims, U0, fmt)
        assert np.abs(_host(lat.links_get()) - U0).max() <= tol, fmt
        lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_kicks_vs_oracle(prec):
    import torch
    dims = (4, 4, 4, 6)
    U0 = links_np(dims, "smooth", 0.5, 43)
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    p = _momenta(dims, 44)
    beta, h = 5.5, 0.37
    eps = EPS64 if prec == "f64" else EPS32
    # gauge kick (the fused kernel of the molecular dynamics)
    mom = to_dev(p.copy())
    lat.gauge_kick(beta, h, mom, prec)
    ref = rhmc.momentum_update(p, rhmc.gauge_force(dims, U, beta), h)
    tol = 4 * eps * np.abs(p).max() + abs(h) * _force_tol(beta, eps)
    assert np.abs(_host(mom) - ref).max() <= tol
    # kick from a given force
    rng = np.random.default_rng(45)
    F = rng.standard_normal((4, rhmc.volume(dims), 3, 3)) + 1j * rng.standard_normal((4, rhmc.volume(dims), 3, 3))
    mom = to_dev(p.copy())
    lat.force_kick(to_dev(F), h, mom, prec)
    ref = rhmc.momentum_update(p, F, h)
    tol = 4 * eps * (np.abs(p).max() + abs(h) * 4 * np.abs(F).max())
    assert np.abs(_host(mom) - ref).max() <= tol
    lat.close()


@pytest.mark.parametrize("fmt", ["18p", "12p"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_link_update_vs_oracle(fmt, prec):
    dims = (4, 2, 4, 4)
    U0 = links_np(dims, "smooth", 0.5, 46)
    lat = lattice_with_links(dims, U0, fmt)
    U = _host(lat.links_get())
    p = 1.5 * _momenta(dims, 47)        # some links need the scaling steps of the exponential
    for h in (0.3, -0.05):
        lat.link_update(to_dev(p), h, prec)
        got = _host(lat.links_get())
        if prec == "f64":
            ref = rhmc.link_update(U, p, h)
            tol = 1e-13
        else:
            # the single precision update reads the single precision half of the field
            ref = rhmc.link_update(U.astype(np.complex64).astype(np.complex128), p.astype(np.float32), h)
            tol = 64 * EPS32
        assert np.abs(got - ref).max() <= tol, (h, np.abs(got - ref).max())
        # the stored field is SU(3) to double precision
        assert np.abs(got @ rhmc.dag(got) - np.eye(3)).max() <= 1e-13
        assert np.abs(np.linalg.det(got) - 1).max() <= 1e-13
        U = got
    lat.close()


# ---------------------------------------------------------------- molecular dynamics
def test_md_pure_gauge_vs_oracle(orc):
    import torch
    dims = (4, 4, 2, 4)
    U0 = syn.smooth_links(dims, 0.5, 9)
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    p = _momenta(dims, 10)
    prm = _params("f64", beta=5.5, tau=0.6, n_md=3, n_g=2)
    mom = to_dev(p.copy())
    info = lat.md_integrate(prm, mom)
    Ur, pr, _ = rhmc.md_integrate(orc, dims, U, p, [], dict(beta=5.5, mass=0.1, tau=0.6, n_md=3, n_g=2,
                                                           rat_md=None, tol_md=1e-12))
    assert np.abs(_host(lat.links_get()) - Ur).max() <= 1e-10
    assert np.abs(_host(mom) - pr).max() <= 1e-10
    # merged kicks: 2 gauge-force evaluations per inner step plus one
    assert info["gauge_forces"] == 2 * (2 * prm.n_md * prm.n_g) + 1
    assert info["fermion_forces"] == 0
    lat.close()


@pytest.mark.parametrize("dims", [(4, 4, 2, 4), (6, 4, 4, 2)])
def test_md_with_fermions_vs_oracle(orc, dims):
    log(f"md with fermions dims={dims}")
    U0 = syn.smooth_links(dims, 0.5, 30)
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    p = _momenta(dims, 31)
    phis = [syn.gaussian_source(dims, 32), syn.gaussian_source(dims, 33)]
    mom = to_dev(p.copy())
    info = lat.md_integrate(_params("f64"), mom, [pack(lat, f) for f in phis])
    Ur, pr, oinfo = rhmc.md_integrate(orc, dims, U, p, phis, _oracle_prm())
    assert np.abs(_host(lat.links_get()) - Ur).max() <= 1e-9
    assert np.abs(_host(mom) - pr).max() <= 1e-8 * max(1.0, np.abs(pr).max())
    assert info["fermion_forces"] == 2 * 4 + 1 and oinfo["fermion_forces"] == 3 * 4
    assert info["md_iters"] > 0
    lat.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_md_two_fields_batched_equal_one_field_doubled(prec):
    """Several pseudo-fermion fields have their solves in one batched call
    and one force over all their solutions; a single field goes through the
    multi-shift solver and the force on its own.  Two copies of one field
    must then move links and momenta as that field alone with the force's
    rational weights doubled, since the force is linear in them."""
    dims = (6, 4, 4, 4)
    log(f"md: two copies of a field against one with doubled weights, {prec}")
    U0 = syn.smooth_links(dims, 0.5, 40)
    p = _momenta(dims, 41)
    phi = syn.gaussian_source(dims, 42)
    a0, al, sh = _rational()
    kw = dict(tol_md=1e-6) if prec == "f32" else {}
    res = []
    for copies, alphas in ((2, al), (1, 2.0 * al)):
        lat = lattice_with_links(dims, U0, "18p")
        mom = to_dev(p.copy())
        f = pack(lat, phi)
        info = lat.md_integrate(_params(prec, rat_md=(a0, alphas, sh), **kw), mom, [f] * copies)
        res.append((_host(lat.links_get()), _host(mom), info))
        lat.close()
    (U2, p2, i2), (U1, p1, i1) = res
    du, dp = np.abs(U2 - U1).max(), np.abs(p2 - p1).max() / max(1.0, np.abs(p1).max())
    log(f"  links {du:.2e}, momenta {dp:.2e}; MD iterations {i2['md_iters']} against 2 x {i1['md_iters']}")
    if prec == "f64":
        assert du <= 1e-11 and dp <= 1e-10
    else:
        assert du <= 1e-4 and dp <= 1e-3
    assert i2["fermion_forces"] == i1["fermion_forces"] == 2 * 4 + 1
    # the same systems under the same stopping rule: one iteration apart at most per solve
    assert abs(i2["md_iters"] - 2 * i1["md_iters"]) <= 2 * i1["fermion_forces"]


def test_md_two_fields_beyond_the_batch_limit():
    """Two fields with a 33-pole force rational have 66 solutions, more than
    one force call takes: the molecular dynamics then solves and applies the
    force field by field.  Two copies of a field must still move links and
    momenta as that field alone with the force weights doubled."""
    dims = (4, 4, 2, 4)
    log("md: two fields with 33 poles each (field by field)")
    U0 = syn.smooth_links(dims, 0.5, 50)
    p = _momenta(dims, 51)
    phi = syn.gaussian_source(dims, 52)
    sh = np.geomspace(1e-3, 5.0, 33)
    al = 0.02 * np.sqrt(sh)
    res = []
    for copies, alphas in ((2, al), (1, 2.0 * al)):
        lat = lattice_with_links(dims, U0, "18p")
        mom = to_dev(p.copy())
        f = pack(lat, phi)
        info = lat.md_integrate(_params("f64", rat_md=(0.1, alphas, sh)), mom, [f] * copies)
        res.append((_host(lat.links_get()), _host(mom), info))
        lat.close()
    (U2, p2, i2), (U1, p1, i1) = res
    du, dp = np.abs(U2 - U1).max(), np.abs(p2 - p1).max() / max(1.0, np.abs(p1).max())
    log(f"  links {du:.2e}, momenta {dp:.2e}; MD iterations {i2['md_iters']} against 2 x {i1['md_iters']}")
    assert du <= 1e-11 and dp <= 1e-10
    # the same solver on the same systems: the same iterations
    assert i2["md_iters"] == 2 * i1["md_iters"]
    assert i2["fermion_forces"] == i1["fermion_forces"] == 2 * 4 + 1


def test_md_single_precision_and_12_real_pairs_vs_oracle(orc):
    """The paper's setting (single precision momenta, gauge update and force
    solves at tol 1e-6) stays close to the double precision oracle over
    tau = 0.5; the 12-real float-pair field in double precision matches it
    to rounding."""
    dims = (4, 4, 2, 4)
    U0 = syn.smooth_links(dims, 0.5, 30)
    p = _momenta(dims, 31)
    phis = [syn.gaussian_source(dims, 32), syn.gaussian_source(dims, 33)]
    # double precision, 12-real pairs
    lat = lattice_with_links(dims, U0, "12p")
    U = _host(lat.links_get())
    mom = to_dev(p.copy())
    lat.md_integrate(_params("f64"), mom, [pack(lat, f) for f in phis])
    Ur, pr, _ = rhmc.md_integrate(orc, dims, U, p, phis, _oracle_prm())
    assert np.abs(_host(lat.links_get()) - Ur).max() <= 1e-9
    assert np.abs(_host(mom) - pr).max() <= 1e-8 * max(1.0, np.abs(pr).max())
    lat.close()
    # single precision, 18-real pairs
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    mom = to_dev(p.copy())
    info = lat.md_integrate(_params("f32", tol_md=1e-6), mom, [pack(lat, f) for f in phis])
    Ur, pr, _ = rhmc.md_integrate(orc, dims, U, p, phis, _oracle_prm())
    du = np.abs(_host(lat.links_get()) - Ur).max()
    dp = np.abs(_host(mom) - pr).max()
    log(f"single precision molecular dynamics against the double precision oracle: links {du:.2e}, momenta {dp:.2e}")
    assert du <= 1e-4 and dp <= 1e-3 * max(1.0, np.abs(pr).max())
    assert info["fermion_forces"] == 2 * 4 + 1
    lat.close()


@pytest.mark.parametrize("n_fields", [1, 2])
def test_trajectory_vs_oracle(orc, n_fields):
    """One field: heatbath and action by the single-field rational
    function; two fields: both fields in one batched application."""
    dims = (4, 4, 2, 4)
    U0 = syn.smooth_links(dims, 0.5, 30)
    p = _momenta(dims, 31)
    xis = [syn.gaussian_source(dims, 40), syn.gaussian_source(dims, 41)][:n_fields]
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    mom = to_dev(p.copy())
    info = lat.rhmc_trajectory(_params("f64"), mom, [pack(lat, x) for x in xis], u=-1.0)
    U1, p1, ref = rhmc.trajectory(orc, dims, U, p, xis, _oracle_prm(), u=-1.0)
    for a, b in zip(info["H0"] + info["H1"], list(ref["H0"]) + list(ref["H1"])):
        assert abs(a - b) <= 1e-10 * abs(b), (a, b)
    assert abs(info["dH"] - ref["dH"]) <= 1e-7, (info["dH"], ref["dH"])
    assert info["accepted"] and ref["accepted"]
    assert np.abs(_host(lat.links_get()) - U1).max() <= 1e-9
    assert np.abs(_host(mom) - p1).max() <= 1e-8 * max(1.0, np.abs(p1).max())
    # a u just above exp(-dH) rejects: the links return to the start
    lat2 = lattice_with_links(dims, U0, "18p")
    before = _host(lat2.links_get())
    u = min(np.exp(-info["dH"]) * (1 + 1e-6), 1 - 1e-12)
    if u < 1 - 1e-12:
        info2 = lat2.rhmc_trajectory(_params("f64"), to_dev(p.copy()), [pack(lat2, x) for x in xis], u=u)
        assert not info2["accepted"]
        assert np.array_equal(_host(lat2.links_get()), before)
    lat.close()
    lat2.close()


def _energy(lat, prm_md, mom, phis, rat, mass, beta):
    import torch
    torch.cuda.synchronize()
    K = 0.5 * float((mom * mom).sum())
    Sf = sum(lat.rational_apply(mass, rat[0], rat[1], rat[2], f, tol=1e-13)[3] for f in phis)
    return K + lat.gauge_action(beta) + Sf


def test_energy_violation_second_order(orc):
    """With the pseudo-fermion fields held fixed, H = K + S_g + S_f changes
    over the molecular dynamics by dH ~ delta^2: halving the outer step
    divides it by about 4; the value agrees with the oracle's."""
    dims = (4, 4, 2, 4)
    U0 = syn.smooth_links(dims, 0.5, 30)
    p = _momenta(dims, 31)
    phis_np = [syn.gaussian_source(dims, 32), syn.gaussian_source(dims, 33)]
    rat = _rational()
    dh = []
    for n_md in (4, 8):
        lat = lattice_with_links(dims, U0, "18p")
        phis = [pack(lat, f) for f in phis_np]
        mom = to_dev(p.copy())
        H0 = _energy(lat, None, mom, phis, rat, 0.1, 5.6)
        lat.md_integrate(_params("f64", n_md=n_md), mom, phis)
        dh.append(_energy(lat, None, mom, phis, rat, 0.1, 5.6) - H0)
        lat.close()
    assert abs(dh[0]) < 0.05 and 3.0 < dh[0] / dh[1] < 5.0, dh
    U = lattice_with_links(dims, U0, "18p").links_get().cpu().numpy()
    prm = _oracle_prm()
    H0 = sum(rhmc.hamiltonian(orc, dims, U, p, phis_np, prm))
    U1, p1, _ = rhmc.md_integrate(orc, dims, U, p, phis_np, prm)
    ref = sum(rhmc.hamiltonian(orc, dims, U1, p1, phis_np, prm)) - H0
    assert abs(dh[0] - ref) <= 1e-8, (dh[0], ref)


@pytest.mark.parametrize("prec,bound", [("f64", 1e-9), ("f32", 1e-4)])
def test_reversibility(prec, bound):
    """Forward tau, momenta flipped, forward tau again: back at the start up
    to rounding.  The violation per degree of freedom, the RMS of the link
    entry and momentum differences, is printed beside the paper's 5e-6 for a
    single precision gauge update."""
    import torch
    dims = (8, 8, 8, 8)
    U0 = syn.smooth_links(dims, 0.5, 50)
    lat = lattice_with_links(dims, U0, "18p")
    U = _host(lat.links_get())
    p = _momenta(dims, 51)
    phis = [pack(lat, syn.gaussian_source(dims, 52))]
    prm = _params(prec, tau=1.0, n_md=5, n_g=4, tol_md=1e-12 if prec == "f64" else 1e-6)
    mom = to_dev(p.copy())
    lat.md_integrate(prm, mom, phis)
    mom.neg_()
    lat.md_integrate(prm, mom, phis)
    U2, p2 = _host(lat.links_get()), -_host(mom)
    n_dof = U.size * 2 + p.size
    viol = np.sqrt((np.sum(np.abs(U2 - U) ** 2) + np.sum((p2 - p) ** 2)) / n_dof)
    log(f"reversibility ({prec}): {viol:.2e} per degree of freedom (paper: about 5e-6)")
    assert viol <= bound
    lat.close()


# ---------------------------------------------------------------- argument checks
def test_rhmc_argument_checks():
    import torch
    import paper_1010_5433_amd as stag
    dims = (4, 4, 4, 4)
    U0 = links_np(dims, "smooth", 0.5, 60)
    lat = lattice_with_links(dims, U0, "18")
    mom = to_dev(_momenta(dims, 61))
    with pytest.raises(stag.StagError, match="PAIRS"):
        lat.md_integrate(_params("f64"), mom)
    with pytest.raises(stag.StagError, match="PAIRS"):
        lat.link_update(mom, 0.1)
    lat.close()
    lat = lattice_with_links(dims, U0, "18p")
    phi = pack(lat, syn.gaussian_source(dims, 62))
    with pytest.raises(stag.StagError, match="tau"):
        lat.md_integrate(_params("f64", tau=0.0), mom, [phi])
    with pytest.raises(stag.StagError, match="n_pf"):
        lat.md_integrate(_params("f64"), mom, [phi] * 17)
    with pytest.raises(stag.StagError, match="rat_md"):
        lat.md_integrate(_params("f64", rat_md=None), mom, [phi])
    with pytest.raises(stag.StagError, match="u must be"):
        lat.rhmc_trajectory(_params("f64"), mom, [phi], u=1.0)
    # momenta overlapping a pseudo-fermion field
    big = torch.zeros(mom.numel() + phi.numel(), dtype=torch.float64, device="cuda")
    inside = big[mom.numel() - 8:mom.numel() - 8 + phi.numel()].view(phi.shape)
    with pytest.raises(stag.StagError, match="overlap"):
        lat.md_integrate(_params("f64"), big[:mom.numel()], [inside])
    # nothing ran: the links are unchanged
    assert np.array_equal(_host(lat.links_get()), _host(lattice_with_links(dims, U0, "18p").links_get()))
    lat.close()
