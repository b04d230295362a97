"""Pseudo-fermion force on the GPU against the oracle's, element by
element: every link format, lattices of one tile, several tiles with a
ragged tail and many tiles, 0 to 64 shifts, both boundary conditions, and
the chain multi-shift solve -> force."""
import numpy as np
import pytest

import stag_synth as syn
from tests.gpu_common import lattice_with_links, links_np, log, pack, to_dev, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_5433_amd  # noqa: F401


def _random_solutions(dims, n, seed):
    rng = np.random.default_rng(seed)
    vh = int(np.prod(dims)) // 2
    return rng.standard_normal((n, vh, 3)) + 1j * rng.standard_normal((n, vh, 3))


def _max_rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("fmt", ["18", "12", "8", "18p", "12p"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 6, 4, 6), (16, 8, 8, 8)])
def test_force_vs_oracle(orc, dims, fmt):
    import torch
    log(f"force dims={dims} fmt={fmt}")
    U = links_np(dims, "smooth", 0.5, 21)
    lat = lattice_with_links(dims, U, fmt)
    for n, seed in ((1, 3), (5, 4)):
        X = _random_solutions(dims, n, seed)
        alphas = list(np.random.default_rng(seed).uniform(-2, 2, n))
        F = lat.fermion_force(alphas, [pack(lat, x) for x in X])
        torch.cuda.synchronize()
        ref = orc.fermion_force(dims, U, alphas, X)
        assert _max_rel(F.cpu().numpy(), ref) <= 1e-12, (n, _max_rel(F.cpu().numpy(), ref))


def test_force_full_size(orc):
    """The force at the benchmark's shape: 32^4, 8-real links, 16 shifts,
    element by element against the oracle."""
    import torch
    dims = (32, 32, 32, 32)
    log("force 32^4, 16 shifts, 8-real links")
    U = links_np(dims, "smooth", 0.5, 301)
    lat = lattice_with_links(dims, U, "8")
    X = _random_solutions(dims, 16, 7)
    alphas = list(np.random.default_rng(8).uniform(0.1, 2, 16))
    F = lat.fermion_force(alphas, [pack(lat, x) for x in X])
    torch.cuda.synchronize()
    ref = orc.fermion_force(dims, U, alphas, X)
    e = _max_rel(F.cpu().numpy(), ref)
    log(f"  largest entry error {e:.2e}")
    assert e <= 1e-12


@pytest.mark.parametrize("antiperiodic", [True, False])
def test_force_boundary_and_64_shifts(orc, antiperiodic):
    import torch
    dims = (4, 2, 4, 6)
    log(f"force 64 shifts antiperiodic={antiperiodic}")
    U = syn.haar_links(dims, 9)
    lat = lattice_with_links(dims, U, "18", antiperiodic)
    X = _random_solutions(dims, 64, 5)
    alphas = list(np.linspace(0.1, 3.0, 64))
    F = lat.fermion_force(alphas, [pack(lat, x) for x in X])
    torch.cuda.synchronize()
    ref = orc.fermion_force(dims, U, alphas, X, antiperiodic_t=antiperiodic)
    assert _max_rel(F.cpu().numpy(), ref) <= 1e-12


def test_force_from_multishift_solutions(orc):
    """The chain of the molecular dynamics: multi-shift solve, then the force
    from its solutions, against the oracle's force from the oracle's solves."""
    import torch
    dims = (8, 8, 4, 4)
    log("force after a multi-shift solve")
    U = links_np(dims, "smooth", 0.5, 23)
    lat = lattice_with_links(dims, U, "12")
    phi = syn.gaussian_source(dims, 12)
    mass, shifts, alphas = 0.1, [1e-3, 0.05, 0.8], [0.3, 0.9, 1.7]
    sols, rc, st = lat.multishift_cg(mass, shifts, pack(lat, phi), tol=1e-12)
    assert rc == 0
    F = lat.fermion_force(alphas, sols)
    torch.cuda.synchronize()
    xo, rco, io = orc.multishift_cg(dims, U, mass, shifts, phi, tol=1e-12)
    ref = orc.fermion_force(dims, U, alphas, xo)
    assert _max_rel(F.cpu().numpy(), ref) <= 1e-9
    # traceless anti-Hermitian on every link
    f = F.cpu().numpy()
    assert np.abs(f + np.conj(np.swapaxes(f, -1, -2))).max() <= 1e-13 * np.abs(f).max()
    assert np.abs(np.trace(f, axis1=-2, axis2=-1)).max() <= 1e-13 * np.abs(f).max()


def test_force_edge_cases():
    import torch
    import paper_1010_5433_amd as stag
    dims = (4, 4, 2, 2)
    log("force edge cases")
    U = links_np(dims, "smooth", 0.5, 2)
    lat = lattice_with_links(dims, U)
    out = torch.full((4, lat.V, 3, 3), 7.0, dtype=torch.complex128, device="cuda")
    lat.fermion_force([], [], out=out)
    torch.cuda.synchronize()
    assert not bool(out.abs().max())
    X = [pack(lat, x) for x in _random_solutions(dims, 65, 1)]
    with pytest.raises(stag.StagError):
        lat.fermion_force([1.0] * 65, X)
    with pytest.raises(stag.StagError):
        lat.fermion_force([float("nan")], X[:1])
    with pytest.raises(ValueError):
        lat.fermion_force([1.0, 2.0], X[:1])
    big = torch.zeros((4, lat.V, 3, 3), dtype=torch.complex128, device="cuda")
    alias = big.view(torch.float64).view(-1)[: 3 * lat.Vh * 2].view(3, lat.Vh, 2)
    with pytest.raises(stag.StagError):
        lat.fermion_force([1.0], [alias], out=big)
    # a solution lying inside the force buffer at an offset
    inner = big.view(torch.float64).view(-1)[40: 40 + 3 * lat.Vh * 2].view(3, lat.Vh, 2)
    with pytest.raises(stag.StagError):
        lat.fermion_force([1.0], [inner], out=big)
    bare = stag.Lattice(dims)
    with pytest.raises(stag.StagError):
        bare.fermion_force([1.0], X[:1])
