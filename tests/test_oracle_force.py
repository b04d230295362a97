"""Pins of the oracle's pseudo-fermion force against the derivative of the
action it belongs to, taken by central finite differences.

The action S(U) = sum_i alpha_i <phi, (M + sigma_i)^-1 phi> is evaluated by
dense direct solves of the oracle's normal operator on lattices of 64-128
sites; each link is moved along U -> exp(i eps T) U with a random traceless
Hermitian T, and (S(+eps) - S(-eps)) / (2 eps) must equal i tr(T F).  A
wrong sign, a dropped end of the link, a swapped outer product, a missing
phase or boundary sign, or the wrong U factor moves the analytic value away
from the difference quotient by O(1), far outside the O(eps^2) truncation.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import stag_synth as syn

MASS = 0.3
SHIFTS = [0.0, 0.1, 1.0]
ALPHAS = [0.5, 0.2, 1.3]


def _dense_m(orc, dims, U, antiperiodic):
    vh = int(np.prod(dims)) // 2
    n = 3 * vh
    M = np.empty((n, n), np.complex128)
    for k in range(n):
        e = np.zeros((vh, 3), np.complex128)
        e.flat[k] = 1.0
        M[:, k] = orc.normal_op(dims, U, MASS, 0.0, e, antiperiodic_t=antiperiodic).ravel()
    return M


def _solutions(orc, dims, U, phi, antiperiodic):
    M = _dense_m(orc, dims, U, antiperiodic)
    return np.stack([np.linalg.solve(M + sg * np.eye(M.shape[0]), phi.ravel()).reshape(-1, 3)
                     for sg in SHIFTS])


def _action(orc, dims, U, phi, antiperiodic):
    X = _solutions(orc, dims, U, phi, antiperiodic)
    return sum(a * np.vdot(phi.ravel(), x.ravel()).real for a, x in zip(ALPHAS, X))


def _random_generator(rng):
    lam = syn.gell_mann()
    c = rng.standard_normal(8)
    return np.einsum("k,kab->ab", c, lam) / 2


@pytest.mark.parametrize("dims", [(4, 2, 2, 4), (2, 4, 4, 2)])
@pytest.mark.parametrize("antiperiodic", [True, False])
def test_force_is_the_action_derivative(orc, dims, antiperiodic):
    rng = np.random.default_rng(11)
    U = syn.haar_links(dims, 5)
    V = int(np.prod(dims))
    phi = syn.gaussian_source(dims, 3)
    X = _solutions(orc, dims, U, phi, antiperiodic)
    F = orc.fermion_force(dims, U, ALPHAS, X, antiperiodic_t=antiperiodic)
    eps = 1e-4
    # every direction, sites of both parities, and the last time slice
    # (where the antiperiodic sign sits)
    sites = [0, 1, V - 1, V - 2, int(rng.integers(V))]
    for mu in range(4):
        for lex in sites:
            T = _random_generator(rng)
            Up, Um = U.copy(), U.copy()
            Up[mu, lex] = sla.expm(1j * eps * T) @ U[mu, lex]
            Um[mu, lex] = sla.expm(-1j * eps * T) @ U[mu, lex]
            fd = (_action(orc, dims, Up, phi, antiperiodic) - _action(orc, dims, Um, phi, antiperiodic)) / (2 * eps)
            an = 1j * np.trace(T @ F[mu, lex])
            assert abs(an.imag) <= 1e-12 * max(1.0, abs(an.real))
            assert abs(an.real - fd) <= 1e-6 * max(1.0, abs(fd)), (mu, lex, an.real, fd)


def test_force_is_in_the_algebra_and_linear_in_alpha(orc):
    """Traceless anti-Hermitian at every link; zero for no shifts; the sum of
    the single-shift forces (each weighted by its alpha) for several."""
    dims = (4, 4, 2, 2)
    U = syn.haar_links(dims, 8)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((3, int(np.prod(dims)) // 2, 3)) + 1j * rng.standard_normal((3, int(np.prod(dims)) // 2, 3))
    F = orc.fermion_force(dims, U, ALPHAS, X)
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() <= 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() <= 1e-14
    parts = sum(orc.fermion_force(dims, U, [a], X[i:i + 1]) for i, a in enumerate(ALPHAS))
    assert np.abs(F - parts).max() <= 1e-13 * np.abs(F).max()
    assert not np.any(orc.fermion_force(dims, U, [], X[:0]))
