"""Pins of the FP64 oracle of the learned preconditioner.

  * special case: with weights that pick +-1/2 on forward/backward hops the
    network is exactly M = m^2 - D_eo D_oe, computed by the independently
    pinned operator oracle   -> hop definitions, eta, boundary, daggers
  * gauge equivariance P[U^Omega](Omega r) = Omega P[U](r)
  * linearity in r
  * central finite differences of Re <g, P(r)> against the analytic gradient
    (relative error <= 1e-7)        -> every backward term
"""
import numpy as np
import pytest

import stag_synth as syn
from tests import lattice_np as ln

NP = 656
W1S, W1H, W2, WOUT = 0, 8, 72, 648


def rand_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(NP) + 1j * rng.standard_normal(NP))


def normal_op_theta(mass):
    """Weights that make P = M = m^2 - D_eo D_oe (channel 0 only)."""
    th = np.zeros(NP, np.complex128)
    th[W1S + 0] = 1.0
    for d in range(8):
        th[W1H + 8 * 0 + d] = 0.5 if d < 4 else -0.5            # phi1 = D_oe r
    th[W2 + 72 * 0 + 0] = mass * mass                             # self: m^2 r
    for d in range(8):
        th[W2 + 72 * 0 + 8 + 8 * d + 0] = -(0.5 if d < 4 else -0.5)  # - D_eo phi1
    th[WOUT + 0] = 1.0
    return th


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 2), (6, 4, 2, 8)])
def test_net_reduces_to_normal_operator(orc, dims):
    U = syn.haar_links(dims, 3)
    r = syn.gaussian_source(dims, 4)
    m = 0.2
    got = orc.net_forward(dims, U, normal_op_theta(m), r)
    want = orc.normal_op(dims, U, m, 0.0, r)
    assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want)


def test_net_layer1_is_dslash(orc):
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 5)
    r = syn.gaussian_source(dims, 6)
    th = normal_op_theta(0.1)
    phi1 = orc.net_layer1_odd(dims, U, th, r)
    want = orc.dslash_eo(dims, U, 1, r)
    assert np.linalg.norm(phi1[:, 0, :] - want) <= 1e-14 * np.linalg.norm(want)
    assert np.max(np.abs(phi1[:, 1:, :])) == 0.0


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_net_gauge_equivariant(orc, dims):
    rng = np.random.default_rng(9)
    V = int(np.prod(dims))
    U = syn.haar_links(dims, 7)
    omega = syn.haar_su3(V, rng)
    Ug = ln.gauge_transform(dims, U, omega)
    ev = ln.sites_of_parity(dims, 0)
    r = syn.gaussian_source(dims, 8)
    th = rand_theta(10)
    lhs = orc.net_forward(dims, Ug, th, np.einsum("nij,nj->ni", omega[ev], r))
    rhs = np.einsum("nij,nj->ni", omega[ev], orc.net_forward(dims, U, th, r))
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_net_linear_in_input(orc):
    dims = (4, 4, 4, 4)
    U = syn.haar_links(dims, 1)
    th = rand_theta(2)
    a, b = syn.gaussian_source(dims, 3), syn.gaussian_source(dims, 4)
    lhs = orc.net_forward(dims, U, th, (2 - 1j) * a + 0.5 * b)
    rhs = (2 - 1j) * orc.net_forward(dims, U, th, a) + 0.5 * orc.net_forward(dims, U, th, b)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_net_gradient_finite_differences(orc, dims):
    U = syn.haar_links(dims, 11)
    r = syn.gaussian_source(dims, 12)
    g = syn.gaussian_source(dims, 13)
    th = rand_theta(14)
    grad = orc.net_backward(dims, U, th, r, g)

    def L(t):
        return float(np.real(np.vdot(g, orc.net_forward(dims, U, t, r))))

    rng = np.random.default_rng(15)
    idx = list(range(0, 8)) + list(range(8, 72, 5)) + list(rng.choice(np.arange(72, 648), 40, replace=False)) \
        + list(range(648, 656))
    h = 1e-6
    worst = 0.0
    for j in idx:
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            tp, tm = th.copy(), th.copy()
            tp[j] += h * unit
            tm[j] -= h * unit
            fd = (L(tp) - L(tm)) / (2 * h)
            an = part(grad[j])
            worst = max(worst, abs(fd - an) / max(1e-8, np.max(np.abs(grad))))
    assert worst <= 1e-7, worst
