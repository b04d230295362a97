"""Pins of the rational-function application (the RHMC's heatbath and
Metropolis action, Section 2) and of the Zolotarev coefficient generator.

  * oracle r(M) b = alpha0 b + sum_i alpha_i (M + s_i)^-1 b:
      - free field: plane waves are eigenvectors, so r(M) acts on each as
        the scalar r(lambda_p)                          -> closed form
      - dense direct solves on small Haar lattices       -> brute force
      - Zolotarev coefficients for x^(-1/2) reproduce M^(-1/2) b from the
        dense eigen-decomposition within the approximation error
  * Zolotarev generator (host code of the library, no GPU): the relative
    error alternates in sign 2n + 1 times with equal magnitude (Chebyshev's
    alternation theorem: the best approximation of its type), the claimed
    error is the observed maximum, poles are negative reals and residues
    positive.
"""
import numpy as np
import pytest

import stag_synth as syn
from tests import lattice_np as ln


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _zolotarev(power, lo, hi, n):
    import paper_1010_5433_amd as stag
    return stag.zolotarev(power, lo, hi, n)


@pytest.mark.parametrize("B,n", [(1e2, 4), (1e4, 8), (1.6e5, 12), (1e6, 16), (1e6, 24)])
def test_zolotarev_alternation(B, n):
    a0, al, sh, err = _zolotarev(-1, 0.5, 0.5 * B, n)
    assert a0 == 0.0
    assert all(a > 0 for a in al) and all(s > 0 for s in sh)
    assert all(s1 < s2 for s1, s2 in zip(sh, sh[1:]))
    x = 0.5 * np.exp(np.linspace(0.0, np.log(B), 200001))
    e = (a0 + sum(a / (x + s) for a, s in zip(al, sh))) * np.sqrt(x) - 1.0
    emax = np.abs(e).max()
    assert abs(emax - err) <= 1e-3 * err + 1e-15
    # alternation: among the points where |e| > err / 2 (away from the zeros,
    # where rounding could flip signs) the sign changes exactly 2n times, and
    # every run reaches err
    big = np.abs(e) > 0.5 * err
    sg, eb = np.sign(e[big]), e[big]
    cut = np.where(np.diff(sg) != 0)[0] + 1
    assert len(cut) == 2 * n
    peaks = np.array([np.abs(r).max() for r in np.split(eb, cut)])
    assert peaks.min() >= 0.995 * err
    # more poles, smaller error
    if n > 4:
        assert err < _zolotarev(-1, 0.5, 0.5 * B, n - 4)[3]


@pytest.mark.parametrize("B,n", [(1e4, 8), (1e6, 16)])
def test_zolotarev_square_root_form(B, n):
    """x^(1/2) = x * x^(-1/2): same poles, same relative error."""
    a0, al, sh, err = _zolotarev(1, 2.0, 2.0 * B, n)
    b0, bl, th, err_m = _zolotarev(-1, 2.0, 2.0 * B, n)
    assert np.allclose(sh, th, rtol=0, atol=0)
    x = 2.0 * np.exp(np.linspace(0.0, np.log(B), 100001))
    e = (a0 + sum(a / (x + s) for a, s in zip(al, sh))) / np.sqrt(x) - 1.0
    assert abs(np.abs(e).max() - err_m) <= 1e-3 * err_m + 1e-12
    assert a0 > 0 and all(a < 0 for a in al)


def _alternations(power, lo, hi, a0, al, sh, npts=200001):
    x = lo * np.exp(np.linspace(0.0, np.log(hi / lo), npts))
    e = (a0 + sum(a / (x + s) for a, s in zip(al, sh))) / x ** power - 1.0
    emax = np.abs(e).max()
    big = np.abs(e) > 0.5 * emax
    sg, eb = np.sign(e[big]), e[big]
    cut = np.where(np.diff(sg) != 0)[0] + 1
    peaks = np.array([np.abs(r).max() for r in np.split(eb, cut)])
    return emax, len(cut), peaks.min() / emax


@pytest.mark.parametrize("power", [0.25, -0.25, 0.125, -0.75, -0.375])
@pytest.mark.parametrize("n", [8, 14, 20])
def test_rational_power_alternation(power, n):
    """Remez's result for other powers: 2n sign changes between equal peaks
    (the alternation certificate of the best approximation of its type), the
    claimed error is the observed one, and the sign pattern of the residues
    matches the function (x^-p: positive residues, alpha0 = 0; x^q: alpha0 > 0,
    negative residues)."""
    import paper_1010_5433_amd as stag
    lo, hi = 1e-4, 16.0001
    a0, al, sh, err = stag.rational_power(power, lo, hi, n)
    emax, nalt, spread = _alternations(power, lo, hi, a0, al, sh)
    assert nalt == 2 * n
    assert spread >= 0.995
    assert abs(emax - err) <= 1e-2 * err
    assert all(s > 0 for s in sh)
    if power < 0:
        assert a0 == 0.0 and all(a > 0 for a in al)
    else:
        assert a0 > 0 and all(a < 0 for a in al)
    if n > 8:
        assert err < stag.rational_power(power, lo, hi, n - 6)[3]


def test_rational_power_half_is_zolotarev():
    import paper_1010_5433_amd as stag
    assert stag.rational_power(-0.5, 0.01, 5.0, 10) == stag.zolotarev(-1, 0.01, 5.0, 10)
    with pytest.raises(stag.StagError):
        stag.rational_power(0.0, 0.01, 5.0, 10)
    with pytest.raises(stag.StagError):
        stag.rational_power(1.0, 0.01, 5.0, 10)
    with pytest.raises(stag.StagError):
        stag.rational_power(0.25, 0.01, 5.0, 30)


def test_zolotarev_rejects_bad_arguments():
    import paper_1010_5433_amd as stag
    for args in [(0, 1.0, 2.0, 4), (-1, 0.0, 2.0, 4), (-1, 2.0, 1.0, 4), (-1, 1.0, 2.0, 0), (-1, 1.0, 2.0, 65)]:
        with pytest.raises(stag.StagError):
            stag.zolotarev(*args)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_rational_free_field_closed_form(orc, dims):
    rng = np.random.default_rng(23)
    m = 0.1
    ns = [tuple(int(rng.integers(0, d)) for d in dims) for _ in range(4)]
    waves, lams = [], []
    for n in ns:
        colour = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        full, p = ln.plane_wave(dims, n, colour)
        waves.append(ln.restrict(dims, 0, full))
        lams.append(m * m + np.sum(np.sin(p) ** 2))
    b = sum(waves)
    alpha0, alphas, shifts = 0.3, [0.7, -0.2, 1.5], [0.0, 0.4, 2.5]
    out, rc, info = orc.rational_apply(dims, ln.free_links(dims), m, alpha0, alphas, shifts, b, tol=1e-13)
    assert rc == 0
    want = sum(w * (alpha0 + sum(a / (lam + s) for a, s in zip(alphas, shifts))) for w, lam in zip(waves, lams))
    assert rel(out, want) <= 1e-12
    assert abs(info["dot"] - np.vdot(b, want).real) <= 1e-12 * abs(np.vdot(b, want).real)


@pytest.mark.parametrize("dims,seed", [((2, 2, 2, 2), 3), ((4, 2, 2, 4), 8)])
def test_rational_dense(orc, dims, seed):
    U = syn.haar_links(dims, seed)
    m = 0.2
    vh = int(np.prod(dims)) // 2
    b = syn.gaussian_source(dims, seed + 1)
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, m, 0.0, v), 3 * vh)
    alpha0, alphas, shifts = -0.4, [1.0, 0.25, -0.6, 2.0], [0.0, 0.01, 0.3, 5.0]
    tol = 1e-11
    out, rc, info = orc.rational_apply(dims, U, m, alpha0, alphas, shifts, b, tol=tol)
    assert rc == 0
    bb = b.ravel()
    want = alpha0 * bb + sum(a * np.linalg.solve(M + s * np.eye(3 * vh), bb) for a, s in zip(alphas, shifts))
    # error bound: tol ||b|| sum |alpha_i| / (m^2 + s_i), plus rounding
    bound = tol * np.linalg.norm(bb) * sum(abs(a) / (m * m + s) for a, s in zip(alphas, shifts))
    assert np.linalg.norm(out.ravel() - want) <= 2 * bound + 1e-13 * np.linalg.norm(want)


def test_rational_zolotarev_inverse_square_root(orc):
    """r(M) b with Zolotarev's x^(-1/2) on [m^2, m^2 + 16] (the spectrum of M
    lies there: |D_hop| <= 4) equals M^(-1/2) b from the dense
    eigen-decomposition within the approximation error."""
    dims = (4, 4, 2, 2)
    U = syn.haar_links(dims, 31)
    m = 0.1
    vh = int(np.prod(dims)) // 2
    b = syn.gaussian_source(dims, 32)
    M = ln.dense_normal_matrix(lambda v: orc.normal_op(dims, U, m, 0.0, v), 3 * vh)
    w, V = np.linalg.eigh(M)
    assert w[0] >= m * m - 1e-12 and w[-1] <= m * m + 16
    bb = b.ravel()
    exact = V @ ((V.conj().T @ bb) / np.sqrt(w))
    a0, al, sh, err = _zolotarev(-1, m * m, m * m + 16.0, 16)
    out, rc, info = orc.rational_apply(dims, U, m, a0, al, sh, b, tol=1e-13)
    assert rc == 0
    assert rel(out.ravel(), exact) <= err + 1e-11
    action = np.vdot(bb, exact).real
    assert abs(info["dot"] - action) <= (err + 1e-11) * action
