"""CPU checks of the entrywise error bounds the GPU parity tests use
(tests/entrywise.py): the bounds hold for perturbations they claim to
cover, computed with the oracle alone, and are tight enough to catch a
single wrong entry."""
import numpy as np
import pytest

import stag_synth as syn
from tests import entrywise as ew
from tests import lattice_np as ln

DIMS = [(4, 4, 4, 4), (6, 4, 2, 8)]


def _round32(a):
    return a.real.astype(np.float32).astype(np.float64) + 1j * a.imag.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("dims", DIMS)
def test_magnitude_sum_dominates_the_operator(orc, dims):
    """|D v| <= abs_hop(|U|, |v|) entrywise: the magnitude sum visits the
    same neighbours and links as the operator."""
    U = syn.haar_links(dims, 3)
    v = syn.gaussian_source(dims, 4)
    for par in (0, 1):
        d = orc.dslash_eo(dims, U, par, v)
        s = ew.abs_hop(dims, np.abs(U), par, np.abs(v))
        assert np.all(np.abs(d) <= s * (1 + 1e-12))
        # and is not loose by more than the cancellation of 8 hops
        assert np.median(s / np.maximum(np.abs(d), 1e-300)) < 20


@pytest.mark.parametrize("dims", DIMS)
def test_single_precision_rounding_inside_the_bound(orc, dims):
    """Links and vector rounded to single precision, applied exactly (the
    oracle in FP64): the change stays inside the FP32 '18' bound with room
    left for the arithmetic."""
    U = syn.haar_links(dims, 5)
    v = syn.gaussian_source(dims, 6)
    for par in (0, 1):
        exact = orc.dslash_eo(dims, U, par, v)
        rounded = orc.dslash_eo(dims, _round32(U), par, _round32(v))
        bound = ew.dslash_bound(dims, U, "18", "f32", par, v)
        assert ew.check_entrywise(rounded, exact, bound, "f32 rounding") < 0.1


@pytest.mark.parametrize("dims", DIMS)
def test_two_row_rebuild_inside_the_bound(orc, dims):
    """Third rows rebuilt as conj(row0 x row1) from the stored rows: the
    change of the operator stays inside the FP64 '12' bound."""
    U = syn.smooth_links(dims, 0.5, 7)
    R = U.copy()
    R[..., 2, :] = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    v = syn.gaussian_source(dims, 8)
    for par in (0, 1):
        bound = ew.dslash_bound(dims, U, "12", "f64", par, v)
        ew.check_entrywise(orc.dslash_eo(dims, R, par, v), orc.dslash_eo(dims, U, par, v), bound, "12 rebuild")


def test_one_wrong_entry_is_caught(orc):
    """A single entry off by 1e-12 (far below the norm of the output, so a
    norm ratio of 1e-14 over 8^4 entries would hide it) fails the bound."""
    dims = (8, 8, 8, 8)
    U = syn.smooth_links(dims, 0.5, 9)
    v = syn.gaussian_source(dims, 10)
    want = orc.dslash_eo(dims, U, 0, v)
    got = want.copy()
    got[1234, 2] += 1e-12
    bound = ew.dslash_bound(dims, U, "18", "f64", 0, v)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-14
    with pytest.raises(AssertionError):
        ew.check_entrywise(got, want, bound, "planted")


@pytest.mark.parametrize("dims", DIMS)
def test_normal_op_bound_covers_rounded_links(orc, dims):
    """Normal operator on single precision rounded links and source against
    the exact one: inside the FP32 bound."""
    U = syn.smooth_links(dims, 0.5, 11)
    p = syn.gaussian_source(dims, 12)
    c = 0.02 ** 2 + 0.3
    exact = orc.normal_op(dims, U, 0.02, 0.3, p)
    rounded = orc.normal_op(dims, _round32(U), 0.02, 0.3, _round32(p))
    bound = ew.normal_op_bound(dims, U, "18", "f32", c, p)
    assert ew.check_entrywise(rounded, exact, bound, "normal op f32 rounding") < 0.1


def test_eight_real_delta_grows_near_vanishing_u00():
    """The 8-real rebuild takes |u00| from 1 - |u01|^2 - |u02|^2: its bound
    grows as 1/|u00| for links whose first entry is small."""
    dims = (2, 2, 2, 2)
    U = syn.haar_links(dims, 13)
    d = ew.link_delta(U, "8", "f32")
    u00 = np.abs(U[..., 0, 0])
    k = np.argmin(u00.ravel())
    assert d.ravel()[k] >= 8 * ew.EPS32 / u00.ravel()[k]
    assert np.all(ew.link_delta(ln.free_links(dims), "18", "f64") == 0)
