"""Pin of the oracle's geometry tables (orc_tables) against an independent
NumPy construction from coordinates.

The tables follow the site conventions of the operator (the paper prints
none; the textbook staggered definitions are used): lex = x0 + L0*(x1 +
L1*(x2 + L2*x3)), parity = sum of coordinates mod 2, eo = lex >> 1, eight
hops d = +x,+y,+z,+t,-x,-y,-z,-t, the sign of forward hop mu at x is
eta_mu(x) s_mu(x) and of backward hop mu is eta_mu(x) s_mu(x - mu), with
s_mu(y) = -1 exactly when mu is time, the time boundary is antiperiodic and
y sits on the last time slice (the link from y3 = L3-1 to y3 = 0).

Here every entry is rebuilt from tests/lattice_np.py (coordinates in
lexicographic order, periodic shifts of the whole coordinate array) and the
boundary sign is read off the coordinates of the site the link starts
from, so a slip in the oracle's slot order, neighbour wrap, eta range or
boundary placement shows up as a mismatch."""
import numpy as np
import pytest

from tests import lattice_np as ln

LATTICES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 4), (6, 4, 2, 8), (2, 6, 4, 2), (8, 2, 2, 6)]


def numpy_tables(dims, antiperiodic):
    L = [int(d) for d in dims]
    V = int(np.prod(L))
    vh = V // 2
    X = ln.coords(dims)
    par = ln.parity(X)
    nbr = np.zeros((2, 8, vh), np.int32)
    coord = np.zeros((2, vh, 4), np.int32)
    sign = np.zeros((2, 8, vh), np.int32)
    for p in (0, 1):
        sites = np.nonzero(par == p)[0]          # lex order
        # lex >> 1 enumerates each parity's sites exactly once, in lex order
        assert np.array_equal(sites >> 1, np.arange(vh))
        coord[p] = X[sites]
        for mu in range(4):
            fw = ln.shifted_lex(dims, mu, +1)[sites]
            bw = ln.shifted_lex(dims, mu, -1)[sites]
            nbr[p, mu] = fw >> 1
            nbr[p, 4 + mu] = bw >> 1
            eta = np.where(X[sites, :mu].sum(axis=1) % 2 == 1, -1, 1)

            def s(start):   # sign carried by the link U_mu(start)
                last = X[start, 3] == L[3] - 1
                return np.where(antiperiodic and mu == 3, np.where(last, -1, 1), 1)

            sign[p, mu] = eta * s(sites)
            sign[p, 4 + mu] = eta * s(bw)
    return nbr, coord, sign


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("antiperiodic", [True, False])
def test_tables_match_numpy_geometry(orc, dims, antiperiodic):
    onbr, ocoord, osign = orc.tables(dims, antiperiodic)
    nbr, coord, sign = numpy_tables(dims, antiperiodic)
    assert np.array_equal(ocoord, coord)
    assert np.array_equal(onbr, nbr)
    assert np.array_equal(osign, sign)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 8)])
def test_time_boundary_sign_flip(orc, dims):
    """The antiperiodic boundary flips exactly the forward time hops that
    leave the last time slice and the backward time hops that leave the
    first one; the periodic tables have no flip at all."""
    _, coord, s_ap = orc.tables(dims, True)
    _, _, s_p = orc.tables(dims, False)
    L3 = dims[3]
    for p in (0, 1):
        x3 = coord[p, :, 3]
        flip = s_ap[p] * s_p[p]            # -1 where the boundary acts
        expect = np.ones_like(flip)
        expect[3, x3 == L3 - 1] = -1
        expect[7, x3 == 0] = -1
        assert np.array_equal(flip, expect)
        # eta_0 = 1 everywhere: the x hops carry no phase
        assert np.all(s_p[p, 0] == 1) and np.all(s_p[p, 4] == 1)


def test_neighbours_are_mutual(orc):
    """Forward hop mu from (p, i) lands on (1-p, j) whose backward hop mu
    returns to i: the two slots describe the same link, so they carry the
    same sign (eta_mu does not depend on x_mu)."""
    dims = (6, 4, 2, 8)
    nbr, _, sign = orc.tables(dims, True)
    for p in (0, 1):
        for mu in range(4):
            j = nbr[p, mu]
            assert np.array_equal(nbr[1 - p, 4 + mu][j], np.arange(len(j)))
            assert np.array_equal(sign[1 - p, 4 + mu][j], sign[p, mu])
