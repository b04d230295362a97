"""Entry-by-entry error bounds for comparing the HIP operators with the
FP64 oracle (NumPy, test side only).

A global norm ratio can hide a wrong slice of a large lattice (one
boundary plane of 32^4 is 3 % of the entries).  These helpers bound the
difference of every output entry instead, by the standard forward error
analysis of a sum of products: if out_a = sum_k t_k is evaluated in
floating point with unit roundoff e, |fl(out_a) - out_a| <= n e sum_k |t_k|.
For the hopping term
    (D v)_a(x) = 1/2 sum_mu [+-(U_mu(x) v(x+mu))_a +- (U_mu(x-mu)^dag v(x-mu))_a]
the magnitude sum is the same expression with every sign dropped and |U|,
|v| taken entrywise (abs_hop below).  A stored link format that rebuilds
entries (12 or 8 reals, float pairs, single precision) adds, per link, an
absolute entry error delta (link_delta below), which reaches the output
through the same hop with delta * ones(3, 3) in place of |U|.

Bounds used (e = unit roundoff of the kernel's arithmetic):
  * arithmetic, both sides together: gamma = 128 e of the magnitude sum
    (24 complex products per output entry, <= ~37 e each side);
  * links: delta per link, derived from the stored field itself:
      18 reals  : rounding of the stored entries (0 in FP64);
      12 reals  : + |conj(row0 x row1) - row2| (the field's own defect from
                  SU(3)) + 8 e for the rebuild;
      8 reals   : + the unitarity and determinant defect + 8 e (1 + 1/|u00|)
                  (|u00| = sqrt(1 - |u01|^2 - |u02|^2) loses e/|u00|);
      pairs     : + 2^-48 per entry in FP64 (a = hi + lo to 2^-48 |a|).
"""
import numpy as np

from tests import lattice_np as ln

EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24
GAMMA_MULT = 128


def unit_roundoff(prec):
    return EPS64 if prec == "f64" else EPS32


def abs_hop(dims, W, out_parity, vabs):
    """1/2 sum_mu [W_mu(x) vabs(x+mu) + W_mu(x-mu)^T vabs(x-mu)] for the
    sites x of out_parity (eo order).  W: (4, V, 3, 3) non-negative
    matrices, or (4, V) non-negative scalars standing for scalar * ones(3,3).
    vabs: (V/2, 3) non-negative, on the other parity."""
    V = int(np.prod(dims))
    sites = ln.sites_of_parity(dims, out_parity)
    full = np.zeros((V, 3))
    full[ln.sites_of_parity(dims, 1 - out_parity)] = vabs
    acc = np.zeros((len(sites), 3))
    scalar = W.ndim == 2
    for mu in range(4):
        fw = ln.shifted_lex(dims, mu, +1)[sites]
        bw = ln.shifted_lex(dims, mu, -1)[sites]
        if scalar:
            acc += (W[mu, sites] * full[fw].sum(axis=1))[:, None]
            acc += (W[mu, bw] * full[bw].sum(axis=1))[:, None]
        else:
            acc += np.einsum("sab,sb->sa", W[mu, sites], full[fw])
            acc += np.einsum("sba,sb->sa", W[mu, bw], full[bw])
    return 0.5 * acc


def link_delta(U, fmt, prec):
    """(4, V) bound on the absolute error of every link entry the kernel
    uses, for storage format fmt ('18', '12', '8', '18p', '12p') read in
    precision prec ('f64' or 'f32')."""
    e = unit_roundoff(prec)
    rows = fmt.rstrip("p")
    pairs = fmt.endswith("p")
    d = np.zeros(U.shape[:2])
    if prec == "f32":
        d += np.sqrt(2.0) * EPS32                       # stored entries rounded to single
    elif pairs:
        d += np.sqrt(2.0) * 2.0 ** -48                  # hi + lo
    if rows == "12":
        r2 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
        d += np.abs(r2 - U[..., 2, :]).max(axis=-1) + 8 * e
    elif rows == "8":
        eye = np.eye(3)
        uu = U @ np.conj(np.swapaxes(U, -1, -2))
        defect = np.maximum(np.abs(uu - eye).max(axis=(-1, -2)), np.abs(np.linalg.det(U) - 1.0))
        u00 = np.maximum(np.abs(U[..., 0, 0]), 1e-300)
        d += defect + 8 * e * (1.0 + 1.0 / u00)
    return d


def dslash_bound(dims, U, fmt, prec, out_parity, v):
    """Entrywise bound on |D_gpu v - D_oracle v| for the half hopping term."""
    gamma = GAMMA_MULT * unit_roundoff(prec)
    av = np.abs(v)
    return gamma * abs_hop(dims, np.abs(U), out_parity, av) + abs_hop(dims, link_delta(U, fmt, prec), out_parity, av)


def normal_op_bound(dims, U, fmt, prec, c, p):
    """Entrywise bound on the difference of (c p - D_eo D_oe p) between
    the kernel and the oracle: the first half's bound E_t propagates
    through the second half together with its own rounding."""
    gamma = GAMMA_MULT * unit_roundoff(prec)
    aU, dl = np.abs(U), link_delta(U, fmt, prec)
    ap = np.abs(p)
    s_t = abs_hop(dims, aU, 1, ap)
    e_t = gamma * s_t + abs_hop(dims, dl, 1, ap)
    t_mag = s_t + e_t
    return (gamma * abs(c) * ap + gamma * abs_hop(dims, aU, 0, t_mag) + abs_hop(dims, dl, 0, t_mag)
            + abs_hop(dims, aU, 0, e_t) + abs_hop(dims, dl, 0, e_t))


def check_entrywise(got, want, bound, what=""):
    """Every |got - want| within its bound; on failure report the worst
    entry (site, colour) and how many entries fail."""
    err = np.abs(got - want)
    bad = err > bound
    if bad.any():
        k = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {err.size} entries over their bound; worst at {k}: "
                             f"|diff| {err[k]:.3e} > bound {bound[k]:.3e}")
    return float((err / np.maximum(bound, 1e-300)).max())


def max_entry_err(got, want):
    """Largest entry error in units of the largest reference entry."""
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))
