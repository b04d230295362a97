"""Test-side lattice helpers in NumPy (written independently of the oracle's
C code and of the HIP path): coordinates, parities and site maps used to
build plane waves, gauge transformations and translations."""
import numpy as np


def coords(dims):
    """(V, 4) coordinates in lexicographic order, x0 fastest."""
    L = [int(d) for d in dims]
    g = np.meshgrid(*[np.arange(l) for l in L], indexing="ij")
    # lex = x0 + L0*(x1 + L1*(x2 + L2*x3)): x0 fastest -> Fortran order
    return np.stack([a.ravel(order="F") for a in g], axis=1)


def lex_of(x, dims):
    L = [int(d) for d in dims]
    return x[..., 0] + L[0] * (x[..., 1] + L[1] * (x[..., 2] + L[2] * x[..., 3]))


def parity(x):
    return x.sum(axis=-1) % 2


def sites_of_parity(dims, p):
    """Lexicographic indices of the sites of parity p, in eo order."""
    x = coords(dims)
    return np.nonzero(parity(x) == p)[0]


def shifted_lex(dims, mu, step):
    """lex index of x + step*mu-hat for every lex site x (periodic)."""
    x = coords(dims).copy()
    x[:, mu] = (x[:, mu] + step) % int(dims[mu])
    return lex_of(x, dims)


def embed(dims, p, v):
    """eo vector on parity p -> full-lattice (V,3) vector, zero elsewhere."""
    full = np.zeros((int(np.prod(dims)), 3), np.complex128)
    full[sites_of_parity(dims, p)] = v
    return full


def restrict(dims, p, full):
    return full[sites_of_parity(dims, p)]


def plane_wave(dims, n, colour, antiperiodic_t=True):
    """exp(i p.x) * colour on every site, p_mu = 2 pi n_mu / L_mu, with
    p_3 = 2 pi (n_3 + 1/2) / L_3 for antiperiodic time."""
    L = np.array(dims, float)
    p = 2 * np.pi * np.array(n, float) / L
    if antiperiodic_t:
        p[3] = 2 * np.pi * (n[3] + 0.5) / L[3]
    x = coords(dims)
    ph = np.exp(1j * (x @ p))
    return ph[:, None] * np.asarray(colour)[None, :], p


def free_links(dims):
    V = int(np.prod(dims))
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()


def gauge_transform(dims, links, omega):
    """U'_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^dag."""
    out = np.empty_like(links)
    for mu in range(4):
        fwd = shifted_lex(dims, mu, +1)
        out[mu] = omega @ links[mu] @ np.conj(np.swapaxes(omega[fwd], -1, -2))
    return out


def dense_normal_matrix(apply, n):
    """Columns of an operator applied to unit vectors (n = 3 V/2)."""
    M = np.zeros((n, n), np.complex128)
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1.0
        M[:, k] = apply(e.reshape(-1, 3)).ravel()
    return M
