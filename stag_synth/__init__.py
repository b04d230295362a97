"""Seeded synthetic inputs for the staggered even/odd solver.

This module is shared by the FP64 CPU oracle and by the HIP path; it holds
random draws only (gauge links, sources, shift lists) and none of the
operator or solver arithmetic.  Everything is a pure function of its seed.

Layouts (the "canonical" layout both sides agree on):
  links   : complex128 array (4, V, 3, 3), indexed [mu][lex][row][col]
            where lex = x0 + L0*(x1 + L1*(x2 + L2*x3)), mu = 0..3 = x, y, z, t.
  vectors : complex128 array (V/2, 3), indexed [eo][colour] on one parity.

The paper's thermalised ensembles (Section 7) are not available; the two
generators below stand in for them:
  * haar_links   : independent Haar-random SU(3) links (a "hot start"),
  * smooth_links : U = exp(i*eps*H) with H a Gaussian traceless Hermitian
                   matrix per link, projected back onto SU(3).  eps = 0.5
                   gives fields with plaquette well above zero, closer to a
                   thermalised configuration than Haar noise.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "haar_su3", "haar_links", "smooth_links", "gaussian_source",
    "gaussian_sources", "logspace_shifts", "su3_project", "CONFIGS",
    "config", "gell_mann",
]


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def _complex_gaussian(rng: np.random.Generator, shape, var: float = 1.0):
    """Complex Gaussian with E|z|^2 = var; real part drawn first, then imaginary."""
    s = np.sqrt(var / 2.0)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * s


def haar_su3(n: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, shape (n, 3, 3).

    Mezzadri's recipe (Notices AMS 54 (2007) 592): QR of a complex Gaussian
    matrix with the phases of diag(R) moved into Q gives Haar U(3); dividing
    by the principal cube root of the determinant lands in SU(3).
    """
    z = _complex_gaussian(rng, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q * np.exp(-1j * np.angle(det) / 3.0)[:, None, None]
    return q


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j; l[1, 1, 0] = 1j
    l[2, 0, 0] = 1; l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j; l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j; l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3); l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def su3_project(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): an SU(3) matrix."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def haar_links(dims, seed: int) -> np.ndarray:
    """Haar-random SU(3) gauge field, canonical layout (4, V, 3, 3)."""
    v = volume(dims)
    rng = np.random.default_rng(seed)
    return haar_su3(4 * v, rng).reshape(4, v, 3, 3)


def smooth_links(dims, eps: float, seed: int, chunk: int = 1 << 20) -> np.ndarray:
    """U = SU(3)-projected exp(i*eps*H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1).

    The exponential is taken through the eigen-decomposition of H.  Drawn in
    chunks of links so that large lattices stay within memory.
    """
    v = volume(dims)
    n = 4 * v
    rng = np.random.default_rng(seed)
    lam = gell_mann() / 2.0
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        h = rng.standard_normal((e - s, 8))
        H = np.einsum("na,aij->nij", h, lam)
        w, vec = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        u = np.einsum("nik,nk,njk->nij", vec, ph, vec.conj())
        out[s:e] = su3_project(u)
    return out.reshape(4, v, 3, 3)


def gaussian_source(dims, seed: int) -> np.ndarray:
    """One even-site colour vector (V/2, 3); Re, Im i.i.d. N(0, 1/2)."""
    vh = volume(dims) // 2
    rng = np.random.default_rng(seed)
    return _complex_gaussian(rng, (vh, 3))


def gaussian_sources(dims, seed: int, count: int) -> np.ndarray:
    """`count` even-site sources (count, V/2, 3) from one stream."""
    vh = volume(dims) // 2
    rng = np.random.default_rng(seed)
    return _complex_gaussian(rng, (count, vh, 3))


def logspace_shifts(lo: float, hi: float, n: int) -> np.ndarray:
    return np.logspace(np.log10(lo), np.log10(hi), n)


# The five workloads.  Sizes, masses and shift ranges follow the problem
# statement; seeds are fixed here once and for all.
CONFIGS = {
    "c1_4x4x4x4_haar": dict(
        dims=(4, 4, 4, 4), links=("haar", None, 101), mass=0.1,
        shifts=(1e-4, 1.0, 8), source_seed=102, tol=1e-10, prec="f64"),
    "c2_32x32x32x8_smooth": dict(
        dims=(32, 32, 32, 8), links=("smooth", 0.5, 201), mass=0.02,
        shifts=(1e-5, 2.0, 12), source_seed=202, tol=1e-10, prec="f64"),
    "c3_32x32x32x32_smooth": dict(
        dims=(32, 32, 32, 32), links=("smooth", 0.5, 301), mass=0.01,
        shifts=(1e-6, 4.0, 16), source_seed=302, tol=1e-10, prec="mixed"),
    "c4_batched": dict(
        systems=[
            dict(dims=(24, 24, 24, 6), links=("smooth", 0.5, 400), mass=0.02,
                 shifts=(1e-5, 2.0, 16), source_seeds=tuple(range(401, 409))),
            dict(dims=(8, 8, 8, 8), links=("smooth", 0.5, 411), mass=0.05,
                 shifts=(1e-4, 1.0, 8), source_seeds=(421,)),
            dict(dims=(12, 12, 12, 12), links=("smooth", 0.5, 412), mass=0.05,
                 shifts=(1e-4, 1.0, 8), source_seeds=(422,)),
            dict(dims=(16, 16, 16, 8), links=("smooth", 0.5, 413), mass=0.05,
                 shifts=(1e-4, 1.0, 8), source_seeds=(423,)),
        ], tol=1e-10, prec="mixed"),
    "c5_learned": dict(
        train_dims=(16, 16, 16, 16), test_dims=(32, 32, 32, 32), eps=0.5,
        mass=0.01, shift=0.0, train_link_seeds=tuple(range(500, 516)),
        sources_per_field=256, train_source_seed=600,
        test_link_seeds=(550, 551, 552, 553), test_source_seed=650, tol=1e-10),
}


def config(name: str) -> dict:
    return CONFIGS[name]


def make_links(spec, dims) -> np.ndarray:
    kind, eps, seed = spec
    if kind == "haar":
        return haar_links(dims, seed)
    if kind == "smooth":
        return smooth_links(dims, eps, seed)
    raise ValueError(kind)
