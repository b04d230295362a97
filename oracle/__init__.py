"""Python access to the FP64 CPU oracle (liborc.so, built from orc.c).

TEST INFRASTRUCTURE.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark import this package; the library package never does.

All arrays are NumPy complex128 in the canonical layout:
  links (4, V, 3, 3) [mu][lex][row][col], vectors (V/2, 3) [eo][colour],
  full-lattice vectors (V, 3) [lex][colour].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
SOURCES = ("orc.c", "orc_net.c")

_c = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


def compile_sources(srcs, out_path):
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", out_path]
    subprocess.run(cmd + list(srcs) + ["-lm"], check=True)
    return out_path


def build(force: bool = True) -> str:
    """Compile the oracle sources into liborc.so with gcc + OpenMP."""
    srcs = [os.path.join(_HERE, f) for f in SOURCES if os.path.exists(os.path.join(_HERE, f))]
    if force or not os.path.exists(_LIB_PATH):
        compile_sources(srcs, _LIB_PATH)
    return _LIB_PATH


def _bind(L):
    L.orc_dhop_full.argtypes = [_c, _i, _c, _c, _c]
    L.orc_dslash_eo.argtypes = [_c, _i, _c, _i, _c, _c]
    L.orc_normal_op.argtypes = [_c, _i, _c, _d, _d, _c, _c]
    L.orc_tables.argtypes = [_c, _i, _c, _c, _c]
    L.orc_true_residual.argtypes = [_c, _i, _c, _d, _d, _c, _c]
    L.orc_true_residual.restype = _d
    L.orc_cg.argtypes = [_c, _i, _c, _d, _d, _c, _c, _d, _i, _c, _c, _c]
    L.orc_multishift_cg.argtypes = [_c, _i, _c, _d, _i, _c, _c, _c, _d, _i,
                                    _c, _c, _c, _c]
    L.orc_fermion_force.argtypes = [_c, _i, _c, _i, _c, _c, _c]
    for f in (L.orc_dhop_full, L.orc_dslash_eo, L.orc_normal_op, L.orc_tables,
              L.orc_cg, L.orc_multishift_cg, L.orc_fermion_force):
        f.restype = _i
    if hasattr(L, "orc_net_forward"):
        L.orc_net_forward.argtypes = [_c, _i, _c, _c, _c, _c]
        L.orc_net_layer1_odd.argtypes = [_c, _i, _c, _c, _c, _c]
        L.orc_net_backward.argtypes = [_c, _i, _c, _c, _c, _c, _c]
        L.orc_net_nparam.argtypes = []
        for f in (L.orc_net_forward, L.orc_net_layer1_odd, L.orc_net_backward, L.orc_net_nparam):
            f.restype = _i
    return L


def _dims(dims):
    return (ctypes.c_int * 4)(*[int(d) for d in dims])


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"{what}: oracle returned {rc}")
    return rc


class Oracle:
    """The oracle's entry points bound to one build of the library."""

    def __init__(self, L):
        self.L = L

    def dhop_full(self, dims, links, vec, antiperiodic_t=True):
        links, vec = _cplx(links), _cplx(vec)
        out = np.empty_like(vec)
        _check(self.L.orc_dhop_full(_dims(dims), int(antiperiodic_t), _p(links), _p(vec),
                                    _p(out)), "dhop_full")
        return out

    def dslash_eo(self, dims, links, out_parity, vec, antiperiodic_t=True):
        links, vec = _cplx(links), _cplx(vec)
        out = np.empty_like(vec)
        _check(self.L.orc_dslash_eo(_dims(dims), int(antiperiodic_t), _p(links),
                                    int(out_parity), _p(vec), _p(out)), "dslash_eo")
        return out

    def normal_op(self, dims, links, mass, shift, vec, antiperiodic_t=True):
        links, vec = _cplx(links), _cplx(vec)
        out = np.empty_like(vec)
        _check(self.L.orc_normal_op(_dims(dims), int(antiperiodic_t), _p(links), float(mass),
                                    float(shift), _p(vec), _p(out)), "normal_op")
        return out

    def tables(self, dims, antiperiodic_t=True):
        """(nbr [2,8,V/2], coord [2,V/2,4], sign [2,8,V/2]) as int32."""
        vh = int(np.prod(dims)) // 2
        nbr = np.zeros((2, 8, vh), np.int32)
        coord = np.zeros((2, vh, 4), np.int32)
        sign = np.zeros((2, 8, vh), np.int32)
        _check(self.L.orc_tables(_dims(dims), int(antiperiodic_t), _p(nbr), _p(coord),
                                 _p(sign)), "tables")
        return nbr, coord, sign

    def true_residual(self, dims, links, mass, shift, b, x, antiperiodic_t=True):
        links, b, x = _cplx(links), _cplx(b), _cplx(x)
        return self.L.orc_true_residual(_dims(dims), int(antiperiodic_t), _p(links),
                                        float(mass), float(shift), _p(b), _p(x))

    def cg(self, dims, links, mass, shift, b, x0=None, tol=1e-10, max_iter=10000,
           antiperiodic_t=True):
        """Single-shift CG from x0 (zero if None). Returns (x, status, info)."""
        links, b = _cplx(links), _cplx(b)
        x = np.zeros_like(b) if x0 is None else _cplx(x0).copy()
        it = ctypes.c_int(0)
        ri, rt = ctypes.c_double(0), ctypes.c_double(0)
        rc = _check(self.L.orc_cg(_dims(dims), int(antiperiodic_t), _p(links), float(mass),
                                  float(shift), _p(b), _p(x), float(tol), int(max_iter),
                                  ctypes.byref(it), ctypes.byref(ri), ctypes.byref(rt)), "cg")
        return x, rc, dict(iters=it.value, resid_iter=ri.value, resid_true=rt.value)

    def multishift_cg(self, dims, links, mass, shifts, b, tol=1e-10, max_iter=100000,
                      antiperiodic_t=True):
        """Returns (x [n, V/2, 3], status, info)."""
        links, b = _cplx(links), _cplx(b)
        shifts = np.ascontiguousarray(shifts, dtype=np.float64)
        n = shifts.size
        x = np.zeros((n,) + b.shape, np.complex128)
        it = ctypes.c_int(0)
        its = np.zeros(n, np.int32)
        ri = np.zeros(n)
        rt = np.zeros(n)
        rc = _check(self.L.orc_multishift_cg(_dims(dims), int(antiperiodic_t), _p(links),
                                             float(mass), n, _p(shifts), _p(b), _p(x),
                                             float(tol), int(max_iter), ctypes.byref(it),
                                             _p(its), _p(ri), _p(rt)), "multishift_cg")
        return x, rc, dict(iters=it.value, iters_shift=its, resid_iter=ri, resid_true=rt)

    def rational_apply(self, dims, links, mass, alpha0, alphas, shifts, b, tol=1e-10, max_iter=100000,
                       antiperiodic_t=True):
        """r(M) b = alpha0 b + sum_i alpha_i (M + shift_i)^-1 b, the partial
        fraction form of the rational functions the RHMC applies (Section 2:
        rational approximations for the Metropolis step and the molecular
        dynamics), by its definition: each (M + shift_i)^-1 b from the
        multi-shift CG above, then the weighted sum.
        Returns (out, status, info); info as multishift_cg, plus dot = Re <b, out>."""
        b = _cplx(b)
        x, rc, info = self.multishift_cg(dims, links, mass, shifts, b, tol=tol, max_iter=max_iter,
                                         antiperiodic_t=antiperiodic_t)
        out = float(alpha0) * b
        for a, xi in zip(alphas, x):
            out = out + float(a) * xi
        info = dict(info, dot=float(np.vdot(b, out).real))
        return out, rc, info

    def fermion_force(self, dims, links, alphas, x, antiperiodic_t=True):
        """Pseudo-fermion force F_mu(x) = TA(U_mu(x) W_mu(x)) of the action
        sum_i alpha_i <phi, (M + sigma_i)^-1 phi>, from the solutions
        x [n, V/2, 3] (Section 2: the molecular dynamics force from the
        multi-shift solutions).  W collects the outer products of X_i and
        Y_i = -D_oe X_i at the two ends of each link; for U -> exp(i eps T) U
        the action changes at the rate i tr(T F).  Returns (4, V, 3, 3)."""
        links = _cplx(links)
        x = _cplx(np.asarray(x).reshape(len(alphas), int(np.prod(dims)) // 2, 3))
        alphas = np.ascontiguousarray(alphas, dtype=np.float64)
        force = np.empty(links.shape, np.complex128)
        _check(self.L.orc_fermion_force(_dims(dims), int(antiperiodic_t), _p(links), int(alphas.size),
                                        _p(alphas), _p(x), _p(force)), "fermion_force")
        return force

    # ---------------------------------------------------------------- learned preconditioner
    NET_NPARAM = 656

    def net_forward(self, dims, links, theta, r, antiperiodic_t=True):
        """P(r) on even sites; theta: complex (656,), r: (V/2, 3)."""
        links, theta, r = _cplx(links), _cplx(theta), _cplx(r)
        out = np.empty_like(r)
        _check(self.L.orc_net_forward(_dims(dims), int(antiperiodic_t), _p(links), _p(theta), _p(r),
                                      _p(out)), "net_forward")
        return out

    def net_layer1_odd(self, dims, links, theta, r, antiperiodic_t=True):
        links, theta, r = _cplx(links), _cplx(theta), _cplx(r)
        out = np.empty((r.shape[0], 8, 3), np.complex128)
        _check(self.L.orc_net_layer1_odd(_dims(dims), int(antiperiodic_t), _p(links), _p(theta), _p(r),
                                         _p(out)), "net_layer1_odd")
        return out

    def net_backward(self, dims, links, theta, r, g, antiperiodic_t=True):
        """Gradient of Re <g, P(r)> w.r.t. Re/Im of theta, as one complex array."""
        links, theta, r, g = _cplx(links), _cplx(theta), _cplx(r), _cplx(g)
        grad = np.empty(self.NET_NPARAM, np.complex128)
        _check(self.L.orc_net_backward(_dims(dims), int(antiperiodic_t), _p(links), _p(theta), _p(r),
                                       _p(g), _p(grad)), "net_backward")
        return grad


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _default = Oracle(_bind(ctypes.CDLL(_LIB_PATH)))
    return _default


def lib():
    return default().L


def load(path) -> Oracle:
    """An Oracle bound to the library at `path` (used to test the pins
    against deliberately broken builds of the oracle source)."""
    return Oracle(_bind(ctypes.CDLL(path)))


def __getattr__(name):
    # module-level access (oracle.dslash_eo(...)) goes to the default build
    if name in ("dhop_full", "dslash_eo", "normal_op", "tables", "true_residual", "cg",
                "multishift_cg", "net_forward", "net_layer1_odd", "net_backward"):
        return getattr(default(), name)
    raise AttributeError(name)
