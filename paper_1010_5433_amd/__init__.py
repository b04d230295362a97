"""Python binding of libstag.so, the MI355X even/odd staggered solver library.

A thin ctypes layer over the C ABI in include/stag.h: it passes device
pointers from torch tensors and the current HIP stream, and converts status
codes.  Every step of the computation runs in the library's HIP kernels;
there is no Python or CPU fallback -- importing fails loudly when the built
library is missing.

Library vectors are torch tensors of shape (3, V/2, 2) (colour plane, site,
re/im), float64 for STAG_F64 and float32 for STAG_F32.
"""
from __future__ import annotations

import ctypes
import os

import torch

from ._abi import (F32, F64, MIXED, LINK8, LINK12, LINK18, LINK12_PAIRS, LINK18_PAIRS, MIX_BF16, MIX_FOLDED, MIX_FOLDED_BF16, MIX_FP32, NET_NPARAM, CgStats, StagError,
                   System, batch_flags, load_library, status_name, Rational, RhmcParams, RhmcInfo)

__all__ = ["Lattice", "CgStats", "StagError", "F64", "F32", "MIXED", "LINK18", "LINK12",
           "library_path", "vec_empty", "multishift_cg_batched", "batch_last_config", "Net", "zolotarev", "rational_power",
           "NET_NPARAM", "rhmc_params"]

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libstag.so")


_L = load_library(library_path())

_PREC = {"f64": F64, "f32": F32, "mixed": MIXED, F64: F64, F32: F32, MIXED: MIXED}
_FMT = {"18": LINK18, "12": LINK12, "8": LINK8, 18: LINK18, 12: LINK12, 8: LINK8,
        "18p": LINK18_PAIRS, "12p": LINK12_PAIRS}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _check(rc: int, what: str):
    if rc < 0:
        raise StagError(rc, f"{what}: {status_name(rc)}: {_L.stag_last_error().decode()}")
    return rc


def vec_empty(vh: int, prec="f64", device="cuda") -> torch.Tensor:
    dt = torch.float64 if _PREC[prec] == F64 else torch.float32
    return torch.empty((3, vh, 2), dtype=dt, device=device)


class Lattice:
    """A lattice handle: geometry, packed links and solver work buffers."""

    def __init__(self, dims, antiperiodic_t: bool = True):
        self.dims = tuple(int(d) for d in dims)
        self.V = 1
        for d in self.dims:
            self.V *= d
        self.Vh = self.V // 2
        h = ctypes.c_void_p()
        _check(_L.stag_lattice_create((ctypes.c_int * 4)(*self.dims), int(antiperiodic_t),
                                      ctypes.byref(h)), "stag_lattice_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _L.stag_lattice_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- set-up
    def set_links(self, links: torch.Tensor, fmt="18"):
        """links: complex128 device tensor (4, V, 3, 3), canonical layout."""
        if links.dtype != torch.complex128 or tuple(links.shape) != (4, self.V, 3, 3):
            raise ValueError("links must be complex128 of shape (4, V, 3, 3)")
        _check(_L.stag_links_set(self._h, _ptr(links), _FMT[fmt], _stream()), "stag_links_set")

    def tables(self):
        nbr = torch.empty((2, 8, self.Vh), dtype=torch.int32, device="cuda")
        coord = torch.empty((2, self.Vh, 4), dtype=torch.int32, device="cuda")
        sign = torch.empty((2, 8, self.Vh), dtype=torch.int32, device="cuda")
        _check(_L.stag_tables(self._h, _ptr(nbr), _ptr(coord), _ptr(sign), _stream()), "stag_tables")
        return nbr, coord, sign

    def pack(self, canonical: torch.Tensor, prec="f64", out=None) -> torch.Tensor:
        """complex128 (V/2, 3) device tensor -> library vector."""
        if canonical.dtype != torch.complex128 or tuple(canonical.shape) != (self.Vh, 3):
            raise ValueError("canonical vector must be complex128 of shape (V/2, 3)")
        out = vec_empty(self.Vh, prec) if out is None else out
        _check(_L.stag_vec_pack(self._h, _ptr(canonical), _ptr(out), _PREC[prec], _stream()),
               "stag_vec_pack")
        return out

    def unpack(self, vec: torch.Tensor, prec=None) -> torch.Tensor:
        prec = prec if prec is not None else ("f64" if vec.dtype == torch.float64 else "f32")
        out = torch.empty((self.Vh, 3), dtype=torch.complex128, device="cuda")
        _check(_L.stag_vec_unpack(self._h, _ptr(vec), _ptr(out), _PREC[prec], _stream()),
               "stag_vec_unpack")
        return out

    # ---------------------------------------------------------------- operator
    def dslash_eo(self, out_parity: int, vec: torch.Tensor, out=None) -> torch.Tensor:
        prec = "f64" if vec.dtype == torch.float64 else "f32"
        out = torch.empty_like(vec) if out is None else out
        _check(_L.stag_dslash_eo(self._h, int(out_parity), _ptr(vec), _ptr(out), _PREC[prec],
                                 _stream()), "stag_dslash_eo")
        return out

    def normal_op(self, mass: float, shift: float, vec: torch.Tensor, out=None) -> torch.Tensor:
        prec = "f64" if vec.dtype == torch.float64 else "f32"
        out = torch.empty_like(vec) if out is None else out
        _check(_L.stag_normal_op(self._h, float(mass), float(shift), _ptr(vec), _ptr(out),
                                 _PREC[prec], _stream()), "stag_normal_op")
        return out

    def normal_op_noalloc(self, mass: float, shift: float, vec: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """normal_op with the library's static scratch: `out` must be given."""
        prec = "f64" if vec.dtype == torch.float64 else "f32"
        _check(_L.stag_normal_op_noalloc(self._h, float(mass), float(shift), _ptr(vec), _ptr(out),
                                         _PREC[prec], _stream()), "stag_normal_op_noalloc")
        return out

    # ---------------------------------------------------------------- solvers
    def multishift_cg(self, mass, shifts, src: torch.Tensor, sols=None, tol=1e-10,
                      max_iter=100000, prec="f64"):
        """Solve (M + shifts[i]) x_i = src.  Returns (sols, status, stats)."""
        shifts = [float(s) for s in shifts]
        n = len(shifts)
        if sols is None:
            sols = [torch.empty_like(src) for _ in range(n)]
        arr = (ctypes.c_double * n)(*shifts)
        ptrs = (ctypes.c_void_p * n)(*[_ptr(x).value for x in sols])
        st = CgStats()
        rc = _check(_L.stag_multishift_cg(self._h, float(mass), arr, n, _ptr(src), ptrs, float(tol),
                                          int(max_iter), _PREC[prec], ctypes.byref(st), _stream()),
                    "stag_multishift_cg")
        return sols, rc, st.to_dict(n)

    def rational_apply(self, mass, alpha0, alphas, shifts, src: torch.Tensor, out=None, tol=1e-10,
                       max_iter=100000):
        """out = alpha0 src + sum_i alphas[i] (M + shifts[i])^-1 src (double
        precision).  Returns (out, status, stats, Re <src, out>)."""
        shifts = [float(s) for s in shifts]
        alphas = [float(a) for a in alphas]
        n = len(shifts)
        if len(alphas) != n:
            raise ValueError("alphas and shifts differ in length")
        if out is None:
            out = torch.empty_like(src)
        sh = (ctypes.c_double * n)(*shifts)
        al = (ctypes.c_double * n)(*alphas)
        dot = ctypes.c_double(0.0)
        st = CgStats()
        rc = _check(_L.stag_rational_apply(self._h, float(mass), float(alpha0), al, sh, n, _ptr(src), _ptr(out),
                                           float(tol), int(max_iter), ctypes.byref(dot), ctypes.byref(st),
                                           _stream()), "stag_rational_apply")
        return out, rc, st.to_dict(n), dot.value

    def fermion_force(self, alphas, sols, out=None) -> torch.Tensor:
        """Pseudo-fermion force TA(U W) of sum_i alphas[i] <phi, (M + sigma_i)^-1 phi>
        from the solutions sols[i] = (M + sigma_i)^-1 phi (double precision
        library vectors).  Returns a complex128 (4, V, 3, 3) device tensor."""
        alphas = [float(a) for a in alphas]
        n = len(alphas)
        if len(sols) != n:
            raise ValueError("alphas and sols differ in length")
        for x in sols:
            if x.dtype != torch.float64 or tuple(x.shape) != (3, self.Vh, 2):
                raise ValueError("solutions must be double precision library vectors")
        if out is None:
            out = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device="cuda")
        elif out.dtype != torch.complex128 or tuple(out.shape) != (4, self.V, 3, 3):
            raise ValueError("out must be complex128 of shape (4, V, 3, 3)")
        al = (ctypes.c_double * max(n, 1))(*alphas)
        xp = (ctypes.c_void_p * max(n, 1))(*[_ptr(x).value for x in sols])
        _check(_L.stag_fermion_force(self._h, n, al, xp, _ptr(out), _stream()), "stag_fermion_force")
        return out

    def rational_apply_multi(self, mass, alpha0, alphas, shifts, srcs, outs=None, tol=1e-10,
                             max_iter=100000):
        """The rational function applied to several fields in one batched
        call.  Returns (outs, status, list of stats, list of Re <src_k, out_k>)."""
        shifts = [float(s) for s in shifts]
        alphas = [float(a) for a in alphas]
        n, m = len(shifts), len(srcs)
        if len(alphas) != n:
            raise ValueError("alphas and shifts differ in length")
        if outs is None:
            outs = [torch.empty_like(v) for v in srcs]
        sh = (ctypes.c_double * n)(*shifts)
        al = (ctypes.c_double * n)(*alphas)
        sp = (ctypes.c_void_p * m)(*[_ptr(v).value for v in srcs])
        op = (ctypes.c_void_p * m)(*[_ptr(v).value for v in outs])
        dots = (ctypes.c_double * m)()
        st = (CgStats * m)()
        rc = _check(_L.stag_rational_apply_multi(self._h, float(mass), float(alpha0), al, sh, n, sp, op, m,
                                                 float(tol), int(max_iter), dots, st, _stream()),
                    "stag_rational_apply_multi")
        return outs, rc, [st[k].to_dict(n) for k in range(m)], list(dots)

    # ---------------------------------------------------------------- RHMC trajectory
    def links_get(self) -> torch.Tensor:
        """complex128 (4, V, 3, 3) copy of the double precision link field."""
        out = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device="cuda")
        _check(_L.stag_links_get(self._h, _ptr(out), _stream()), "stag_links_get")
        return out

    def gauge_force(self, beta: float, prec="f64", out=None) -> torch.Tensor:
        out = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device="cuda") if out is None else out
        _check(_L.stag_gauge_force(self._h, float(beta), _ptr(out), _PREC[prec], _stream()), "stag_gauge_force")
        return out

    def gauge_action(self, beta: float) -> float:
        a = ctypes.c_double(0.0)
        _check(_L.stag_gauge_action(self._h, float(beta), ctypes.byref(a), _stream()), "stag_gauge_action")
        return a.value

    def gauge_kick(self, beta: float, h: float, mom: torch.Tensor, prec="f64") -> torch.Tensor:
        """mom: float64 (4, V, 8) device tensor, updated in place."""
        _check(_L.stag_gauge_kick(self._h, float(beta), float(h), _ptr(mom), _PREC[prec], _stream()),
               "stag_gauge_kick")
        return mom

    def force_kick(self, force: torch.Tensor, h: float, mom: torch.Tensor, prec="f64") -> torch.Tensor:
        _check(_L.stag_force_kick(self._h, _ptr(force), float(h), _ptr(mom), _PREC[prec], _stream()),
               "stag_force_kick")
        return mom

    def link_update(self, mom: torch.Tensor, h: float, prec="f64"):
        _check(_L.stag_link_update(self._h, _ptr(mom), float(h), _PREC[prec], _stream()), "stag_link_update")

    def md_integrate(self, prm: RhmcParams, mom: torch.Tensor, phis=()):
        """Molecular dynamics in place on the links and mom; returns the info dict."""
        info = RhmcInfo()
        arr = (ctypes.c_void_p * max(1, len(phis)))(*[t.data_ptr() for t in phis])
        for t in phis:
            _ptr(t)
        _check(_L.stag_md_integrate(self._h, ctypes.byref(prm), _ptr(mom), len(phis), arr, ctypes.byref(info),
                                    _stream()), "stag_md_integrate")
        return info.to_dict()

    def rhmc_trajectory(self, prm: RhmcParams, mom: torch.Tensor, xis=(), u=-1.0):
        info = RhmcInfo()
        arr = (ctypes.c_void_p * max(1, len(xis)))(*[t.data_ptr() for t in xis])
        for t in xis:
            _ptr(t)
        _check(_L.stag_rhmc_trajectory(self._h, ctypes.byref(prm), _ptr(mom), len(xis), arr, float(u),
                                       ctypes.byref(info), _stream()), "stag_rhmc_trajectory")
        return info.to_dict()

    def cg(self, mass, shift, src: torch.Tensor, x: torch.Tensor, tol=1e-10, max_iter=100000,
           prec="f64"):
        """Single-shift CG for (M + shift) x = src from the given x (overwritten)."""
        st = CgStats()
        rc = _check(_L.stag_cg(self._h, float(mass), float(shift), _ptr(src), _ptr(x), float(tol),
                               int(max_iter), _PREC[prec], ctypes.byref(st), _stream()), "stag_cg")
        return x, rc, st.to_dict(1)

    def fcg_solve(self, mass, shift, src: torch.Tensor, x: torch.Tensor, net=None, mode="folded_bf16", tol=1e-10,
                  max_iter=100000):
        """Flexible CG for (M + shift) x = src preconditioned by `net` (a Net, or
        None for plain double precision CG) evaluated in `mode` ("folded_bf16",
        the fastest; "folded"; or the layered forms "bf16" and "fp32"), from
        the given x (overwritten)."""
        st = CgStats()
        rc = _check(_L.stag_fcg_solve(self._h, float(mass), float(shift), _ptr(src), _ptr(x),
                                      net._h if net is not None else None, _MIX.get(mode, mode), float(tol),
                                      int(max_iter), ctypes.byref(st), _stream()), "stag_fcg_solve")
        return x, rc, st.to_dict(1)


_MIX = {"bf16": MIX_BF16, "fp32": MIX_FP32, "folded": MIX_FOLDED, "folded_bf16": MIX_FOLDED_BF16}


class Net:
    """The learned gauge-equivariant preconditioner (656 complex parameters).

    Vectors are single precision library vectors (float32, (3, V/2, 2)) of the
    lattice passed to each call."""

    def __init__(self, theta=None):
        h = ctypes.c_void_p()
        _check(_L.stag_net_create(ctypes.byref(h)), "stag_net_create")
        self._h = h
        if theta is not None:
            self.set_params(theta)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _L.stag_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _as_doubles(theta):
        import numpy as np
        t = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128).reshape(NET_NPARAM))
        return t, t.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def set_params(self, theta):
        """theta: 656 complex numbers (array-like)."""
        t, p = self._as_doubles(theta)
        _check(_L.stag_net_set_params(self._h, p), "stag_net_set_params")

    def get_params(self):
        import numpy as np
        t = np.zeros(NET_NPARAM, np.complex128)
        _check(_L.stag_net_get_params(self._h, t.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))), "stag_net_get_params")
        return t

    def apply(self, lat: Lattice, r: torch.Tensor, out=None, mode="bf16") -> torch.Tensor:
        out = torch.empty_like(r) if out is None else out
        _check(_L.stag_net_apply(self._h, lat._h, _ptr(r), _ptr(out), _MIX.get(mode, mode), _stream()),
               "stag_net_apply")
        return out

    def grad(self, lat: Lattice, r: torch.Tensor, g: torch.Tensor, mode="fp32"):
        """Gradient of Re <g, P(r)> as 656 complex numbers dL/dRe + i dL/dIm."""
        import numpy as np
        out = np.zeros(NET_NPARAM, np.complex128)
        _check(_L.stag_net_grad(self._h, lat._h, _ptr(r), _ptr(g), out.view(np.float64).ctypes.data_as(
            ctypes.POINTER(ctypes.c_double)), _MIX.get(mode, mode), _stream()), "stag_net_grad")
        return out

    def train_step(self, lat: Lattice, b: torch.Tensor, x: torch.Tensor, lr: float, mode="bf16") -> float:
        """One Adam step on n pairs; b, x: float32 (n, 3, V/2, 2).  Returns the loss."""
        if b.dim() != 4 or b.shape != x.shape:
            raise ValueError("b and x must be (n, 3, V/2, 2) with equal shapes")
        loss = ctypes.c_double(0.0)
        _check(_L.stag_net_train_step(self._h, lat._h, _ptr(b), _ptr(x), int(b.shape[0]), float(lr),
                                      _MIX.get(mode, mode), ctypes.byref(loss), _stream()), "stag_net_train_step")
        return loss.value


def _rational(r) -> Rational:
    out = Rational()
    if r is None:
        return out
    a0, al, sh = r
    if len(al) != len(sh) or not 1 <= len(al) <= 64:
        raise ValueError("a rational function needs 1 to 64 (weight, shift) pairs")
    out.alpha0 = float(a0)
    out.n = len(al)
    for i, (a, s_) in enumerate(zip(al, sh)):
        out.alpha[i] = float(a)
        out.shift[i] = float(s_)
    return out


def rhmc_params(beta, mass, tau, n_md, n_g, prec="f32", tol_md=1e-8, tol_act=1e-10, rat_md=None,
                rat_act=None, rat_hb=None, max_iter=100000) -> RhmcParams:
    """Parameters of stag_md_integrate / stag_rhmc_trajectory; each rational
    function is (alpha0, alphas, shifts)."""
    p = RhmcParams()
    p.beta, p.mass, p.tau = float(beta), float(mass), float(tau)
    p.n_md, p.n_g = int(n_md), int(n_g)
    p.md_prec = _PREC[prec]
    p.max_iter = int(max_iter)
    p.tol_md, p.tol_act = float(tol_md), float(tol_act)
    p.rat_md, p.rat_act, p.rat_hb = _rational(rat_md), _rational(rat_act), _rational(rat_hb)
    return p


def zolotarev(power, lo, hi, n):
    """Zolotarev's optimal relative approximation of x^(-1/2) (power -1) or
    x^(1/2) (power +1) on [lo, hi] with n poles: (alpha0, alphas, shifts,
    max relative error)."""
    a0 = ctypes.c_double(0.0)
    al = (ctypes.c_double * n)()
    sh = (ctypes.c_double * n)()
    err = ctypes.c_double(0.0)
    _check(_L.stag_zolotarev(int(power), float(lo), float(hi), int(n), ctypes.byref(a0), al, sh,
                             ctypes.byref(err)), "stag_zolotarev")
    return a0.value, list(al), list(sh), err.value


def rational_power(power, lo, hi, n):
    """Best relative approximation of x^power (power in (-1, 0) or (0, 1)) on
    [lo, hi] with n poles: (alpha0, alphas, shifts, max relative error)."""
    a0 = ctypes.c_double(0.0)
    al = (ctypes.c_double * n)()
    sh = (ctypes.c_double * n)()
    err = ctypes.c_double(0.0)
    _check(_L.stag_rational_power(float(power), float(lo), float(hi), int(n), ctypes.byref(a0), al, sh,
                                  ctypes.byref(err)), "stag_rational_power")
    return a0.value, list(al), list(sh), err.value


def multishift_cg_batched(systems, tol=1e-10, max_iter=100000, prec="f64", no_graph=False,
                          rpt=0, block=0, per_lattice=False):
    """Batched multi-shift CG.  systems: list of dicts with keys lat (Lattice),
    mass, shifts, src (library vector) and optionally sols.  Systems on the
    same Lattice share link loads.  Returns (list of sols, status, list of
    stats dicts).  rpt/block force a launch shape (0: autotune); no_graph
    launches every kernel instead of replaying the captured block of 16
    iterations; per_lattice makes one multi-RHS Dslash launch per lattice
    and group instead of one for all lattices."""
    n = len(systems)
    keep = []
    arr = (System * n)()
    all_sols = []
    for k, y in enumerate(systems):
        shifts = [float(v) for v in y["shifts"]]
        sols = y.get("sols") or [torch.empty_like(y["src"]) for _ in shifts]
        all_sols.append(sols)
        sh = (ctypes.c_double * len(shifts))(*shifts)
        sp = (ctypes.c_void_p * len(shifts))(*[_ptr(x).value for x in sols])
        keep += [sh, sp]
        arr[k].lat = y["lat"]._h
        arr[k].mass = float(y["mass"])
        arr[k].n_shifts = len(shifts)
        arr[k].shifts = sh
        arr[k].src = _ptr(y["src"])
        arr[k].sols = sp
    st = (CgStats * n)()
    rc = _check(_L.stag_multishift_cg_batched(arr, n, float(tol), int(max_iter), _PREC[prec],
                                              batch_flags(no_graph, rpt, block, per_lattice), st, _stream()),
                "stag_multishift_cg_batched")
    return all_sols, rc, [st[k].to_dict(len(systems[k]["shifts"])) for k in range(n)]


def batch_last_config():
    b, r = ctypes.c_int(0), ctypes.c_int(0)
    _check(_L.stag_batch_last_config(ctypes.byref(b), ctypes.byref(r)), "stag_batch_last_config")
    return b.value, r.value
