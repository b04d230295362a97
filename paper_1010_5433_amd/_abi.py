"""ctypes declarations of the C ABI (include/stag.h).  Importable without a
GPU: loading the shared library and resolving its symbols needs no device."""
from __future__ import annotations

import ctypes
import os

STAG_OK, STAG_ENOCONV, STAG_EBREAKDOWN = 0, 1, 2
STAG_EINVAL, STAG_ENOMEM, STAG_EHIP = -1, -2, -3
F64, F32, MIXED = 0, 1, 2
LINK18, LINK12, LINK8, LINK18_PAIRS, LINK12_PAIRS = 0, 1, 2, 3, 4
MAX_SHIFTS = 64
NET_NPARAM = 656
MIX_BF16, MIX_FP32, MIX_FOLDED, MIX_FOLDED_BF16 = 0, 1, 2, 3

_NAMES = {0: "STAG_OK", 1: "STAG_ENOCONV", 2: "STAG_EBREAKDOWN", -1: "STAG_EINVAL",
          -2: "STAG_ENOMEM", -3: "STAG_EHIP"}


def status_name(rc: int) -> str:
    return _NAMES.get(rc, f"status {rc}")


class StagError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class CgStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("n_reliable", ctypes.c_int),
        ("refine_iters", ctypes.c_int),
        ("fallback_used", ctypes.c_int),
        ("iters_shift", ctypes.c_int * MAX_SHIFTS),
        ("resid_iter", ctypes.c_double * MAX_SHIFTS),
        ("resid_true", ctypes.c_double * MAX_SHIFTS),
        ("resid_unrefined", ctypes.c_double * MAX_SHIFTS),
        ("refine_iters_shift", ctypes.c_int * MAX_SHIFTS),
        ("seconds", ctypes.c_double),
    ]

    def to_dict(self, n: int) -> dict:
        return dict(iters=self.iters, n_reliable=self.n_reliable, refine_iters=self.refine_iters,
                    fallback_used=self.fallback_used,
                    iters_shift=list(self.iters_shift[:n]), resid_iter=list(self.resid_iter[:n]),
                    resid_true=list(self.resid_true[:n]),
                    resid_unrefined=list(self.resid_unrefined[:n]),
                    refine_iters_shift=list(self.refine_iters_shift[:n]), seconds=self.seconds)


_v, _i, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double


class System(ctypes.Structure):
    _fields_ = [
        ("lat", _v),
        ("mass", _d),
        ("n_shifts", _i),
        ("shifts", ctypes.POINTER(_d)),
        ("src", _v),
        ("sols", ctypes.POINTER(_v)),
    ]


BATCH_NO_GRAPH = 0x1
BATCH_PER_LATTICE = 0x2


def batch_flags(no_graph=False, rpt=0, block=0, per_lattice=False):
    return ((BATCH_NO_GRAPH if no_graph else 0) | (BATCH_PER_LATTICE if per_lattice else 0) | ((rpt & 0xF) << 4) |
            (((block // 64) & 0xF) << 8))


MAX_PSEUDOFERMIONS = 16


class Rational(ctypes.Structure):
    _fields_ = [
        ("alpha0", _d),
        ("n", _i),
        ("alpha", _d * MAX_SHIFTS),
        ("shift", _d * MAX_SHIFTS),
    ]


class RhmcParams(ctypes.Structure):
    _fields_ = [
        ("beta", _d),
        ("mass", _d),
        ("tau", _d),
        ("n_md", _i),
        ("n_g", _i),
        ("md_prec", _i),
        ("max_iter", _i),
        ("tol_md", _d),
        ("tol_act", _d),
        ("rat_md", Rational),
        ("rat_act", Rational),
        ("rat_hb", Rational),
    ]


class RhmcInfo(ctypes.Structure):
    _fields_ = [
        ("dH", _d),
        ("H0", _d * 3),
        ("H1", _d * 3),
        ("accepted", _i),
        ("fermion_forces", _i),
        ("gauge_forces", _i),
        ("md_iters", _i),
        ("action_iters", _i),
        ("seconds", _d),
    ]

    def to_dict(self) -> dict:
        return dict(dH=self.dH, H0=list(self.H0), H1=list(self.H1), accepted=bool(self.accepted),
                    fermion_forces=self.fermion_forces, gauge_forces=self.gauge_forces,
                    md_iters=self.md_iters, action_iters=self.action_iters, seconds=self.seconds)


# name -> (restype, argtypes); the full set of entry points of include/stag.h
SIGNATURES = {
    "stag_lattice_create": (_i, [ctypes.POINTER(ctypes.c_int), _i, ctypes.POINTER(_v)]),
    "stag_lattice_destroy": (_i, [_v]),
    "stag_half_volume": (ctypes.c_int64, [_v]),
    "stag_links_set": (_i, [_v, _v, _i, _v]),
    "stag_tables": (_i, [_v, _v, _v, _v, _v]),
    "stag_vec_pack": (_i, [_v, _v, _v, _i, _v]),
    "stag_vec_unpack": (_i, [_v, _v, _v, _i, _v]),
    "stag_dslash_eo": (_i, [_v, _i, _v, _v, _i, _v]),
    "stag_normal_op": (_i, [_v, _d, _d, _v, _v, _i, _v]),
    "stag_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "stag_normal_op_noalloc": (_i, [_v, _d, _d, _v, _v, _i, _v]),
    "stag_multishift_cg": (_i, [_v, _d, ctypes.POINTER(_d), _i, _v, ctypes.POINTER(_v), _d, _i, _i,
                                ctypes.POINTER(CgStats), _v]),
    "stag_cg": (_i, [_v, _d, _d, _v, _v, _d, _i, _i, ctypes.POINTER(CgStats), _v]),
    "stag_multishift_cg_batched": (_i, [ctypes.POINTER(System), _i, _d, _i, _i, _i,
                                        ctypes.POINTER(CgStats), _v]),
    "stag_batch_last_config": (_i, [ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "stag_net_create": (_i, [ctypes.POINTER(_v)]),
    "stag_net_destroy": (_i, [_v]),
    "stag_net_set_params": (_i, [_v, ctypes.POINTER(_d)]),
    "stag_net_get_params": (_i, [_v, ctypes.POINTER(_d)]),
    "stag_net_apply": (_i, [_v, _v, _v, _v, _i, _v]),
    "stag_net_grad": (_i, [_v, _v, _v, _v, ctypes.POINTER(_d), _i, _v]),
    "stag_net_train_step": (_i, [_v, _v, _v, _v, _i, _d, _i, ctypes.POINTER(_d), _v]),
    "stag_fcg_solve": (_i, [_v, _d, _d, _v, _v, _v, _i, _d, _i, ctypes.POINTER(CgStats), _v]),
    "stag_fermion_force": (_i, [_v, _i, ctypes.POINTER(_d), ctypes.POINTER(_v), _v, _v]),
    "stag_links_get": (_i, [_v, _v, _v]),
    "stag_gauge_force": (_i, [_v, _d, _v, _i, _v]),
    "stag_gauge_action": (_i, [_v, _d, ctypes.POINTER(_d), _v]),
    "stag_gauge_kick": (_i, [_v, _d, _d, _v, _i, _v]),
    "stag_force_kick": (_i, [_v, _v, _d, _v, _i, _v]),
    "stag_link_update": (_i, [_v, _v, _d, _i, _v]),
    "stag_md_integrate": (_i, [_v, ctypes.POINTER(RhmcParams), _v, _i, ctypes.POINTER(_v),
                               ctypes.POINTER(RhmcInfo), _v]),
    "stag_rhmc_trajectory": (_i, [_v, ctypes.POINTER(RhmcParams), _v, _i, ctypes.POINTER(_v), _d,
                                  ctypes.POINTER(RhmcInfo), _v]),
    "stag_rational_apply": (_i, [_v, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d), _i, _v, _v, _d, _i,
                                 ctypes.POINTER(_d), ctypes.POINTER(CgStats), _v]),
    "stag_rational_apply_multi": (_i, [_v, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d), _i,
                                       ctypes.POINTER(_v), ctypes.POINTER(_v), _i, _d, _i, ctypes.POINTER(_d),
                                       ctypes.POINTER(CgStats), _v]),
    "stag_zolotarev": (_i, [_i, _d, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                            ctypes.POINTER(_d)]),
    "stag_rational_power": (_i, [_d, _d, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                 ctypes.POINTER(_d)]),
    "stag_hbm_probe": (_i, [_v, _v, ctypes.c_int64, _i, _v]),
    "stag_status_string": (ctypes.c_char_p, [_i]),
    "stag_last_error": (ctypes.c_char_p, []),
}


def load_library(path: str):
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()' or python -m paper_1010_5433_amd.build)")
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L
