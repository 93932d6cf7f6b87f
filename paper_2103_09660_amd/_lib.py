"""ctypes loader for ``libhnv.so`` (the C ABI declared in include/hnv.h).

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_2103_09660_amd._build`` or ``__graft_entry__.build()``);
there is no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhnv.so")

HNV_OK, HNV_EINVAL, HNV_ERANGE, HNV_EUNSORTED, HNV_EUNSUPPORTED, HNV_EWORKSPACE, HNV_EDEVICE, HNV_ENOMEM = range(8)
STATUS_NAMES = {0: "HNV_OK", 1: "HNV_EINVAL", 2: "HNV_ERANGE", 3: "HNV_EUNSORTED", 4: "HNV_EUNSUPPORTED",
                5: "HNV_EWORKSPACE", 6: "HNV_EDEVICE", 7: "HNV_ENOMEM"}
HNV_F32, HNV_BF16 = 0, 1
HNV_ORDER_JACOBI, HNV_ORDER_EDGE_FIRST = 0, 1
HNV_SCORE_VARIANCE, HNV_SCORE_MEAN, HNV_SCORE_MIN, HNV_SCORE_MAX = 0, 1, 2, 3
HNV_PROF_SWEEP, HNV_PROF_FUSED, HNV_PROF_ADJ_NODE, HNV_PROF_ADJ_EDGE = 0, 1, 2, 3

i64 = ctypes.c_int64
i32 = ctypes.c_int32
i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
f32p = ctypes.POINTER(ctypes.c_float)
f64p = ctypes.POINTER(ctypes.c_double)
vp = ctypes.c_void_p


class HnvLevel(ctypes.Structure):
    _fields_ = [("n_nodes", i64), ("n_edges", i64), ("nnz", i64),
                ("edge_ptr", i64p), ("edge_idx", i32p), ("edge_w", f32p),
                ("node_ptr", i64p), ("node_idx", i32p)]


class HnvLevelDev(ctypes.Structure):
    _fields_ = [("n_nodes", i64), ("n_edges", i64), ("nnz", i64),
                ("edge_ptr", vp), ("edge_idx", vp), ("edge_w", vp)]


class HnvMap(ctypes.Structure):
    _fields_ = [("node_rep", i32p), ("edge_rep", i32p)]


class HnvMapDev(ctypes.Structure):
    """hnv_map holding device pointers."""
    _fields_ = [("node_rep", vp), ("edge_rep", vp)]


class HnvOptions(ctypes.Structure):
    _fields_ = [("panel_cols", i32), ("small_max", i32), ("chunk", i32), ("order", i32)]


class HnvError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_SIGS = {
    "hnv_abi_version": (ctypes.c_int, []),
    "hnv_last_error": (ctypes.c_char_p, []),
    "hnv_validate_level": (ctypes.c_int, [ctypes.POINTER(HnvLevel)]),
    "hnv_coarsen_level": (ctypes.c_int, [ctypes.POINTER(HnvLevel), i32p, i32p, i64p, i32p, f32p, i64p, i64p, i64p]),
    "hnv_coarsen_workspace_bytes": (ctypes.c_int, [i64, i64, i64, ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_coarsen_level_device": (ctypes.c_int, [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, i64p, vp,
                                                ctypes.c_size_t, vp]),
    "hnv_coarsen_features_workspace_bytes": (ctypes.c_int, [i64, i64, i64, ctypes.c_int,
                                                            ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_coarsen_level_features_device": (ctypes.c_int, [i64, i64, i64, vp, vp, vp, vp, ctypes.c_int, vp, vp, vp,
                                                         vp, vp, vp, i64p, vp, ctypes.c_size_t, vp]),
    "hnv_plan_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(HnvLevel), ctypes.POINTER(HnvMap), ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int, ctypes.POINTER(HnvOptions),
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_plan_create": (ctypes.c_int, [ctypes.POINTER(HnvLevel), ctypes.POINTER(HnvMap), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(HnvOptions), ctypes.c_int, vp, ctypes.c_size_t,
                                       vp, ctypes.POINTER(vp)]),
    "hnv_plan_workspace_bytes_device": (ctypes.c_int, [ctypes.POINTER(HnvLevelDev), ctypes.POINTER(HnvMapDev),
                                                       ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                       ctypes.POINTER(HnvOptions), ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_plan_create_device": (ctypes.c_int, [ctypes.POINTER(HnvLevelDev), ctypes.POINTER(HnvMapDev), ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.POINTER(HnvOptions), ctypes.c_int,
                                              vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
    "hnv_plan_destroy": (ctypes.c_int, [vp]),
    "hnv_plan_level_info": (ctypes.c_int, [vp, ctypes.c_int, i64p, i64p, i64p]),
    "hnv_set_edge_weights": (ctypes.c_int, [vp, ctypes.c_int, vp, vp]),
    "hnv_set_edge_logweights": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "hnv_refine": (ctypes.c_int, [vp, vp, vp, i32p, ctypes.c_float, ctypes.c_double, vp, i32p, vp]),
    "hnv_project": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "hnv_sweep": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_float, ctypes.c_int, vp, vp]),
    "hnv_sweep_noalloc": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_float, ctypes.c_int, vp, vp]),
    "hnv_sweep_adjoint": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_float, vp]),
    "hnv_sweep_adjoint_split": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, ctypes.c_float, vp]),
    "hnv_weight_grad_finish": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "hnv_project_adjoint": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "hnv_logweight_grad": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
    "hnv_plan_set_profiling": (ctypes.c_int, [vp, ctypes.c_int]),
    "hnv_plan_profile_read": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, i64p, f64p]),
    "hnv_score_workspace_bytes": (ctypes.c_int, [i64p, i64, ctypes.c_int, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_score_plan_create": (ctypes.c_int, [i64p, i32p, i64, i64, ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t,
                                             vp, ctypes.POINTER(vp)]),
    "hnv_score_workspace_bytes_device": (ctypes.c_int, [i64, i64, ctypes.c_int, ctypes.c_int,
                                                        ctypes.POINTER(ctypes.c_size_t)]),
    "hnv_score_plan_create_device": (ctypes.c_int, [vp, vp, i64, i64, i64, ctypes.c_int, ctypes.c_int, vp,
                                                    ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
    "hnv_score_plan_destroy": (ctypes.c_int, [vp]),
    "hnv_score_candidates": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, vp]),
    "hnv_cast": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.c_int, i64, vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_09660_amd._build` "
                              "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names() -> list:
    return list(_SIGS)


def last_error() -> str:
    return lib().hnv_last_error().decode()


def check(status: int, where: str) -> None:
    if status != HNV_OK:
        raise HnvError(status, where, last_error())


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args), name)
