"""ctypes declarations of the libcaps C ABI (include/caps.h).

Loading fails loudly when libcaps.so has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcaps.so")

c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_vp = ctypes.c_void_p

STATUS = {0: "CAPS_OK", -1: "CAPS_EINVAL", -2: "CAPS_ENOMEM", -3: "CAPS_EDEVICE",
          -4: "CAPS_EUNSUPPORTED", -5: "CAPS_EBUSY", -6: "CAPS_EIO"}


class CapsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class BuildParams(ctypes.Structure):
    _fields_ = [("metric", c_i32), ("n_partitions", c_i32), ("kmeans_iters", c_i32),
                ("aft_height", c_i32), ("seed", c_u64), ("init_ids", c_vp),
                ("precision", c_i32), ("reserved", c_i32), ("assign", c_vp)]


class SearchParams(ctypes.Structure):
    _fields_ = [("k", c_i32), ("nprobe", c_i32), ("rule", c_i32), ("mode", c_i32),
                ("rerank", c_i32), ("routing", c_i32), ("flags", c_i32), ("rescue_grid", c_i32),
                ("workspace_bytes", c_i64)]


SEARCH_VALIDATE = 1
SEARCH_DISJUNCTIVE = 2
OR = -1          # constraint attribute that separates the AND-terms of a disjunctive query
MAX_TERMS = 4


class RouterParams(ctypes.Structure):
    _fields_ = [("hidden", c_i32), ("epochs", c_i32), ("batch", c_i32), ("reset", c_i32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("in_scale", ctypes.c_float), ("in_shift", ctypes.c_float),
                ("fallback_prob", ctypes.c_float), ("reserved", c_i32), ("seed", c_u64)]


class RouterInfo(ctypes.Structure):
    _fields_ = [("present", c_i32), ("din", c_i32), ("dpad", c_i32), ("hidden", c_i32),
                ("n_out", c_i32), ("in_scale", ctypes.c_float), ("in_shift", ctypes.c_float),
                ("fallback_prob", ctypes.c_float), ("steps", c_i64)]


class ServerParams(ctypes.Structure):
    _fields_ = [("k", c_i32), ("nprobe", c_i32), ("mode", c_i32), ("routing", c_i32), ("rerank", c_i32),
                ("max_batch", c_i32), ("streams", c_i32), ("queue_slots", c_i32),
                ("max_constraints", c_i32), ("flags", c_i32), ("workspace_bytes", c_i64),
                ("batch_window_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("rejected", c_i64), ("failed", c_i64),
                ("batches", c_i64), ("mean_batch", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("qps", ctypes.c_double), ("max_batch", c_i32), ("reserved", c_i32)]


PREC = {"none": 0, "fp32": 0, "bf16": 1, "fp8": 2, "fp16": 3}


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", c_i64), ("d", c_i32), ("n_partitions", c_i32), ("aft_height", c_i32),
                ("metric", c_i32), ("n_dense", c_i32), ("label_vocab", c_i32),
                ("n_tokens", c_i32), ("max_subpartition", c_i32), ("precision", c_i32),
                ("lowp_dpad", c_i32), ("label_slots", c_i32), ("reserved", c_i32), ("device_bytes", c_i64)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", c_i64 * 8)]


STAGES = ["prep", "route", "topm", "select", "scan", "merge", "seed", "rescue"]

# name -> (restype, argtypes); every symbol include/caps.h declares
SIGNATURES = {
    "caps_build": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32,
                           ctypes.POINTER(BuildParams), c_vp, ctypes.POINTER(c_vp)]),
    "caps_insert": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp]),
    "caps_bliss_assign": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp]),
    "caps_search": (c_i32, [c_vp, ctypes.POINTER(SearchParams), c_vp, c_i32, c_vp, c_vp, c_vp,
                            c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_search_static": (c_i32, [c_vp, ctypes.POINTER(SearchParams), c_vp, c_i32, c_vp, c_vp, c_vp,
                                   c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_search_debug": (c_i32, [c_vp, ctypes.POINTER(SearchParams), c_vp, c_i32, c_vp, c_vp, c_vp,
                                  c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_search_workspace": (c_i32, [c_vp, ctypes.POINTER(SearchParams), c_i32, ctypes.POINTER(c_i64)]),
    "caps_search_probes": (c_i32, [c_vp, ctypes.POINTER(SearchParams), c_vp, c_i32, c_vp, c_vp,
                                   c_vp, c_i32, c_vp, c_vp, c_vp]),
    "caps_index_info": (c_i32, [c_vp, ctypes.POINTER(IndexInfo)]),
    "caps_index_export": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_index_export_lowp": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "caps_router_labels": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_vp, c_vp]),
    "caps_router_train": (c_i32, [c_vp, ctypes.POINTER(RouterParams), c_vp, c_i32, c_vp, c_vp, c_vp,
                                  c_i32, c_vp, c_i32, c_vp, c_vp]),
    "caps_router_set": (c_i32, [c_vp, ctypes.POINTER(RouterParams), c_vp, c_vp, c_vp, c_vp]),
    "caps_router_get": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_router_info": (c_i32, [c_vp, ctypes.POINTER(RouterInfo)]),
    "caps_router_logits": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]),
    "caps_router_grads": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_i32, c_vp,
                                  c_vp, c_vp, c_vp, c_vp, c_vp]),
    "caps_server_create": (c_i32, [c_vp, ctypes.POINTER(ServerParams), ctypes.POINTER(c_vp)]),
    "caps_server_submit": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, ctypes.POINTER(c_u64)]),
    "caps_server_replay": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]),
    "caps_server_poll": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(c_i32)]),
    "caps_server_drain": (c_i32, [c_vp, ctypes.c_double]),
    "caps_server_stats": (c_i32, [c_vp, ctypes.POINTER(ServerStats), c_i32]),
    "caps_server_destroy": (None, [c_vp]),
    "caps_save": (c_i32, [c_vp, ctypes.c_char_p]),
    "caps_load": (c_i32, [ctypes.c_char_p, c_vp, ctypes.POINTER(c_vp)]),
    "caps_free": (None, [c_vp]),
    "caps_profile_enable": (c_i32, [c_i32]),
    "caps_profile_read": (c_i32, [ctypes.POINTER(Profile)]),
    "caps_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libcaps.so (built in-tree by paper_2308_15014_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python -m paper_2308_15014_amd.build) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def profile_enable(on: bool = True):
    check(lib().caps_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{stage: (total ms, launches)} since profile_enable(True)."""
    p = Profile()
    check(lib().caps_profile_read(ctypes.byref(p)))
    return {s: (p.ms[i], int(p.launches[i])) for i, s in enumerate(STAGES)}


def check(status: int):
    if status != 0:
        msg = lib().caps_last_error()
        raise CapsError(status, msg.decode() if msg else "")
