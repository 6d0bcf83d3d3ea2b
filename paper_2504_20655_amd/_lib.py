"""ctypes declarations of the C ABI in include/wroute.h (libwroute.so).

torch is imported first so that the process has exactly one HIP runtime:
the library then binds to the runtime torch already loaded, and device
pointers and streams from torch are valid for it.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwroute.so")

u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
i32 = ctypes.c_int32
vp = ctypes.c_void_p
st = ctypes.c_int  # wr_status


class RunInfo(ctypes.Structure):
    _fields_ = [("algo", u32), ("unique_sources", u32), ("chunks", u32), ("passes", u32),
                ("work_items", u64), ("relax_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", u32), ("relaxations", u64),
                ("alg_bytes", u64)]


class Schedule(ctypes.Structure):
    _fields_ = [("tile_vertices", u32), ("waves_per_group", u32), ("passes_per_replay", u32),
                ("blocks_per_unit", u32), ("grid_tile_w", u32), ("grid_tile_h", u32)]


class WmsParams(ctypes.Structure):
    _fields_ = [("nx", u32), ("ny", u32), ("nz", u32), ("n_articles", u32), ("mmax", u32),
                ("purchase_orders", u32), ("articles_per_order", u32), ("clusters", u32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_source_slots", u32), ("mem_budget_bytes", u64), ("max_queue", u32),
                ("passes_per_step", u32), ("resident_epochs", u32)]


class ReqInfo(ctypes.Structure):
    _fields_ = [("epoch", u64), ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("P", u32), ("status", st)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", u64), ("completed", u64), ("failed", u64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("throughput_per_s", ctypes.c_double),
                ("max_inflight_requests", u32), ("steps", u64)]


# name -> (restype, argtypes); every symbol include/wroute.h declares
SIGNATURES = {
    "wr_status_str": (ctypes.c_char_p, [st]),
    "wr_last_error": (ctypes.c_char_p, []),
    "wr_version": (ctypes.c_char_p, []),
    "wr_context_create": (st, [ctypes.c_int, u64, vp]),
    "wr_context_destroy": (st, [vp]),
    "wr_context_memory": (st, [vp, vp, vp]),
    "wr_validate_csr": (st, [u32, u32, vp, vp, vp]),
    "wr_graph_create_csr": (st, [vp, u32, u32, vp, vp, vp, u32, vp]),
    "wr_graph_destroy": (st, [vp]),
    "wr_graph_set_segments": (st, [vp, vp, u32]),
    "wr_graph_segment_grid": (st, [vp, u32, u32, u32, u32, u32]),
    "wr_graph_segment_info": (st, [vp, vp, vp, vp]),
    "wr_graph_update_weights": (st, [vp, u32, vp, vp, vp]),
    "wr_graph_epoch": (st, [vp, vp]),
    "wr_sssp": (st, [vp, u32, vp, vp, vp, u32, vp]),
    "wr_order_matrices": (st, [vp, u32, vp, vp, vp, vp, u32, vp]),
    "wr_order_routes": (st, [vp, u32, vp, vp, vp, vp, u32, vp]),
    "wr_order_routes_static": (st, [vp, u32, vp, vp, vp, vp, u32, vp]),
    "wr_order_routes_clustered": (st, [vp, u32, vp, vp, vp, u32, vp, vp, vp, u32, vp]),
    "wr_wms_run": (st, [vp, vp, u32, u32, vp, vp, vp, vp, vp, vp, vp, u32, vp]),
    "wr_graph_last_run": (st, [vp, vp]),
    "wr_autotune": (st, [vp, u32, ctypes.c_char_p]),
    "wr_graph_set_schedule": (st, [vp, u32, u32, u32]),
    "wr_graph_get_schedule": (st, [vp, vp]),
    "wr_graph_set_blocks_per_unit": (st, [vp, u32]),
    "wr_debug_fault": (st, [u32, u64]),
    "wr_server_create": (st, [vp, vp, vp]),
    "wr_server_submit": (st, [vp, u32, vp, vp]),
    "wr_server_poll": (st, [vp, u64, vp, vp]),
    "wr_server_update_weights": (st, [vp, u32, vp, vp]),
    "wr_server_stats": (st, [vp, vp]),
    "wr_server_drain": (st, [vp]),
    "wr_server_destroy": (st, [vp]),
}

_lib = None


def load():
    """Loads libwroute.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2504_20655_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
