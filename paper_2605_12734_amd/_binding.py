"""ctypes binding of libod.so (include/od.h), argument marshalling only.

Every step of the hot path runs inside libod's HIP kernels; this module only
converts Python arguments to the C ABI and PyTorch device buffers / streams to
raw pointers.  If the library has not been built the import fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libod.so")

OD_OK = 0
OD_EINVAL = -22
OD_ENOMEM = -12
OD_EAGAIN = -11
OD_ENOTREADY = -61
OD_ECANCELED = -125
OD_ETIMEDOUT = -110
OD_ESCHED = -71
OD_EHIP = -1000
STATUS_NAMES = {0: "OD_OK", -22: "OD_EINVAL", -12: "OD_ENOMEM", -11: "OD_EAGAIN", -61: "OD_ENOTREADY",
                -125: "OD_ECANCELED", -110: "OD_ETIMEDOUT", -71: "OD_ESCHED", -1000: "OD_EHIP"}
HINT_NONTEMPORAL, HINT_SPATIAL_ORDER, HINT_SCHEDULE_CHECK = 1, 2, 4
HINT_ONE_STEP = 4096

OD_F32, OD_F64 = 4, 8
EXEC = {"per_chare": 0, "fused": 1, "graph": 2, "persistent": 3, "msgdriven": 4}

c_i32, c_i64, c_u64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_void_p, ctypes.c_size_t)


class od_block(ctypes.Structure):
    _fields_ = [("origin", c_i32 * 3), ("extent", c_i32 * 3)]


class od_config(ctypes.Structure):
    _fields_ = [("n", c_i64 * 3), ("block", c_i64 * 3), ("odf", c_i32), ("blocks", ctypes.POINTER(od_block)),
                ("nblocks", c_i32), ("dtype", ctypes.c_int), ("bc", c_dbl * 6), ("seed", c_u64),
                ("exec", ctypes.c_int), ("tile", c_i32 * 3), ("imbalance_pct", c_i32),
                ("imbalance_max_extra", c_i32), ("hints", c_i32), ("stencil", c_i32),
                ("block_cell", ctypes.POINTER(c_i32)), ("wait_s", ctypes.c_double)]


class od_plan_info(ctypes.Structure):
    _fields_ = [("nchares", c_i32), ("ntiles", c_i32), ("npseudo", c_i32), ("interior", c_i64),
                ("halo_cells", c_i64), ("bytes_per_iter", c_i64), ("tile", c_i32 * 3), ("grid_wgs", c_i32),
                ("schedule", c_i32), ("coop_waves", c_i32), ("field_bytes", c_i64), ("control_bytes", c_i64),
                ("steps_per_pass", c_i32), ("bytes_per_pass", c_i64)]


class od_tile_info(ctypes.Structure):
    _fields_ = [("chare", c_i32), ("origin", c_i32 * 3), ("extent", c_i32 * 3), ("src_kind", c_i32 * 6),
                ("src", c_i32 * 6), ("src_origin", (c_i32 * 3) * 6)]


class od_request(ctypes.Structure):
    _fields_ = [("n", c_i64), ("dtype", ctypes.c_int), ("odf", c_i32), ("tol", c_dbl), ("max_iters", c_i64),
                ("check_every", c_i32), ("seed", c_u64), ("bc", c_dbl * 6), ("t_arrival", c_dbl)]


class od_info(ctypes.Structure):
    _fields_ = [("state", c_i32), ("iters", c_i64), ("residual", c_dbl), ("t_submit", c_dbl),
                ("t_admit", c_dbl), ("t_done", c_dbl), ("t_arrival", c_dbl)]


class od_server_stats(ctypes.Structure):
    _fields_ = [("epochs", c_i64), ("epoch_s", c_dbl), ("admit_s", c_dbl), ("retire_s", c_dbl), ("idle_s", c_dbl)]


class od_overlap_result(ctypes.Structure):
    _fields_ = [("total_threads", c_i64), ("nkernels", c_i32), ("nstreams", c_i32), ("work", c_i32),
                ("pad", c_i32), ("makespan_us", c_dbl), ("host_us", c_dbl), ("enqueue_us", c_dbl)]


# name -> (restype, argtypes); the full exported surface of include/od.h
SIGNATURES = {
    "od_config_default": (None, [ctypes.POINTER(od_config)]),
    "od_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(od_config), ctypes.POINTER(c_sz)]),
    "od_create": (ctypes.c_int, [ctypes.POINTER(od_config), c_vp, c_vp, c_sz, ctypes.POINTER(c_vp)]),
    "od_create_static": (ctypes.c_int, [ctypes.POINTER(od_config), c_vp, c_vp, c_sz, ctypes.POINTER(c_vp)]),
    "od_plan_create": (ctypes.c_int, [ctypes.POINTER(od_config), ctypes.POINTER(c_vp)]),
    "od_iterate": (ctypes.c_int, [c_vp, c_i64]),
    "od_residual": (ctypes.c_int, [c_vp, ctypes.POINTER(c_dbl)]),
    "od_iterations": (ctypes.c_int, [c_vp, ctypes.POINTER(c_i64)]),
    "od_read": (ctypes.c_int, [c_vp, c_vp, c_sz]),
    "od_write": (ctypes.c_int, [c_vp, c_vp, c_sz]),
    "od_read_points": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp]),
    "od_plan": (ctypes.c_int, [c_vp, ctypes.POINTER(od_plan_info)]),
    "od_tile_info_get": (ctypes.c_int, [c_vp, c_i32, ctypes.POINTER(od_tile_info)]),
    "od_tile_deps": (ctypes.c_int, [c_vp, c_i32, ctypes.POINTER(c_i32), c_i32, ctypes.POINTER(c_i32)]),
    "od_chare_get": (ctypes.c_int, [c_vp, c_i32, ctypes.POINTER(od_block)]),
    "od_timeline": (ctypes.c_int, [c_vp, c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "od_extra_sweeps": (ctypes.c_int, [c_vp, c_i64, c_vp, c_i32]),
    "od_destroy": (ctypes.c_int, [c_vp]),
    "od_stream_copy": (ctypes.c_int, [c_vp, c_vp, c_vp, c_sz, c_i32, ctypes.POINTER(c_dbl)]),
    "od_stream_bench": (ctypes.c_int, [c_vp, c_vp, c_vp, c_sz, c_i32, c_i32, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i32)]),
    "od_time_iterate": (ctypes.c_int, [c_vp, c_i64, ctypes.POINTER(c_dbl)]),
    "od_block_cells": (ctypes.c_int, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "od_read_block": (ctypes.c_int, [c_vp, c_i32, c_vp, c_sz]),
    "od_write_block": (ctypes.c_int, [c_vp, c_i32, c_vp, c_sz]),
    "od_server_stats_get": (ctypes.c_int, [c_vp, ctypes.POINTER(od_server_stats)]),
    "od_launch_overlap_bytes": (c_sz, [c_i64]),
    "od_launch_overlap": (ctypes.c_int, [c_vp, c_sz, c_i64, c_i32, c_i32, c_i32, ctypes.POINTER(od_overlap_result)]),
    "od_autotune": (ctypes.c_int, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "od_server_create": (ctypes.c_int, [c_vp, c_vp, c_sz, c_i32, ctypes.POINTER(c_vp)]),
    "od_request_bytes": (ctypes.c_int, [ctypes.POINTER(od_request), ctypes.POINTER(c_sz)]),
    "od_server_control_bytes": (ctypes.c_int, [c_i32, ctypes.POINTER(c_sz)]),
    "od_submit": (ctypes.c_int, [c_vp, ctypes.POINTER(od_request), ctypes.POINTER(c_u64)]),
    "od_server_set_hints": (ctypes.c_int, [c_vp, c_i32, c_u64]),
    "od_server_step": (ctypes.c_int, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "od_poll": (ctypes.c_int, [c_vp, c_u64, ctypes.POINTER(od_info)]),
    "od_fetch": (ctypes.c_int, [c_vp, c_u64, c_vp, c_sz]),
    "od_server_destroy": (ctypes.c_int, [c_vp]),
    "od_last_error": (ctypes.c_char_p, []),
    "od_version": (ctypes.c_char_p, []),
}

_lib = None


class ODError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def lib():
    """Load libod.so; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_2605_12734_amd/build.py (hipcc, gfx950)")
    # libod links the HIP runtime by its soname; PyTorch loads its own copy
    # of that runtime by path.  Load PyTorch first so the dynamic linker
    # binds libod to the same runtime: two HIP runtimes in one process do
    # not share the device (the second finds no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int, where: str) -> None:
    if status != OD_OK:
        raise ODError(status, where, lib().od_last_error().decode(errors="replace"))
