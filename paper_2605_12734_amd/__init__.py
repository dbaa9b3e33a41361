"""MI355X-native overdecomposed 3D Jacobi (one GPU's share of chares).

Python face of ``libod.so`` (see ``include/od.h``).  PyTorch supplies only
device memory (the caller-owned workspace) and the HIP stream; every step of
the hot path -- halo pack / exchange / unpack, the 7-point sweep, the
residual, the iteration control -- runs in libod's HIP kernels.

    from paper_2605_12734_amd import Grid
    g = Grid(512, odf=4096, dtype="f64", exec="graph")
    g.iterate(200)
    r = g.residual()
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence

import numpy as np

from . import _binding as B
from ._binding import ODError, check, lib

HINT_ONE_STEP = B.HINT_ONE_STEP   # od_config.hints bit 12: one step per pass

__all__ = ["Grid", "Grid2D", "ODError", "DEFAULT_BC", "stream_copy_seconds", "plan_info", "tile_infos", "lib",
           "Server", "launch_overlap"]

DEFAULT_BC = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
_DTYPES = {"f64": (B.OD_F64, np.float64), "f32": (B.OD_F32, np.float32),
           np.float64: (B.OD_F64, np.float64), np.float32: (B.OD_F32, np.float32)}


def _dims(n) -> tuple:
    if np.isscalar(n):
        return (int(n),) * 3
    return tuple(int(v) for v in n)


def make_config(n, odf: int = 8, block=None, blocks: Optional[Sequence] = None, dtype="f64",
                bc=DEFAULT_BC, seed: int = 12734, exec: str = "graph", tile=None,
                imbalance_pct: int = 0, imbalance_max_extra: int = 0, hints: int = 0, stencil: int = 7,
                cell: Optional[Sequence] = None, wait_s: float = 0.0):
    """Fill an od_config; returns (cfg, keepalive) where keepalive holds arrays it points to.
    `cell`: per explicit block, its cell edge in grid units (multi-resolution).
    `wait_s`: bound on device-side waits of cooperative launches (0 = 10 s)."""
    cfg = B.od_config()
    lib().od_config_default(ctypes.byref(cfg))
    nx, ny, nz = _dims(n)
    cfg.n[0], cfg.n[1], cfg.n[2] = nx, ny, nz
    cfg.odf = int(odf)
    if block is not None:
        bx, by, bz = _dims(block)
        cfg.block[0], cfg.block[1], cfg.block[2] = bx, by, bz
    keep = None
    if blocks is not None:
        arr = (B.od_block * len(blocks))()
        for i, (o, e) in enumerate(blocks):
            for d in range(3):
                arr[i].origin[d] = int(o[d])
                arr[i].extent[d] = int(e[d])
        cfg.blocks = ctypes.cast(arr, ctypes.POINTER(B.od_block))
        cfg.nblocks = len(blocks)
        keep = [arr]
        if cell is not None:
            if len(cell) != len(blocks):
                raise ValueError("one cell size per block")
            carr = (ctypes.c_int32 * len(cell))(*[int(v) for v in cell])
            cfg.block_cell = ctypes.cast(carr, ctypes.POINTER(ctypes.c_int32))
            keep.append(carr)
    elif cell is not None:
        raise ValueError("cell sizes need explicit blocks")
    cfg.dtype = _DTYPES[dtype][0]
    for i in range(6):
        cfg.bc[i] = float(bc[i])
    cfg.seed = int(seed) & (2**64 - 1)
    cfg.exec = B.EXEC[exec]
    if tile is not None:
        for d in range(3):
            cfg.tile[d] = int(tile[d])
    cfg.imbalance_pct = int(imbalance_pct)
    cfg.imbalance_max_extra = int(imbalance_max_extra)
    cfg.hints = int(hints)
    cfg.stencil = int(stencil)
    cfg.wait_s = float(wait_s)
    return cfg, keep


def workspace_bytes(**kw) -> int:
    cfg, _keep = make_config(**kw)
    out = ctypes.c_size_t()
    check(lib().od_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "od_workspace_bytes")
    return int(out.value)


class _PlanHandle:
    """Host-only plan (decomposition, tiles, halo maps); no device needed."""

    def __init__(self, **kw):
        cfg, self._keep = make_config(**kw)
        h = ctypes.c_void_p()
        check(lib().od_plan_create(ctypes.byref(cfg), ctypes.byref(h)), "od_plan_create")
        self.h = h

    def close(self):
        if self.h:
            lib().od_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_info(handle) -> dict:
    info = B.od_plan_info()
    check(lib().od_plan(handle, ctypes.byref(info)), "od_plan")
    return {"nchares": info.nchares, "ntiles": info.ntiles, "npseudo": info.npseudo,
            "interior": info.interior, "halo_cells": info.halo_cells,
            "bytes_per_iter": info.bytes_per_iter, "tile": tuple(info.tile), "grid_wgs": info.grid_wgs,
            "schedule": info.schedule, "coop_waves": info.coop_waves,
            "field_bytes": info.field_bytes, "control_bytes": info.control_bytes,
            "steps_per_pass": info.steps_per_pass, "bytes_per_pass": info.bytes_per_pass}


def tile_infos(handle, count: int) -> list:
    out = []
    ti = B.od_tile_info()
    for t in range(count):
        check(lib().od_tile_info_get(handle, t, ctypes.byref(ti)), "od_tile_info_get")
        out.append({"chare": ti.chare, "origin": tuple(ti.origin), "extent": tuple(ti.extent),
                    "src_kind": tuple(ti.src_kind), "src": tuple(ti.src),
                    "src_origin": tuple(tuple(ti.src_origin[f]) for f in range(6))})
    return out


def tile_deps(handle, count: int) -> list:
    """Message-driven dependency list of every tile (host data)."""
    out = []
    n = ctypes.c_int32()
    for t in range(count):
        check(lib().od_tile_deps(handle, t, None, 0, ctypes.byref(n)), "od_tile_deps")
        buf = (ctypes.c_int32 * max(1, n.value))()
        check(lib().od_tile_deps(handle, t, buf, n.value, ctypes.byref(n)), "od_tile_deps")
        out.append(tuple(buf[:n.value]))
    return out


def chare_boxes(handle, count: int) -> list:
    out = []
    b = B.od_block()
    for c in range(count):
        check(lib().od_chare_get(handle, c, ctypes.byref(b)), "od_chare_get")
        out.append((tuple(b.origin), tuple(b.extent)))
    return out


def extra_sweeps(handle, nchares: int, step: int) -> np.ndarray:
    """Load-imbalance draw of one step: extra sweep re-runs per chare."""
    out = np.zeros(nchares, dtype=np.int32)
    check(lib().od_extra_sweeps(handle, int(step), out.ctypes.data_as(ctypes.c_void_p), int(nchares)),
          "od_extra_sweeps")
    return out


def imbalance_draw(steps: Iterable[int], **kw) -> np.ndarray:
    """Extra sweep re-runs per (step, chare) of a configuration, from a
    host-only plan (rows in the order of `steps`)."""
    p = _PlanHandle(**kw)
    try:
        C = plan_info(p.h)["nchares"]
        return np.stack([extra_sweeps(p.h, C, t) for t in steps])
    finally:
        p.close()


def host_plan(**kw) -> dict:
    """Decomposition and halo maps of a configuration, computed on the host."""
    p = _PlanHandle(**kw)
    try:
        info = plan_info(p.h)
        info["tiles"] = tile_infos(p.h, info["ntiles"])
        info["chares"] = chare_boxes(p.h, info["nchares"])
        if kw.get("exec") == "msgdriven":
            info["deps"] = tile_deps(p.h, info["ntiles"])
        return info
    finally:
        p.close()


class Grid:
    """One GPU's overdecomposed grid: chares with their own storage in a
    caller-owned (PyTorch) device workspace, driven through libod."""

    def __init__(self, n, odf: int = 8, block=None, blocks=None, dtype="f64", bc=DEFAULT_BC,
                 seed: int = 12734, exec: str = "graph", tile=None, imbalance_pct: int = 0,
                 imbalance_max_extra: int = 0, hints: int = 0, stencil: int = 7, device: str = "cuda:0",
                 stream=None, cell=None, wait_s: float = 0.0):
        import torch

        self.n = _dims(n)
        self.dtype = _DTYPES[dtype][1]
        self.exec = exec
        cfg, self._keep = make_config(n=n, odf=odf, block=block, blocks=blocks, dtype=dtype, bc=bc, seed=seed,
                                      exec=exec, tile=tile, imbalance_pct=imbalance_pct,
                                      imbalance_max_extra=imbalance_max_extra, hints=hints, stencil=stencil,
                                      cell=cell, wait_s=wait_s)
        nbytes = ctypes.c_size_t()
        check(lib().od_workspace_bytes(ctypes.byref(cfg), ctypes.byref(nbytes)), "od_workspace_bytes")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().od_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(h)),
                  "od_create")
        self.h = h

    # -- hot path ---------------------------------------------------------
    def iterate(self, n: int) -> None:
        check(lib().od_iterate(self.h, int(n)), "od_iterate")

    def time_iterate(self, n: int) -> float:
        s = ctypes.c_double()
        check(lib().od_time_iterate(self.h, int(n), ctypes.byref(s)), "od_time_iterate")
        return float(s.value)

    def residual(self) -> float:
        r = ctypes.c_double()
        check(lib().od_residual(self.h, ctypes.byref(r)), "od_residual")
        return float(r.value)

    def iterations(self) -> int:
        v = ctypes.c_int64()
        check(lib().od_iterations(self.h, ctypes.byref(v)), "od_iterations")
        return int(v.value)

    # -- I/O --------------------------------------------------------------
    def read(self) -> np.ndarray:
        nx, ny, nz = self.n
        out = np.empty((nz + 2, ny + 2, nx + 2), dtype=self.dtype)
        check(lib().od_read(self.h, out.ctypes.data, out.nbytes), "od_read")
        return out

    def block_cells(self, b: int) -> tuple:
        c = (ctypes.c_int32 * 3)()
        check(lib().od_block_cells(self.h, int(b), c), "od_block_cells")
        return tuple(c)

    def read_block(self, b: int) -> np.ndarray:
        """Chare b's interior cells, shape (cz, cy, cx)."""
        cx, cy, cz = self.block_cells(b)
        out = np.empty((cz, cy, cx), dtype=self.dtype)
        check(lib().od_read_block(self.h, int(b), out.ctypes.data, out.nbytes), "od_read_block")
        return out

    def write_block(self, b: int, A: np.ndarray) -> None:
        cx, cy, cz = self.block_cells(b)
        A = np.ascontiguousarray(A, dtype=self.dtype)
        if A.shape != (cz, cy, cx):
            raise ValueError(f"block shape {A.shape} != {(cz, cy, cx)}")
        check(lib().od_write_block(self.h, int(b), A.ctypes.data, A.nbytes), "od_write_block")

    def write(self, U: np.ndarray) -> None:
        nx, ny, nz = self.n
        U = np.ascontiguousarray(U, dtype=self.dtype)
        if U.shape != (nz + 2, ny + 2, nx + 2):
            raise ValueError(f"field shape {U.shape} != {(nz + 2, ny + 2, nx + 2)}")
        check(lib().od_write(self.h, U.ctypes.data, U.nbytes), "od_write")

    def read_points(self, idx: Iterable[int]) -> np.ndarray:
        idx = np.ascontiguousarray(np.asarray(list(idx) if not isinstance(idx, np.ndarray) else idx,
                                              dtype=np.int64))
        out = np.empty(idx.shape[0], dtype=self.dtype)
        check(lib().od_read_points(self.h, idx.ctypes.data, idx.shape[0], out.ctypes.data), "od_read_points")
        return out

    # -- introspection ----------------------------------------------------
    def plan(self) -> dict:
        return plan_info(self.h)

    def tiles(self) -> list:
        return tile_infos(self.h, self.plan()["ntiles"])

    def timeline(self, max_iters: int = 1024) -> np.ndarray:
        """Persistent grids created with hints bit 3: per iteration of the last
        od_iterate, microseconds to the first / last workgroup start and the
        first / last finish of its tiles (rows of 4)."""
        out = np.zeros((max_iters, 4), dtype=np.float64)
        n = ctypes.c_int32()
        check(lib().od_timeline(self.h, out.ctypes.data_as(ctypes.c_void_p), int(max_iters), ctypes.byref(n)),
              "od_timeline")
        return out[: n.value]

    def autotune(self, iters: int = 3) -> tuple:
        t = (ctypes.c_int32 * 3)()
        check(lib().od_autotune(self.h, int(iters), t), "od_autotune")
        return tuple(t)

    def close(self) -> None:
        if getattr(self, "h", None):
            check(lib().od_destroy(self.h), "od_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid2D(Grid):
    """The paper's Jacobi2D workload: a 5-point stencil on an nx x ny grid,
    stored as an (nx, 1, ny) grid whose second direction is marched in
    registers.  Fields read/written here are 2D padded (ny+2, nx+2) arrays,
    bc = (x-, x+, y-, y+)."""

    def __init__(self, n2, odf: int = 1, dtype="f64", bc=(1.0, 0.0, 0.0, 0.0), **kw):
        nx, ny = (int(n2), int(n2)) if np.isscalar(n2) else (int(n2[0]), int(n2[1]))
        self.n2 = (nx, ny)
        bc3 = (bc[0], bc[1], 0.0, 0.0, bc[2], bc[3])
        super().__init__((nx, 1, ny), odf=odf, dtype=dtype, bc=bc3, stencil=5, **kw)

    def read(self) -> np.ndarray:
        return np.ascontiguousarray(super().read()[:, 1, :])

    def write(self, U: np.ndarray) -> None:
        nx, ny = self.n2
        U = np.asarray(U, dtype=self.dtype)
        if U.shape != (ny + 2, nx + 2):
            raise ValueError(f"field shape {U.shape} != {(ny + 2, nx + 2)}")
        F = np.zeros((ny + 2, 3, nx + 2), dtype=self.dtype)
        F[:, 1, :] = U
        super().write(F)

    def read_points(self, idx) -> np.ndarray:
        # 2D linear index j*nx + i is the 3D index (k*1 + 0)*nx + i with k = j
        return super().read_points(idx)


def stream_copy_seconds(nbytes: int, iters: int = 10, device: str = "cuda:0") -> float:
    """Seconds for `iters` device copies of nbytes with libod's copy kernel."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = ctypes.c_double()
    st = torch.cuda.current_stream(torch.device(device))
    check(lib().od_stream_copy(ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(dst.data_ptr()),
                               ctypes.c_void_p(src.data_ptr()), nbytes, int(iters), ctypes.byref(s)),
          "od_stream_copy")
    return float(s.value)


def hbm_ceilings(nbytes: int = 4 << 30, iters: int = 8, device: str = "cuda:0") -> dict:
    """Measured HBM bandwidth (GB/s) of libod's streaming kernels on buffers
    of nbytes: copy (2 * nbytes per pass), read-only and write-only (nbytes
    per pass); the fastest variant of each, and its index."""
    import torch

    a = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    b = torch.zeros(nbytes, dtype=torch.uint8, device=device)
    st = torch.cuda.current_stream(torch.device(device))
    out = {}
    try:
        for kind, name, mult in ((0, "copy", 2), (1, "read", 1), (2, "write", 1)):
            s = ctypes.c_double()
            v = ctypes.c_int32()
            check(lib().od_stream_bench(ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(b.data_ptr()),
                                        ctypes.c_void_p(a.data_ptr()), int(nbytes), int(iters), kind,
                                        ctypes.byref(s), ctypes.byref(v)), "od_stream_bench")
            out[name + "_gbps"] = round(mult * nbytes * iters / s.value / 1e9, 1)
            out[name + "_variant"] = int(v.value)
    finally:
        del a, b
    out["bytes"] = int(nbytes)
    return out


def launch_overlap(total_threads: int, nkernels: int, nstreams: int | None = None, work: int = 2000,
                   device: str = "cuda:0", return_outputs: bool = False):
    """Kernel-overlap microbenchmark: total_threads threads of `work`
    multiply-adds split into nkernels kernels on min(nstreams, nkernels)
    streams, all released at once.  Returns the od_overlap_result fields as
    a dict (plus the uint32 outputs if asked)."""
    import torch

    from ._binding import od_overlap_result

    nstreams = min(int(nkernels), 64) if nstreams is None else int(nstreams)
    nbytes = int(lib().od_launch_overlap_bytes(int(total_threads)))
    if nbytes == 0:
        raise ValueError("total_threads must be positive")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    res = od_overlap_result()
    with torch.cuda.device(torch.device(device)):
        torch.cuda.synchronize()
        check(lib().od_launch_overlap(ctypes.c_void_p(ws.data_ptr()), nbytes, int(total_threads), int(nkernels),
                                      nstreams, int(work), ctypes.byref(res)), "od_launch_overlap")
    out = {f: getattr(res, f) for f, _ in res._fields_ if f != "pad"}
    if return_outputs:
        out["outputs"] = ws[256:].view(torch.int32).cpu().numpy().view(np.uint32)
    return out


def Server(*args, **kwargs):  # replaced by the serving module once built
    from .serving import Server as _S
    return _S(*args, **kwargs)
