"""Reference oracle for the overdecomposed 3D Jacobi hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_2605_12734_amd``) never imports it and shares no code with it.

It wraps ``jacobi_oracle.c`` (plain C, fp64/fp32, no fusion, no blocking):
the undecomposed Jacobi iteration over one global padded grid that every
overdecomposition of the grid must reproduce exactly (Section III: chares
only change how the work is mapped, not what it computes; Section V,
Jacobi2D: Jacobi iterations with halo exchange).  ``brute.py`` holds a
pure-Python version of the same definition for tiny grids.

Layout of every field handled here: a numpy array of shape
(nz+2, ny+2, nx+2), x fastest, the ghost shell holding the Dirichlet values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "ml_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "libjacobi_oracle.so")
_lib = None

DEFAULT_BC = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def build(force: bool = True) -> str:
    """Compile the C oracle in-tree with the flags its bit-exactness needs."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(f) for f in _SRCS):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64, i64, dp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_splitmix64.argtypes = [u64, u64]
    lib.oracle_splitmix64.restype = u64
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    for suf, ct in (("f64", ctypes.c_double), ("f32", ctypes.c_float)):
        f = getattr(lib, "oracle_init_" + suf)
        f.argtypes = [dp, i64, i64, i64, u64, ctypes.POINTER(ctypes.c_double)]
        f.restype = None
        f = getattr(lib, "oracle_init_box_" + suf)
        f.argtypes = [dp, i64, i64, i64, u64, ctypes.POINTER(ctypes.c_double), i64, i64, i64, i64, i64, i64]
        f.restype = None
        f = getattr(lib, "oracle_sweep_" + suf)
        f.argtypes = [dp, dp, i64, i64, i64]
        f.restype = ct
        f = getattr(lib, "oracle_jacobi_" + suf)
        f.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_double, i64,
                      ctypes.POINTER(ctypes.c_double)]
        f.restype = i64
        f = getattr(lib, "oracle_init2d_" + suf)
        f.argtypes = [dp, i64, i64, u64, ctypes.POINTER(ctypes.c_double)]
        f.restype = None
        f = getattr(lib, "oracle_init2d_box_" + suf)
        f.argtypes = [dp, i64, i64, u64, ctypes.POINTER(ctypes.c_double), i64, i64, i64, i64]
        f.restype = None
        f = getattr(lib, "oracle_sweep2d_" + suf)
        f.argtypes = [dp, dp, i64, i64]
        f.restype = ct
        f = getattr(lib, "oracle_jacobi2d_" + suf)
        f.argtypes = [dp, dp, i64, i64, i64, ctypes.c_double, i64, ctypes.POINTER(ctypes.c_double)]
        f.restype = i64
    _lib = lib
    return lib


def _suffix(dtype) -> str:
    dt = np.dtype(dtype)
    if dt == np.float64:
        return "f64"
    if dt == np.float32:
        return "f32"
    raise ValueError(f"oracle supports float64/float32, not {dt}")


def _dims(n):
    if np.isscalar(n):
        return int(n), int(n), int(n)
    nx, ny, nz = (int(v) for v in n)
    return nx, ny, nz


def splitmix64(seed: int, idx: int) -> int:
    """idx-th output (0-based) of the SplitMix64 stream seeded with seed."""
    return int(_load().oracle_splitmix64(seed & (2**64 - 1), idx))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def init_field(n, dtype=np.float64, seed: int = 12734, bc=DEFAULT_BC) -> np.ndarray:
    """Padded global field: SplitMix64 interior, Dirichlet ghost faces."""
    nx, ny, nz = _dims(n)
    U = np.empty((nz + 2, ny + 2, nx + 2), dtype=dtype)
    bcarr = (ctypes.c_double * 6)(*[float(b) for b in bc])
    getattr(_load(), "oracle_init_" + _suffix(dtype))(
        U.ctypes.data, nx, ny, nz, seed & (2**64 - 1), bcarr)
    return U


def sweep(U: np.ndarray):
    """One sweep of the padded field U; returns (V, residual)."""
    U = np.ascontiguousarray(U)
    nz, ny, nx = (s - 2 for s in U.shape)
    V = U.copy()
    r = getattr(_load(), "oracle_sweep_" + _suffix(U.dtype))(U.ctypes.data, V.ctypes.data, nx, ny, nz)
    return V, float(r)


def jacobi(U: np.ndarray, max_iters: int, tol: float = 0.0, check_every: int = 0):
    """Iterate a copy of the padded field U.

    Stops after iteration ``it`` when ``check_every > 0``,
    ``it % check_every == 0`` and the residual is strictly below ``tol``,
    or after ``max_iters``.  Returns (field, iterations, residual).
    """
    A = np.array(U, copy=True, order="C")
    B = np.empty_like(A)
    nz, ny, nx = (s - 2 for s in A.shape)
    r = ctypes.c_double(0.0)
    it = getattr(_load(), "oracle_jacobi_" + _suffix(A.dtype))(
        A.ctypes.data, B.ctypes.data, nx, ny, nz, int(max_iters), float(tol),
        int(check_every), ctypes.byref(r))
    return A, int(it), float(r.value)


def solve(n, dtype=np.float64, seed: int = 12734, iters: int = 100, bc=DEFAULT_BC,
          tol: float = 0.0, check_every: int = 0):
    """init_field + jacobi in one call: (field, iterations, residual)."""
    return jacobi(init_field(n, dtype, seed, bc), iters, tol, check_every)


def point_values(n, points, iters: int, dtype=np.float64, seed: int = 12734, bc=DEFAULT_BC):
    """Values after `iters` sweeps at interior points (i, j, k) of the global
    grid, each from a sub-box around the point: by domain of dependence a
    point's value after t sweeps depends only on cells within Chebyshev
    distance t, so the box's own shell (distance t+1, or the Dirichlet shell)
    may stay at its initial values."""
    nx, ny, nz = _dims(n)
    bcarr = (ctypes.c_double * 6)(*[float(b) for b in bc])
    out = []
    for (i, j, k) in points:
        lo = [max(0, v - iters) for v in (i, j, k)]
        hi = [min(m - 1, v + iters) for v, m in zip((i, j, k), (nx, ny, nz))]
        bx, by, bz = (h - l + 1 for h, l in zip(hi, lo))
        U = np.empty((bz + 2, by + 2, bx + 2), dtype=dtype)
        getattr(_load(), "oracle_init_box_" + _suffix(dtype))(
            U.ctypes.data, nx, ny, nz, seed & (2**64 - 1), bcarr, lo[0], lo[1], lo[2], bx, by, bz)
        V, _, _ = jacobi(U, iters)
        out.append(V[k - lo[2] + 1, j - lo[1] + 1, i - lo[0] + 1])
    return np.array(out, dtype=dtype)


# ---- Jacobi2D (Section V): 5-point stencil on an (ny+2, nx+2) padded field --

DEFAULT_BC2D = (1.0, 0.0, 0.0, 0.0)


def init_field2d(n2, dtype=np.float64, seed: int = 12734, bc=DEFAULT_BC2D) -> np.ndarray:
    nx, ny = (int(n2), int(n2)) if np.isscalar(n2) else (int(n2[0]), int(n2[1]))
    U = np.empty((ny + 2, nx + 2), dtype=dtype)
    bcarr = (ctypes.c_double * 4)(*[float(b) for b in bc])
    getattr(_load(), "oracle_init2d_" + _suffix(dtype))(U.ctypes.data, nx, ny, seed & (2**64 - 1), bcarr)
    return U


def sweep2d(U: np.ndarray):
    U = np.ascontiguousarray(U)
    ny, nx = (s - 2 for s in U.shape)
    V = U.copy()
    r = getattr(_load(), "oracle_sweep2d_" + _suffix(U.dtype))(U.ctypes.data, V.ctypes.data, nx, ny)
    return V, float(r)


def jacobi2d(U: np.ndarray, max_iters: int, tol: float = 0.0, check_every: int = 0):
    A = np.array(U, copy=True, order="C")
    B = np.empty_like(A)
    ny, nx = (s - 2 for s in A.shape)
    r = ctypes.c_double(0.0)
    it = getattr(_load(), "oracle_jacobi2d_" + _suffix(A.dtype))(
        A.ctypes.data, B.ctypes.data, nx, ny, int(max_iters), float(tol), int(check_every), ctypes.byref(r))
    return A, int(it), float(r.value)


def solve2d(n2, dtype=np.float64, seed: int = 12734, iters: int = 100, bc=DEFAULT_BC2D, tol: float = 0.0,
            check_every: int = 0):
    return jacobi2d(init_field2d(n2, dtype, seed, bc), iters, tol, check_every)


def point_values2d(n2, points, iters: int, dtype=np.float64, seed: int = 12734, bc=DEFAULT_BC2D):
    """2D analogue of point_values: each (i, j) after `iters` sweeps from a
    sub-box of half-width iters (domain of dependence)."""
    nx, ny = int(n2[0]), int(n2[1])
    bcarr = (ctypes.c_double * 4)(*[float(b) for b in bc])
    out = []
    for (i, j) in points:
        lo = [max(0, i - iters), max(0, j - iters)]
        hi = [min(nx - 1, i + iters), min(ny - 1, j + iters)]
        bx, by = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1
        U = np.empty((by + 2, bx + 2), dtype=dtype)
        getattr(_load(), "oracle_init2d_box_" + _suffix(dtype))(
            U.ctypes.data, nx, ny, seed & (2**64 - 1), bcarr, lo[0], lo[1], bx, by)
        V, _, _ = jacobi2d(U, iters)
        out.append(V[j - lo[1] + 1, i - lo[0] + 1])
    return np.array(out, dtype=dtype)


# ---- multi-resolution blocks (ml_oracle.c) ----------------------------------

def _ml_lib():
    lib = _load()
    if not getattr(lib, "_ml_ready", False):
        i64, u64, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.oracle_ml_layout.argtypes = [i64, dp, dp, dp]
        lib.oracle_ml_layout.restype = i64
        for suf in ("f64", "f32"):
            f = getattr(lib, "oracle_ml_init_" + suf)
            f.argtypes = [dp, i64, dp, dp, dp, dp, i64, i64, i64, u64]
            f.restype = None
            f = getattr(lib, "oracle_ml_jacobi_" + suf)
            f.argtypes = [dp, dp, i64, dp, dp, dp, dp, i64, i64, i64, ctypes.POINTER(ctypes.c_double), i64,
                          ctypes.POINTER(ctypes.c_double)]
            f.restype = i64
        lib._ml_ready = True
    return lib


class MLGrid:
    """Multi-resolution blocks: `blocks` = [(origin, extent)] in grid units,
    `cell` = cell edge (units, power of two) per block.  Holds every block's
    padded array in one flat buffer (see ml_oracle.c)."""

    def __init__(self, n, blocks, cell, dtype=np.float64, seed: int = 12734, bc=DEFAULT_BC):
        self.n = _dims(n)
        self.dtype = np.dtype(dtype)
        self.org = np.ascontiguousarray([list(o) for o, _ in blocks], dtype=np.int64)
        self.ext = np.ascontiguousarray([list(e) for _, e in blocks], dtype=np.int64)
        self.h = np.ascontiguousarray(list(cell), dtype=np.int64)
        if len(self.h) != len(blocks):
            raise ValueError("one cell size per block")
        if np.any(self.ext % self.h[:, None]) or np.any(self.org % self.h[:, None]):
            raise ValueError("block origins and extents must be multiples of their cell size")
        self.m = self.ext // self.h[:, None]
        self.offs = np.zeros(len(blocks), dtype=np.int64)
        lib = _ml_lib()
        total = lib.oracle_ml_layout(len(blocks), self.ext.ctypes.data, self.h.ctypes.data, self.offs.ctypes.data)
        self.U = np.zeros(int(total), dtype=self.dtype)
        self.bc = (ctypes.c_double * 6)(*[float(v) for v in bc])
        getattr(lib, "oracle_ml_init_" + _suffix(self.dtype))(
            self.U.ctypes.data, len(blocks), self.org.ctypes.data, self.ext.ctypes.data, self.h.ctypes.data,
            self.offs.ctypes.data, *self.n, int(seed) & (2**64 - 1))
        self.iters = 0
        self.residual = 0.0

    def block(self, b: int) -> np.ndarray:
        """View of block b's padded array, shape (mz+2, my+2, mx+2)."""
        mx, my, mz = (int(v) for v in self.m[b])
        o = int(self.offs[b])
        return self.U[o:o + (mx + 2) * (my + 2) * (mz + 2)].reshape(mz + 2, my + 2, mx + 2)

    def interior(self, b: int) -> np.ndarray:
        return self.block(b)[1:-1, 1:-1, 1:-1].copy()

    def jacobi(self, iters: int) -> float:
        V = np.zeros_like(self.U)
        r = ctypes.c_double()
        lib = _ml_lib()
        done = getattr(lib, "oracle_ml_jacobi_" + _suffix(self.dtype))(
            self.U.ctypes.data, V.ctypes.data, len(self.h), self.org.ctypes.data, self.ext.ctypes.data,
            self.h.ctypes.data, self.offs.ctypes.data, *self.n, self.bc, int(iters), ctypes.byref(r))
        if done < 0:
            raise ValueError("block layout not covered: blocks must tile the domain, and across a "
                             "resolution change the finer block must align to the coarser cells")
        self.iters += int(done)
        self.residual = float(r.value) if done > 0 else self.residual
        return self.residual
