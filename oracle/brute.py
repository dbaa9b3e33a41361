"""Pure-Python brute force of the oracle's definition, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Plain nested loops over Python floats (fp64) or numpy.float32 scalars
(fp32, each operation rounded to single precision).  It restates the same
definition as ``jacobi_oracle.c`` independently: 7-point mean of the face
neighbours added in the order x-, x+, y-, y+, z-, z+, then divided by 6;
Dirichlet ghost shell held fixed; residual = max |u_new - u_old|; initial
interior from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, idx: int) -> int:
    z = (seed + (idx + 1) * _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def unif(h: int, dtype) -> float:
    if np.dtype(dtype) == np.float64:
        return float(h >> 11) * 2.0 ** -53
    return np.float32(h >> 40) * np.float32(2.0 ** -24)


def init_field(nx, ny, nz, dtype, seed, bc):
    T = np.float64 if np.dtype(dtype) == np.float64 else np.float32
    U = [[[T(0) for _ in range(nx + 2)] for _ in range(ny + 2)] for _ in range(nz + 2)]
    for k in range(-1, nz + 1):
        for j in range(-1, ny + 1):
            for i in range(-1, nx + 1):
                outs = [i < 0 or i >= nx, j < 0 or j >= ny, k < 0 or k >= nz]
                if sum(outs) == 0:
                    v = T(unif(splitmix64(seed, (k * ny + j) * nx + i), T))
                elif sum(outs) >= 2:
                    v = T(0)
                elif i < 0:
                    v = T(bc[0])
                elif i >= nx:
                    v = T(bc[1])
                elif j < 0:
                    v = T(bc[2])
                elif j >= ny:
                    v = T(bc[3])
                elif k < 0:
                    v = T(bc[4])
                else:
                    v = T(bc[5])
                U[k + 1][j + 1][i + 1] = v
    return U


def sweep(U):
    nz, ny, nx = len(U) - 2, len(U[0]) - 2, len(U[0][0]) - 2
    T = type(U[1][1][1])
    V = [[list(row) for row in plane] for plane in U]
    r = T(0)
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for i in range(1, nx + 1):
                s = U[k][j][i - 1]
                s = T(s + U[k][j][i + 1])
                s = T(s + U[k][j - 1][i])
                s = T(s + U[k][j + 1][i])
                s = T(s + U[k - 1][j][i])
                s = T(s + U[k + 1][j][i])
                v = T(s / T(6))
                d = abs(T(v - U[k][j][i]))
                if d > r:
                    r = d
                V[k][j][i] = v
    return V, r


def jacobi(U, max_iters, tol=0.0, check_every=0):
    r = 0.0
    it = 0
    while it < max_iters:
        U, r = sweep(U)
        it += 1
        if check_every > 0 and it % check_every == 0 and float(r) < tol:
            break
    return U, it, float(r)


def to_numpy(U, dtype):
    return np.array(U, dtype=dtype)


# ---- Jacobi2D: 5-point, order x-, x+, y-, y+, divided by 4 ------------------

def init_field2d(nx, ny, dtype, seed, bc):
    T = np.float64 if np.dtype(dtype) == np.float64 else np.float32
    U = [[T(0) for _ in range(nx + 2)] for _ in range(ny + 2)]
    for j in range(-1, ny + 1):
        for i in range(-1, nx + 1):
            outs = (i < 0 or i >= nx) + (j < 0 or j >= ny)
            if outs == 0:
                v = T(unif(splitmix64(seed, j * nx + i), T))
            elif outs == 2:
                v = T(0)
            elif i < 0:
                v = T(bc[0])
            elif i >= nx:
                v = T(bc[1])
            elif j < 0:
                v = T(bc[2])
            else:
                v = T(bc[3])
            U[j + 1][i + 1] = v
    return U


def sweep2d(U):
    ny, nx = len(U) - 2, len(U[0]) - 2
    T = type(U[1][1])
    V = [list(row) for row in U]
    r = T(0)
    for j in range(1, ny + 1):
        for i in range(1, nx + 1):
            s = U[j][i - 1]
            s = T(s + U[j][i + 1])
            s = T(s + U[j - 1][i])
            s = T(s + U[j + 1][i])
            v = T(s / T(4))
            d = abs(T(v - U[j][i]))
            if d > r:
                r = d
            V[j][i] = v
    return V, r
