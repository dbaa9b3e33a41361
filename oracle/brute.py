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


# ---- multi-resolution blocks: injection from coarser, face mean of finer ----

def ml_init(n, blocks, cell, dtype, seed):
    """Per block: padded nested list [k][j][i] (ghosts 0), cell (i,j,k) from
    SplitMix64 at the unit index of its lower corner."""
    nx, ny, _ = n
    T = np.float64 if np.dtype(dtype) == np.float64 else np.float32
    out = []
    for (o, e), h in zip(blocks, cell):
        mx, my, mz = e[0] // h, e[1] // h, e[2] // h
        A = [[[T(0) for _ in range(mx + 2)] for _ in range(my + 2)] for _ in range(mz + 2)]
        for k in range(mz):
            for j in range(my):
                for i in range(mx):
                    q = (o[0] + i * h, o[1] + j * h, o[2] + k * h)
                    A[k + 1][j + 1][i + 1] = T(unif(splitmix64(seed, (q[2] * ny + q[1]) * nx + q[0]), T))
        out.append(A)
    return out


def _ml_owner(blocks, p):
    for b, (o, e) in enumerate(blocks):
        if all(o[d] <= p[d] < o[d] + e[d] for d in range(3)):
            return b
    raise ValueError("point not covered")


def ml_step(n, blocks, cell, A, bc):
    """One iteration: fill every ghost layer, then the 7-point update."""
    T = type(A[0][1][1][1])
    for b, ((o, e), h) in enumerate(zip(blocks, cell)):
        m = [e[d] // h for d in range(3)]
        for f in range(6):
            d, hi = f // 2, f % 2
            t1, t2 = [q for q in range(3) if q != d]
            for c2 in range(m[t2]):
                for c1 in range(m[t1]):
                    p = [0, 0, 0]
                    p[t1] = o[t1] + c1 * h
                    p[t2] = o[t2] + c2 * h
                    p[d] = o[d] + e[d] if hi else o[d] - 1
                    if p[d] < 0 or p[d] >= n[d]:
                        v = T(bc[f])
                    else:
                        N = _ml_owner(blocks, p)
                        (oN, _), hN = blocks[N], cell[N]
                        base = [(p[q] - oN[q]) // hN for q in range(3)]
                        B = A[N]
                        if hN >= h:
                            v = B[base[2] + 1][base[1] + 1][base[0] + 1]
                        else:
                            r = h // hN
                            s = None
                            for q2 in range(r):
                                for q1 in range(r):
                                    w = list(base)
                                    w[t1] += q1
                                    w[t2] += q2
                                    x = B[w[2] + 1][w[1] + 1][w[0] + 1]
                                    s = x if s is None else T(s + x)
                            v = T(s / T(r * r))
                    g = [0, 0, 0]
                    g[t1], g[t2] = c1 + 1, c2 + 1
                    g[d] = m[d] + 1 if hi else 0
                    A[b][g[2]][g[1]][g[0]] = v
    res = T(0)
    out = []
    for b, ((o, e), h) in enumerate(zip(blocks, cell)):
        U, ret = sweep(A[b])
        res = max(res, ret)
        out.append(U)
    return out, float(res)


def ml_jacobi(n, blocks, cell, A, iters, bc):
    r = 0.0
    for _ in range(iters):
        A, r = ml_step(n, blocks, cell, A, bc)
    return A, r
