"""Seeded synthetic workload generators shared by tests and the benchmark.

This module holds no arithmetic of the method: it only draws the
*structure* of workloads (uneven AMR-like block layouts, serving request
streams) from seeds.  Both the GPU path and the CPU oracle consume what it
produces; neither is imported here.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
keyed by (stream tag, counter), so every draw is reproducible and
independent of call order.
"""
from __future__ import annotations

import math
from typing import List, Tuple

_M64 = (1 << 64) - 1


def splitmix64(seed: int, idx: int) -> int:
    z = (seed + (idx + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def uniform(seed: int, idx: int) -> float:
    """U[0,1) with 53 random bits."""
    return (splitmix64(seed, idx) >> 11) * 2.0 ** -53


def derive(seed: int, tag: int) -> int:
    """Independent sub-seed for a named stream."""
    return splitmix64(seed ^ 0xA5A5A5A5DEADBEEF, tag)


# ---------------------------------------------------------------------------
# AMR-like uneven blocks: octree refinement of a cubic domain

Block = Tuple[Tuple[int, int, int], Tuple[int, int, int]]


def octree_blocks(n: int = 768, root: int = 128, min_edge: int = 16, p_refine: float = 0.4,
                  seed: int = 12734) -> List[Block]:
    """Octree refinement of an n^3 domain into cubic blocks.

    The domain is first cut into (n/root)^3 root blocks.  Level by level,
    blocks are visited in (z, y, x) origin order and each block with edge
    above `min_edge` draws one uniform number; below `p_refine` it splits
    into 8 children of half the edge.  All blocks share one resolution; only
    their sizes differ (edges root, root/2, ..., min_edge).
    """
    if n % root or root % min_edge:
        raise ValueError("n must be a multiple of root and root of min_edge")
    s = derive(seed, 1)
    level = [((x, y, z), root) for z in range(0, n, root) for y in range(0, n, root) for x in range(0, n, root)]
    done: List[Block] = []
    draw = 0
    while level:
        level.sort(key=lambda b: (b[0][2], b[0][1], b[0][0]))
        nxt = []
        for (o, e) in level:
            if e > min_edge and uniform(s, draw) < p_refine:
                h = e // 2
                for dz in (0, h):
                    for dy in (0, h):
                        for dx in (0, h):
                            nxt.append(((o[0] + dx, o[1] + dy, o[2] + dz), h))
            else:
                done.append((o, (e, e, e)))
            draw += 1
        level = nxt
    done.sort(key=lambda b: (b[0][2], b[0][1], b[0][0]))
    return done


def expected_octree_leaves(n: int = 768, root: int = 128, min_edge: int = 16, p: float = 0.4) -> dict:
    """Expected number of leaves per edge (closed form of the branching process)."""
    roots = (n // root) ** 3
    out = {}
    alive = float(roots)
    e = root
    while e >= min_edge:
        if e == min_edge:
            out[e] = alive
        else:
            out[e] = alive * (1 - p)
            alive = alive * p * 8
        e //= 2
    return out


# ---------------------------------------------------------------------------
# serving: Poisson stream of independent solves


def serving_requests(rate: float, count: int, seed: int = 12734, n_lo: int = 32, n_hi: int = 384,
                     odfs=(1, 8, 64), tol: float = 1e-6, max_iters: int = 2000, check_every: int = 10):
    """`count` requests with exponential inter-arrival gaps of mean 1/rate.

    Sizes are log-uniform cubes in [n_lo, n_hi]; dtype fp32/fp64 with
    probability 1/2; ODF uniform over `odfs` (reduced so that every chare
    has at least one cell per dimension); each request gets its own field
    seed.
    """
    s = derive(seed, 2)
    t = 0.0
    out = []
    for i in range(count):
        u = uniform(s, 5 * i)
        t += -math.log(1.0 - u) / rate
        n = int(round(n_lo * (n_hi / n_lo) ** uniform(s, 5 * i + 1)))
        dtype = "f32" if uniform(s, 5 * i + 2) < 0.5 else "f64"
        odf = odfs[min(len(odfs) - 1, int(uniform(s, 5 * i + 3) * len(odfs)))]
        while round(odf ** (1 / 3)) > n:
            odf //= 8
        out.append({"id": i, "t_arrival": t, "n": n, "dtype": dtype, "odf": max(1, odf), "tol": tol,
                    "max_iters": max_iters, "check_every": check_every,
                    "seed": splitmix64(s, 5 * i + 4)})
    return out
