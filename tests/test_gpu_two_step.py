"""Two Jacobi steps per pass (the fused, graph, persistent and message-driven
forms' default where blocks are at one resolution, also under load imbalance):
the pass reads the field once, keeps the first step on chip and writes the
second.  Every case is compared with the CPU oracle bit for bit (0 ULP),
with odd and even iteration counts (an odd count ends with a single sweep),
ragged tiles, tiles of extent 1, chares of extent 1 (the cells two steps
out then lie two chares away), distinct Dirichlet values on all six faces
(the first step of a boundary ring is the boundary value), and every
compiled two-step tile shape."""
import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od
import workloads

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}
BC6 = (1.0, 0.5, 0.25, 0.125, 2.0, 3.0)
VARIANTS = {"f64": [(32, 32), (32, 16), (32, 8), (64, 8), (64, 16), (16, 16)],
            "f32": [(32, 32), (32, 16), (64, 16)]}


def _same(U, want):
    if not np.array_equal(U, want):
        d = np.argwhere(U != want)
        k, j, i = d[0]
        raise AssertionError(f"{len(d)} cells differ; first at padded (k,j,i)=({k},{j},{i}): "
                             f"{U[k, j, i]!r} vs {want[k, j, i]!r}")


def _case(n, odf, dtype, iters, exec_="fused", tile=None, bc=od.DEFAULT_BC, seed=12734, hints=1):
    want, it_w, r_w = oracle.solve(n, DT[dtype], seed=seed, iters=iters, bc=bc)
    kw = {"tile": tile} if tile else {}
    g = od.Grid(n, odf=odf, dtype=dtype, exec=exec_, bc=bc, seed=seed, hints=hints, **kw)
    try:
        plan = g.plan()
        g.iterate(iters)
        r = g.residual()
        U = g.read()
        it = g.iterations()
    finally:
        g.close()
    _same(U, want)
    assert it == it_w == iters and r == r_w
    return plan


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [1, 2, 5, 12])
@pytest.mark.parametrize("exec_", ["fused", "graph"])
def test_64cubed_2x2x2(dtype, iters, exec_):
    plan = _case(64, 8, dtype, iters, exec_)
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,odf", [((37, 21, 19), 8), ((150, 90, 70), 27), ((12, 6, 5), 27), ((9, 8, 7), 27),
                                   ((1, 1, 1), 1), ((2, 2, 2), 8), ((3, 1, 4), 1), ((40, 3, 33), 8)])
def test_ragged_and_tiny_six_boundary_values(dtype, n, odf):
    plan = _case(n, odf, dtype, 7, tile=(32, 16, 8), bc=BC6, seed=5)
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_every_two_step_variant(dtype):
    # 70 x 45 x 33 over 8 chares: ragged tiles of every shape, z tiles of 1
    for tx, ty in VARIANTS[dtype]:
        for tz in (16, 34):
            plan = _case((70, 45, 33), 8, dtype, 6, tile=(tx, ty, tz), bc=BC6, seed=3)
            assert plan["steps_per_pass"] == 2 and tuple(plan["tile"]) == (tx, ty, tz)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tile_extent_one_on_every_axis(dtype):
    # chares of 33 x 17 x 9 with tiles (32, 16, 8): a last tile of extent 1
    # along each axis, whose ring two cells out lies in the next chare
    _case((66, 34, 18), 8, dtype, 5, tile=(32, 16, 8), bc=BC6, seed=11)


@pytest.mark.parametrize("exec_", ["fused", "graph"])
def test_one_step_hint_and_pairs_identical_at_256(exec_):
    out = []
    for hints in (1, 1 | od.HINT_ONE_STEP):
        g = od.Grid(256, odf=512, dtype="f64", exec=exec_, hints=hints, tile=(32, 32, 32))
        try:
            g.iterate(9)
            out.append((g.read(), g.residual(), g.plan()["steps_per_pass"]))
        finally:
            g.close()
    (a, ra, sa), (b, rb, sb) = out
    assert sa == 2 and sb == 1
    assert np.array_equal(a, b) and ra == rb


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [1, 2, 7, 12])
@pytest.mark.parametrize("hints,sched", [(1, 2), (1 | 8192, 1)])
def test_persistent_pairs(dtype, iters, hints, sched):
    # default: tiles from per-XCD counters claimed as each tile ends;
    # hints bit 13: the fixed stride
    plan = _case(64, 8, dtype, iters, exec_="persistent", hints=hints)
    assert plan["steps_per_pass"] == 2 and plan["schedule"] == sched


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [2, 7])
def test_persistent_pairs_counters(dtype, iters):
    # hints bit 4: tiles taken from per-XCD counters, pass by pass
    plan = _case((150, 90, 70), 27, dtype, iters, exec_="persistent", tile=(32, 16, 16), bc=BC6, seed=9,
                 hints=1 | 16)
    assert plan["steps_per_pass"] == 2 and plan["schedule"] == 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_persistent_pairs_ragged(dtype):
    plan = _case((150, 90, 70), 27, dtype, 9, exec_="persistent", tile=(32, 16, 16), bc=BC6, seed=7)
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("iters", [6, 7])
def test_persistent_pairs_guided_tail(iters):
    # hints bit 5 with two steps per pass: each XCD group's partial last
    # round of tiles is cut into z-ranges (384^3 as 1728 chares of 32^3:
    # 216 tiles per group on 96 workgroups, the last 24 cut into 4 pieces)
    n = 384
    want, _, r_w = oracle.solve(n, np.float64, seed=5, iters=iters, bc=od.DEFAULT_BC)
    g = od.Grid(n, odf=1728, dtype="f64", exec="persistent", tile=(32, 32, 32), hints=1 | 32, seed=5)
    try:
        p = g.plan()
        g.iterate(iters)
        U, r = g.read(), g.residual()
    finally:
        g.close()
    assert p["steps_per_pass"] == 2 and p["schedule"] == 3
    assert p["ntiles"] > 1728
    _same(U, want)
    assert r == r_w


def test_persistent_pairs_then_single_steps_resume():
    # a persistent grid run in pieces (pairs, then an odd step, then pairs)
    # ends on the oracle's bits
    want, _, r_w = oracle.solve(64, np.float64, seed=12734, iters=11, bc=od.DEFAULT_BC)
    g = od.Grid(64, odf=64, dtype="f64", exec="persistent", hints=1)
    try:
        for k in (4, 3, 4):
            g.iterate(k)
        U, r = g.read(), g.residual()
    finally:
        g.close()
    _same(U, want)
    assert r == r_w


def test_not_used_where_unsupported():
    # a forced persistent schedule, the one-step hint and the per-chare form
    # keep one step per pass
    for kw in ({"exec": "persistent", "hints": 2048}, {"exec": "msgdriven", "hints": 4096},
               {"exec": "per_chare"}):
        g = od.Grid(64, odf=8, dtype="f64", **kw)
        try:
            assert g.plan()["steps_per_pass"] == 1
        finally:
            g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("exec_,hints", [("fused", 1), ("persistent", 1), ("persistent", 1 | 8192),
                                         ("persistent", 1 | 16), ("msgdriven", 1), ("msgdriven", 1 | 4)])
def test_pairs_under_imbalance(dtype, exec_, hints):
    # half the chares drawn heavy each step, 1-3 extra runs: a heavy chare's
    # extra one-step sweeps write its own cells of the pass's output parity
    # before the pass overwrites them; 9 iterations (four passes and a single
    # step), then 4 more (the draw continues at step 9)
    n, odf, seed = (70, 45, 38), 27, 5
    want, _, r_w = oracle.solve(n, DT[dtype], seed=seed, iters=13)
    g = od.Grid(n, odf=odf, dtype=dtype, exec=exec_, seed=seed, hints=hints, imbalance_pct=50,
                imbalance_max_extra=3)
    try:
        assert g.plan()["steps_per_pass"] == 2
        g.iterate(9)
        g.iterate(4)
        U, r = g.read(), g.residual()
        assert g.iterations() == 13
    finally:
        g.close()
    _same(U, want)
    assert r == r_w


def test_bytes_per_pass_counts_two_step_reach():
    # 64^3 as 2x2x2 chares of 32^3: every chare has 3 inner faces (two
    # layers each) and 3 inner edges
    g = od.Grid(64, odf=8, dtype="f64", exec="fused")
    try:
        p = g.plan()
    finally:
        g.close()
    per_chare = 3 * 2 * 32 * 32 + 3 * 32
    assert p["bytes_per_pass"] == 8 * (2 * 64 ** 3 + 8 * per_chare)
    assert p["bytes_per_iter"] == 8 * (2 * 64 ** 3 + 8 * 3 * 32 * 32)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("exec_", ["fused", "graph", "persistent", "msgdriven"])
@pytest.mark.parametrize("tile", [(16, 16, 8), (32, 16, 16), (32, 32, 32)])
def test_uneven_octree_pairs(dtype, exec_, tile):
    # explicit blocks at one resolution: tiles are cut until every line of
    # cells a pair reads lies in one block
    if dtype == "f32" and tile == (16, 16, 8):
        tile = (32, 16, 8)
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.5, seed=7)
    want, _, r_w = oracle.solve(96, DT[dtype], seed=3, iters=9, bc=BC6)
    g = od.Grid(96, blocks=blocks, dtype=dtype, exec=exec_, tile=tile, bc=BC6, seed=3, hints=1)
    try:
        assert g.plan()["steps_per_pass"] == 2
        g.iterate(9)
        U, r = g.read(), g.residual()
    finally:
        g.close()
    _same(U, want)
    assert r == r_w


@pytest.mark.parametrize("exec_", ["graph", "persistent"])
def test_1024_odf32768_pairs_sampled(exec_):
    # full size: 1024^3 fp64 as 32768 chares of 32^3, 13 iterations (six
    # pairs and a single step), points in chare interiors and on chare
    # faces, edges and corners, where the pairs read diagonal neighbours
    n = (1024, 1024, 1024)
    iters = 13
    rng = np.random.default_rng(21)
    pts = [tuple(int(v) for v in rng.integers(0, 1024, 3)) for _ in range(24)]
    for c in (31, 32, 63, 64, 511, 512, 991, 992):
        pts += [(c, c, c), (c, c, 100), (c, 7, c), (300, c, c), (0, c, c), (c, 1023, 0)]
    g = od.Grid(n, odf=32768, dtype="f64", exec=exec_, tile=(32, 32, 32), hints=1)
    try:
        assert g.plan()["steps_per_pass"] == 2
        g.iterate(iters)
        got = g.read_points(np.array([(k * n[1] + j) * n[0] + i for (i, j, k) in pts], dtype=np.int64))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [1, 2, 7, 12])
def test_msgdriven_pairs(dtype, iters):
    # message-driven tasks of two steps (an odd count ends with a one-step
    # launch on the same grid)
    plan = _case(64, 8, dtype, iters, exec_="msgdriven")
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_msgdriven_pairs_ragged(dtype):
    plan = _case((150, 90, 70), 27, dtype, 9, exec_="msgdriven", tile=(32, 16, 16), bc=BC6, seed=7)
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("hints", [1 | 64, 1 | 128, 1 | 128 | 512, 1 | 64 | 1024, 1 | 4])
def test_msgdriven_pairs_schedulers(hints):
    # cursor and ready-queue claims, publisher on and off, and the seeded
    # schedule perturbation with its step-window check
    plan = _case(128, 64, "f64", 10, exec_="msgdriven", tile=(16, 16, 16), hints=hints, seed=3)
    assert plan["steps_per_pass"] == 2


def test_msgdriven_pairs_then_single_steps_resume():
    # pairs, a single step, pairs: the tiles' step counters follow both kernels
    want, _, r_w = oracle.solve((96, 64, 48), np.float64, seed=31, iters=9, bc=BC6)
    g = od.Grid((96, 64, 48), odf=27, dtype="f64", exec="msgdriven", bc=BC6, seed=31, hints=1)
    try:
        for k in (3, 4, 2):
            g.iterate(k)
        U, r, it = g.read(), g.residual(), g.iterations()
        assert g.plan()["steps_per_pass"] == 2
    finally:
        g.close()
    _same(U, want)
    assert r == r_w and it == 9


def test_512_odf4096_msgdriven_pairs_sampled():
    n = (512, 512, 512)
    iters = 20
    rng = np.random.default_rng(5)
    pts = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(24)]
    for c in (31, 32, 255, 256, 480, 511):
        pts += [(c, c, c), (c, 0, c), (0, c, 100), (c, 511, 7)]
    g = od.Grid(n, odf=4096, dtype="f64", exec="msgdriven", tile=(32, 16, 32), hints=1)
    try:
        assert g.plan()["steps_per_pass"] == 2
        g.iterate(iters)
        got = g.read_points(np.array([(k * n[1] + j) * n[0] + i for (i, j, k) in pts], dtype=np.int64))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64)
    assert np.array_equal(got, want)
