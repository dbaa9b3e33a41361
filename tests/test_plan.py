"""Host-side decomposition and halo maps, checked by brute force (no GPU).

Every tile face names the chare (or Dirichlet face) its ghost slab is read
from and the slab's global origin.  The checks fill a global index map and
verify, cell by cell, that each ghost cell is the face neighbour of the
tile's boundary cell and lies inside the named source chare; that the tiles
partition every chare; and that the ghost cells read from other chares are
exactly the chare-face cells of the decomposition, each read once.
"""
import json
import os

import numpy as np
import pytest

import paper_2605_12734_amd as od
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _owner_map(n, chares):
    nx, ny, nz = n
    own = -np.ones((nz, ny, nx), dtype=np.int64)
    for c, (o, e) in enumerate(chares):
        sl = own[o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]]
        assert np.all(sl == -1), "chares overlap"
        sl[...] = c
    assert np.all(own >= 0), "chares do not cover the domain"
    return own


def _check_plan(n, plan):
    nx, ny, nz = n
    own = _owner_map(n, plan["chares"])
    covered = np.zeros((nz, ny, nx), dtype=np.int64)
    ghost_reads = {}
    halo = 0
    for t in plan["tiles"]:
        c = t["chare"]
        co, ce = plan["chares"][c]
        o = [co[d] + t["origin"][d] for d in range(3)]
        e = t["extent"]
        for d in range(3):
            assert 0 <= t["origin"][d] and t["origin"][d] + e[d] <= ce[d]
        covered[o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]] += 1
        for f in range(6):
            d = f // 2
            lo = list(o)
            ext = list(e)
            lo[d] = o[d] - 1 if f % 2 == 0 else o[d] + e[d]
            ext[d] = 1
            assert tuple(t["src_origin"][f]) == tuple(lo), (t, f)
            cells = [(x, y, z) for z in range(lo[2], lo[2] + ext[2]) for y in range(lo[1], lo[1] + ext[1])
                     for x in range(lo[0], lo[0] + ext[0])]
            if t["src_kind"][f] == 1:
                # Dirichlet face f of the domain: the slab lies just outside it
                assert t["src"][f] == f
                v = lo[d]
                assert v == -1 if f % 2 == 0 else v == n[d]
            else:
                src = t["src"][f]
                for (x, y, z) in cells:
                    assert 0 <= x < nx and 0 <= y < ny and 0 <= z < nz
                    assert own[z, y, x] == src
                if src != c:
                    halo += len(cells)
                    for cell in cells:
                        ghost_reads[(c, f, cell)] = ghost_reads.get((c, f, cell), 0) + 1
    assert np.all(covered == 1), "tiles must partition the domain"
    # every chare-face ghost cell (owned by another chare) is read exactly once
    expect = 0
    for c, (co, ce) in enumerate(plan["chares"]):
        for f in range(6):
            d = f // 2
            v = co[d] - 1 if f % 2 == 0 else co[d] + ce[d]
            if v < 0 or v >= n[d]:
                continue
            expect += ce[0] * ce[1] * ce[2] // ce[d]
    assert halo == expect == plan["halo_cells"]
    assert all(k == 1 for k in ghost_reads.values())


@pytest.mark.parametrize("n,odf", [((13, 11, 9), 8), ((16, 16, 16), 64), ((7, 5, 9), 12), ((33, 4, 5), 8),
                                   ((9, 9, 9), 1), ((10, 10, 10), 27)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_regular_halo_maps_brute_force(n, odf, dtype):
    plan = od.host_plan(n=n, odf=odf, dtype=dtype)
    assert plan["nchares"] == odf
    _check_plan(n, plan)


@pytest.mark.parametrize("tile", [(16, 8, 3), (32, 8, 5), (16, 16, 16), (64, 4, 7)])
def test_regular_halo_maps_small_tiles(tile):
    n = (37, 21, 19)
    plan = od.host_plan(n=n, odf=8, tile=tile)
    _check_plan(n, plan)


def test_octree_halo_maps_brute_force():
    blocks = workloads.octree_blocks(n=64, root=32, min_edge=8, p_refine=0.5, seed=3)
    sizes = {e[0] for _, e in blocks}
    assert len(sizes) >= 3          # genuinely uneven
    plan = od.host_plan(n=64, blocks=blocks, tile=(16, 8, 8))
    _check_plan((64, 64, 64), plan)


def test_explicit_uneven_slabs():
    # non-cubic, non-aligned slabs of different thickness
    blocks = [((0, 0, 0), (10, 12, 3)), ((0, 0, 3), (10, 5, 7)), ((0, 5, 3), (10, 7, 7))]
    plan = od.host_plan(n=(10, 12, 10), blocks=blocks, tile=(16, 8, 4))
    _check_plan((10, 12, 10), plan)


def test_regular_split_sizes_first_blocks_take_remainder():
    plan = od.host_plan(n=(37, 16, 16), block=(19, 16, 16))
    ext = sorted({c[1][0] for c in plan["chares"]})
    assert ext == [18, 19]
    first = min(plan["chares"], key=lambda c: c[0][0])
    assert first[1][0] == 19


def test_non_cubic_odf_factorisation():
    plan = od.host_plan(n=64, odf=32)
    ks = [len({c[0][d] for c in plan["chares"]}) for d in range(3)]
    assert sorted(ks) == [2, 4, 4] and ks[2] == 4 and ks[0] == 2


def test_algorithmic_bytes_match_closed_form():
    # G = 6 (k-1) N^2 ghost cells read from other chares for a k^3 split
    for n, k in ((64, 2), (512, 16), (96, 4)):
        plan = od.host_plan(n=n, odf=k ** 3)
        assert plan["halo_cells"] == 6 * (k - 1) * n * n
        assert plan["bytes_per_iter"] == 8 * (2 * n ** 3 + 6 * (k - 1) * n * n)


def test_paper_message_size_rule():
    # Section IV: overdecomposing a 2D stencil by 4 halves each message; in
    # 3D a k^3 split shrinks each face message by k^2.
    g = json.load(open(os.path.join(GOLDEN, "paper_message_size.json")))
    for case in g["cases"]:
        n, k = case["n"], case["k"]
        base = od.host_plan(n=(n, n, 1), odf=1)
        split = od.host_plan(n=(n, n, 1), block=(n // k, n // k, 1))
        assert split["nchares"] == case["odf"]
        b_face = base["chares"][0][1][0]
        s_face = split["chares"][0][1][0]
        assert s_face / b_face == case["message_ratio"]
        # 3D: a k^3 split shrinks face messages by k^2
        b3 = od.host_plan(n=n, odf=1)["chares"][0][1]
        s3 = od.host_plan(n=n, odf=k ** 3)["chares"][0][1]
        assert (s3[0] * s3[1]) / (b3[0] * b3[1]) == 1.0 / k ** 2


def test_octree_statistics_match_branching_process():
    blocks = workloads.octree_blocks()
    assert sum(e[0] ** 3 for _, e in blocks) == 768 ** 3
    exp = workloads.expected_octree_leaves()
    counts = {}
    for _, e in blocks:
        counts[e[0]] = counts.get(e[0], 0) + 1
    assert set(counts) <= {16, 32, 64, 128}
    for e, m in exp.items():
        # generous bound for a branching-process count (std grows ~ sqrt(m)
        # times the ancestry's fan-out of 8 per level)
        assert abs(counts.get(e, 0) - m) < 8 * 5 * np.sqrt(m)


@pytest.mark.parametrize("odf,split", [(8, True), (64, True), (512, False)])
def test_msgdriven_groups_under_imbalance(odf, split):
    # message-driven launch position q runs in XCD group q % 8.  Without
    # imbalance the groups are 8 compact boxes of the grid; with imbalance and
    # fewer than 512 chares every chare is cut into 8 boxes, one per group, so
    # a heavy chare's extra sweeps are shared by every XCD.  The tile set and
    # its halo maps do not change.
    n = (128, 128, 128)
    base = dict(n=n, odf=odf, dtype="f64", exec="msgdriven", tile=(16, 8, 16))
    a = od.host_plan(**base)
    b = od.host_plan(**base, imbalance_pct=10, imbalance_max_extra=4)
    key = lambda t: (t["chare"], t["origin"], t["extent"])
    assert sorted(map(key, a["tiles"])) == sorted(map(key, b["tiles"]))
    _check_plan(n, b)
    for plan, spread in ((a, False), (b, split)):
        per_group = [{t["chare"] for q, t in enumerate(plan["tiles"]) if q % 8 == g} for g in range(8)]
        if spread:
            assert all(len(s) == odf for s in per_group)
        else:
            assert all(len(s) <= max(1, odf // 8) + 1 for s in per_group)


def _llround(x):
    return int(np.floor(x + 0.5))


@pytest.mark.parametrize("n,odf", [(64, 8), (96, 27), (256, 4096), (1024, 32768)])
def test_imbalance_draw_exact_count_every_step(n, odf):
    # 10 % of the chares, drawn afresh at every step, each re-running its
    # sweep 1..4 extra times
    steps = range(0, 160)
    D = od.imbalance_draw(steps, n=n, odf=odf, exec="persistent", imbalance_pct=10, imbalance_max_extra=4)
    C = D.shape[1]
    assert C == odf
    m = _llround(0.1 * C)
    assert ((D > 0).sum(axis=1) == m).all()
    assert D.min() >= 0 and D.max() <= 4
    if m * 160 >= 200:
        assert set(np.unique(D[D > 0])) == {1, 2, 3, 4}
    heavy = D > 0
    if C >= 64:
        # not a table with a short period: the set changes step to step and
        # does not repeat 64 steps later
        for t in range(0, 96):
            assert not np.array_equal(heavy[t], heavy[t + 1])
            assert not np.array_equal(heavy[t], heavy[t + 64])


def test_imbalance_order_is_a_permutation():
    # for every count h, exactly h chares are drawn: the per-step order is a
    # bijection of the chare ids (27 chares: pct 0..100 reaches every h)
    for pct in range(0, 101):
        D = od.imbalance_draw(range(0, 12), n=96, odf=27, exec="persistent", imbalance_pct=pct,
                              imbalance_max_extra=3)
        assert ((D > 0).sum(axis=1) == _llround(pct / 100 * 27)).all()


def test_imbalance_draw_frequency_and_seed():
    # each chare is drawn with frequency ~ p over many steps; another seed
    # gives another draw; no imbalance gives zeros
    D = od.imbalance_draw(range(0, 4000), n=64, odf=64, exec="persistent", imbalance_pct=10,
                          imbalance_max_extra=4)
    f = (D > 0).mean(axis=0)
    assert abs(f.mean() - 6 / 64) < 1e-12
    assert f.min() > 0.05 and f.max() < 0.14
    E = od.imbalance_draw(range(0, 50), n=64, odf=64, exec="persistent", imbalance_pct=10,
                          imbalance_max_extra=4, seed=7)
    assert not np.array_equal(D[:50], E)
    Z = od.imbalance_draw(range(0, 5), n=64, odf=64, exec="persistent")
    assert not Z.any()


def _reach2_brute(n, chares):
    """Cells of other chares within two stencil steps (L1 distance <= 2) of
    each chare, inside the domain, counted cell by cell."""
    nx, ny, nz = n
    total = 0
    for (o, e) in chares:
        lo = [max(o[d] - 2, 0) for d in range(3)]
        hi = [min(o[d] + e[d] + 2, n[d]) for d in range(3)]
        for z in range(lo[2], hi[2]):
            for y in range(lo[1], hi[1]):
                for x in range(lo[0], hi[0]):
                    dist = 0
                    for d, v in enumerate((x, y, z)):
                        dist += max(o[d] - v, 0, v - (o[d] + e[d] - 1))
                    if 0 < dist <= 2:
                        total += 1
    return total


@pytest.mark.parametrize("n,odf", [((13, 11, 9), 8), ((12, 6, 5), 27), ((9, 9, 9), 1), ((10, 10, 10), 27),
                                   ((33, 4, 5), 8), ((64, 64, 64), 8)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_two_step_pass_bytes_brute_force(n, odf, dtype):
    plan = od.host_plan(n=n, odf=odf, dtype=dtype, exec="fused")
    s = 8 if dtype == "f64" else 4
    assert plan["steps_per_pass"] == 2
    g2 = _reach2_brute(n, plan["chares"])
    assert plan["bytes_per_pass"] == s * (2 * plan["interior"] + g2)
    assert plan["bytes_per_iter"] == s * (2 * plan["interior"] + plan["halo_cells"])


@pytest.mark.parametrize("kw", [{"exec": "persistent", "hints": 2048}, {"exec": "persistent", "hints": 8},
                                {"exec": "msgdriven", "hints": 4096}, {"exec": "msgdriven", "stencil": 5,
                                                                       "n": (64, 1, 64)},
                                {"exec": "per_chare"},
                                {"exec": "fused", "hints": 4096},
                                {"exec": "fused", "stencil": 5, "n": (64, 1, 64), "imbalance_pct": 10,
                                 "imbalance_max_extra": 2},
                                {"exec": "fused", "tile": (128, 4, 8)}])
def test_two_step_only_where_supported(kw):
    # other forms, the one-step hint, the 2D stencil under imbalance and
    # tile shapes without a two-step variant keep one step per pass
    kw = dict(kw)
    plan = od.host_plan(n=kw.pop("n", (64, 64, 64)), odf=8, dtype="f64", **kw)
    assert plan["steps_per_pass"] == 1
    assert plan["bytes_per_pass"] == plan["bytes_per_iter"]


@pytest.mark.parametrize("exec_,hints", [("fused", 0), ("graph", 0), ("persistent", 0), ("persistent", 16),
                                         ("persistent", 32), ("persistent", 8192), ("msgdriven", 0),
                                         ("msgdriven", 4 | 64), ("msgdriven", 128 | 1024)])
def test_two_step_default_forms(exec_, hints):
    plan = od.host_plan(n=(64, 64, 64), odf=8, dtype="f64", exec=exec_, hints=hints)
    assert plan["steps_per_pass"] == 2


@pytest.mark.parametrize("exec_,hints", [("fused", 0), ("persistent", 0), ("persistent", 8192),
                                         ("persistent", 16), ("msgdriven", 0)])
def test_two_step_under_imbalance(exec_, hints):
    # a heavy chare's extra runs are one-step sweeps before its pass, so the
    # 3D stencil pairs steps under load imbalance too; the bytes of a pass
    # count the pair alone (the extra runs are the imbalance's cost)
    kw = dict(n=(64, 64, 64), odf=8, dtype="f64", exec=exec_, hints=hints)
    a = od.host_plan(**kw)
    b = od.host_plan(**kw, imbalance_pct=10, imbalance_max_extra=4)
    assert b["steps_per_pass"] == 2 and b["bytes_per_pass"] == a["bytes_per_pass"]


def _two_step_boxes(o, e, n):
    """Boxes of cells a pair of steps reads beyond a tile's face slabs
    (tile origin o, extent e): slabs two out, (x, y) corner columns, the
    one-out ring's rows below and above; a box outside the domain along one
    axis is projected onto the boundary layer, along two it is dropped."""
    lo = list(o)
    hi = [o[d] + e[d] for d in range(3)]
    out = []
    for f in range(6):
        d = f // 2
        a, b = list(lo), list(hi)
        a[d] = hi[d] + 1 if f % 2 else lo[d] - 2
        b[d] = a[d] + 1
        out.append((a, b))
    xs, ys, zs = (lo[0] - 1, hi[0]), (lo[1] - 1, hi[1]), (lo[2] - 1, hi[2])
    for k in range(4):
        for fix in ({0: xs[k & 1], 1: ys[k >> 1]}, {0: xs[k & 1], 2: zs[k >> 1]}, {1: ys[k & 1], 2: zs[k >> 1]}):
            a, b = list(lo), list(hi)
            for d, v in fix.items():
                a[d], b[d] = v, v + 1
            out.append((a, b))
    res = []
    for a, b in out:
        outs = [d for d in range(3) if b[d] <= 0 or a[d] >= n[d]]
        if len(outs) >= 2:
            continue
        for d in outs:
            a[d] = 0 if a[d] < 0 else n[d] - 1
            b[d] = a[d] + 1
        res.append((a, b))
    return res


@pytest.mark.parametrize("tile", [(16, 16, 8), (32, 16, 16), (32, 32, 32)])
def test_two_step_octree_tiles_read_single_blocks(tile):
    # explicit blocks: the planner cuts tiles until every box of cells a
    # pair of steps reads beyond the face slabs lies in one block
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.5, seed=7)
    plan = od.host_plan(n=96, blocks=blocks, dtype="f64", exec="fused", tile=tile)
    assert plan["steps_per_pass"] == 2
    n = (96, 96, 96)
    own = _owner_map(n, plan["chares"])
    _check_plan(n, plan)
    for t in plan["tiles"]:
        co, _ = plan["chares"][t["chare"]]
        o = [co[d] + t["origin"][d] for d in range(3)]
        for a, b in _two_step_boxes(o, t["extent"], n):
            ids = np.unique(own[a[2]:b[2], a[1]:b[1], a[0]:b[0]])
            assert len(ids) == 1, (t, a, b, ids)


def _deps_brute(plan, n, reach):
    """Every other tile owning a cell within L1 distance `reach` of a tile's
    box (cells inside the domain), from a cell -> tile owner map."""
    owner = np.full(n[::-1], -1, dtype=np.int64)   # [z, y, x]
    boxes = []
    for i, t in enumerate(plan["tiles"]):
        co = plan["chares"][t["chare"]][0]
        lo = [co[d] + t["origin"][d] for d in range(3)]
        hi = [lo[d] + t["extent"][d] for d in range(3)]
        owner[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = i
        boxes.append((lo, hi))
    assert (owner >= 0).all()
    out = []
    for i, (lo, hi) in enumerate(boxes):
        a = [max(0, lo[d] - reach) for d in range(3)]
        b = [min(n[d], hi[d] + reach) for d in range(3)]
        z, y, x = np.meshgrid(np.arange(a[2], b[2]), np.arange(a[1], b[1]), np.arange(a[0], b[0]), indexing="ij")
        dist = np.zeros(z.shape, dtype=np.int64)
        for d, v in enumerate((x, y, z)):
            dist += np.maximum(0, lo[d] - v) + np.maximum(0, v - (hi[d] - 1))
        sub = owner[a[2]:b[2], a[1]:b[1], a[0]:b[0]]
        got = set(int(v) for v in np.unique(sub[(dist >= 1) & (dist <= reach)]))
        got.discard(i)
        out.append(tuple(sorted(got)))
    return out


@pytest.mark.parametrize("n,odf,tile,hints,spp", [((64, 64, 64), 8, (16, 16, 8), 0, 2),
                                                  ((70, 50, 45), 27, (32, 8, 8), 0, 2),
                                                  ((40, 33, 29), 8, (16, 16, 4), 0, 2),
                                                  ((70, 50, 45), 27, (32, 8, 8), 4096, 1)])
def test_msgdriven_deps_reach_brute_force(n, odf, tile, hints, spp):
    # the message-driven dependency lists are exactly the tiles a task reads
    # (one cell out for single steps, two cells in L1 distance for two-step
    # tasks), checked against a brute-force owner map
    plan = od.host_plan(n=n, odf=odf, dtype="f64", exec="msgdriven", tile=tile, hints=hints)
    assert plan["steps_per_pass"] == spp
    assert plan["deps"] == _deps_brute(plan, n, spp)


@pytest.mark.parametrize("tile", [(16, 16, 8), (32, 16, 16)])
def test_msgdriven_deps_reach_brute_force_octree(tile):
    # explicit blocks at one resolution: the tiles are also cut so every
    # line a pair reads lies in one block; the dependency lists still equal
    # the tiles within two cells (L1) of each tile
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.45, seed=11)
    plan = od.host_plan(n=(96, 96, 96), blocks=blocks, dtype="f64", exec="msgdriven", tile=tile)
    assert plan["steps_per_pass"] == 2
    assert plan["deps"] == _deps_brute(plan, (96, 96, 96), 2)
