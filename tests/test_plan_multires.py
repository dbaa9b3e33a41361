"""Host-side plans of multi-resolution blocks (no GPU): every tile face that
borders a block of another cell size reads the chare's resolution-change
ghost buffer, every other face reads a same-size chare (checked cell by cell
in grid units) or a Dirichlet face; tiles partition each chare's cells;
layouts the definition does not cover are refused."""
import numpy as np
import pytest

import paper_2605_12734_amd as od
import workloads


def _layouts():
    two = ((64, 64, 64), [((0, 0, 0), (32, 64, 64)), ((32, 0, 0), (32, 32, 32)), ((32, 32, 0), (32, 32, 32)),
                          ((32, 0, 32), (32, 32, 32)), ((32, 32, 32), (32, 32, 32))], [2, 1, 1, 1, 1])
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.4, seed=3)
    octo = ((96, 96, 96), blocks, [e[0] // 8 for _, e in blocks])
    return [two, octo]


def _unit_owner(n, blocks):
    own = -np.ones(n[::-1], dtype=np.int64)
    for b, (o, e) in enumerate(blocks):
        own[o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]] = b
    assert np.all(own >= 0)
    return own


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_multires_faces_brute_force(k, dtype):
    n, blocks, cell = _layouts()[k]
    p = od.host_plan(n=n, blocks=blocks, cell=cell, dtype=dtype, exec="fused")
    own = _unit_owner(n, blocks)
    assert p["interior"] == sum(int(np.prod(e)) // h ** 3 for (_, e), h in zip(blocks, cell))
    covered = {b: np.zeros(tuple(e[d] // cell[b] for d in (2, 1, 0)), dtype=np.int64)
               for b, (_, e) in enumerate(blocks)}
    for t in p["tiles"]:
        c = t["chare"]
        (u, _), h = blocks[c], cell[c]
        assert tuple(p["chares"][c][0]) == tuple(u)
        o, e = t["origin"], t["extent"]
        covered[c][o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]] += 1
        m = [blocks[c][1][d] // h for d in range(3)]
        for f in range(6):
            d = f // 2
            lo_cell = o[d] - 1 if f % 2 == 0 else o[d] + e[d]
            if 0 <= lo_cell < m[d]:
                assert t["src_kind"][f] == 0 and t["src"][f] == c
                continue
            # unit slab across the face, tangential extent of the tile
            lo = [u[q] + o[q] * h for q in range(3)]
            hi = [lo[q] + e[q] * h for q in range(3)]
            lo[d] = u[d] - 1 if f % 2 == 0 else u[d] + m[d] * h
            hi[d] = lo[d] + 1
            if lo[d] < 0 or lo[d] >= n[d]:
                assert t["src_kind"][f] == 1 and t["src"][f] == f
                continue
            # the chare's whole face decides whether it is a resolution change
            flo = [u[q] for q in range(3)]
            fhi = [u[q] + m[q] * h for q in range(3)]
            flo[d], fhi[d] = lo[d], hi[d]
            face_owners = np.unique(own[flo[2]:fhi[2], flo[1]:fhi[1], flo[0]:fhi[0]])
            change = any(cell[int(b)] != h for b in face_owners)
            if change:
                assert t["src_kind"][f] == 2 and t["src"][f] == f, (t, f)
            else:
                owners = np.unique(own[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
                assert len(owners) == 1 and t["src_kind"][f] == 0 and t["src"][f] == int(owners[0])
                s = int(owners[0])
                # src_origin: the slab start in cells of the (equal) size
                assert tuple(t["src_origin"][f]) == tuple(v // h for v in lo)
    for b in covered:
        assert np.all(covered[b] == 1)


def test_unit_cells_plan_unchanged():
    # cell sizes all 1 give the same plan as no cell sizes
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.4, seed=4)
    a = od.host_plan(n=96, blocks=blocks, dtype="f64", exec="fused")
    b = od.host_plan(n=96, blocks=blocks, cell=[1] * len(blocks), dtype="f64", exec="fused")
    assert a["tiles"] == b["tiles"] and a["bytes_per_iter"] == b["bytes_per_iter"]


@pytest.mark.parametrize("blocks,cell,exec_", [
    ([((0, 0, 0), (16, 16, 16)), ((16, 0, 0), (16, 4, 16)), ((16, 4, 0), (16, 12, 16))], [8, 2, 2], "fused"),
    ([((0, 0, 0), (16, 16, 16)), ((16, 0, 0), (16, 16, 16))], [3, 1], "fused"),          # not a power of two
    ([((0, 0, 0), (16, 16, 16)), ((16, 0, 0), (16, 16, 16))], [2, 1], "msgdriven"),
    ([((0, 0, 0), (16, 16, 16)), ((16, 0, 0), (16, 16, 16))], [2, 1], "per_chare"),
    ([((0, 0, 0), (12, 16, 16)), ((12, 0, 0), (20, 16, 16))], [8, 1], "fused"),          # origin not a multiple
    ([((0, 0, 0), (32, 32, 32)), ((32, 0, 0), (32, 32, 32))], [32, 1], "fused"),          # cell ratio 32 > 16
])
def test_uncovered_layouts_refused(blocks, cell, exec_):
    n = tuple(max(o[d] + e[d] for o, e in blocks) for d in range(3))
    with pytest.raises(od.ODError):
        od.host_plan(n=n, blocks=blocks, cell=cell, dtype="f64", exec=exec_)


def test_cell_ratio_16_accepted():
    # the largest ratio the ghost fill stages (16 x 16 finer cells per ghost cell)
    blocks = [((0, 0, 0), (32, 32, 32)), ((32, 0, 0), (32, 32, 32))]
    p = od.host_plan(n=(64, 32, 32), blocks=blocks, cell=[16, 1], dtype="f64", exec="fused")
    assert p["interior"] == 8 + 32 ** 3


@pytest.mark.parametrize("kw,ok", [({}, True), ({"hints": 16}, True), ({"hints": 8}, False), ({"hints": 32}, False),
                                   ({"hints": 2048}, False), ({"hints": 8192}, False),
                                   ({"imbalance_pct": 10, "imbalance_max_extra": 2}, False)])
def test_multires_persistent_forms(kw, ok):
    # the persistent form of a multi-resolution grid fills and sweeps in one
    # launch, taking tiles from counters: schedules that fix the tile order,
    # the timeline and imbalance are refused; one step per pass
    n, blocks, cell = _layouts()[0]
    if ok:
        p = od.host_plan(n=n, blocks=blocks, cell=cell, dtype="f64", exec="persistent", **kw)
        assert p["steps_per_pass"] == 1
    else:
        with pytest.raises(od.ODError):
            od.host_plan(n=n, blocks=blocks, cell=cell, dtype="f64", exec="persistent", **kw)
