"""Multi-resolution blocks on the GPU (resolution-change ghost fill +
fused sweep), compared element by element with the multi-resolution oracle
(oracle/ml_oracle.c): small two- and three-level layouts, an octree, and
the 768^3 octree with 16 cells per leaf edge at full size; fp64 and fp32,
fused and graph-captured launches."""
import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od
import workloads

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}


def _two_level():
    blocks = [((0, 0, 0), (32, 64, 64)), ((32, 0, 0), (32, 32, 32)), ((32, 32, 0), (32, 32, 32)),
              ((32, 0, 32), (32, 32, 32)), ((32, 32, 32), (32, 32, 32))]
    return (64, 64, 64), blocks, [2, 1, 1, 1, 1]


def _three_level():
    # cells 4, 2 and 1 meet along x, y and z (ratio-2 and ratio-4 faces)
    s = 8
    base = [((0, 0, 0), (8, 8, 8)),
            ((8, 0, 0), (4, 4, 4)), ((12, 0, 0), (4, 4, 4)), ((8, 4, 0), (4, 4, 4)), ((12, 4, 0), (4, 4, 4)),
            ((8, 0, 4), (4, 4, 4)), ((12, 0, 4), (4, 4, 4)), ((8, 4, 4), (4, 4, 4)), ((12, 4, 4), (4, 4, 4)),
            ((0, 8, 0), (16, 8, 8)), ((0, 0, 8), (16, 16, 8))]
    blocks = [(tuple(v * s for v in o), tuple(v * s for v in e)) for o, e in base]
    return (128, 128, 128), blocks, [4, 2, 2, 2, 1, 2, 2, 2, 2, 2, 4]


def _octree(n=96, root=32, min_edge=8, seed=3):
    blocks = workloads.octree_blocks(n=n, root=root, min_edge=min_edge, p_refine=0.4, seed=seed)
    return (n, n, n), blocks, [e[0] // min_edge for _, e in blocks]


def _compare(n, blocks, cell, dtype, exec_, iters, tile=None, bc=oracle.DEFAULT_BC, seed=12734):
    want = oracle.MLGrid(n, blocks, cell, DT[dtype], seed=seed, bc=bc)
    r_want = want.jacobi(iters)
    g = od.Grid(n, blocks=blocks, cell=cell, dtype=dtype, exec=exec_, tile=tile, seed=seed, bc=bc, hints=1)
    try:
        g.iterate(iters)
        r = g.residual()
        for b in range(len(blocks)):
            got = g.read_block(b)
            assert np.array_equal(got, want.interior(b)), (b, blocks[b], cell[b])
    finally:
        g.close()
    assert r == r_want


def _ratio_16():
    # a 2^3-cell block beside 32^3 unit cells and a 4^3-cell block: ratio-16
    # and ratio-4 faces (one ghost cell averages 256 finer cells)
    blocks = [((0, 0, 0), (32, 32, 32)), ((32, 0, 0), (32, 32, 32)), ((0, 32, 0), (64, 32, 32))]
    return (64, 64, 32), blocks, [16, 1, 4]


def _ratio_8_octree():
    # octree leaves of edge 8..64 units, 8 cells per leaf edge: ratios up to 8
    blocks = workloads.octree_blocks(n=128, root=64, min_edge=8, p_refine=0.45, seed=5)
    return (128, 128, 128), blocks, [e[0] // 8 for _, e in blocks]


@pytest.mark.parametrize("layout", [_two_level, _three_level, _octree, _ratio_16, _ratio_8_octree])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("exec_", ["fused", "graph", "persistent"])
def test_multires_matches_oracle(layout, dtype, exec_):
    n, blocks, cell = layout()
    _compare(n, blocks, cell, dtype, exec_, 7)


@pytest.mark.parametrize("tile", [(16, 8, 8), (32, 4, 16), (64, 8, 32)])
@pytest.mark.parametrize("exec_", ["fused", "persistent"])
def test_multires_tile_shapes(tile, exec_):
    n, blocks, cell = _three_level()
    _compare(n, blocks, cell, "f64", exec_, 5, tile=tile)


def test_multires_persistent_resume_and_autotune():
    # one cooperative launch per call (fill, barrier, sweep, barrier per
    # iteration): calls of 1, 4 and 6 iterations on an autotuned grid
    n, blocks, cell = _octree(n=128, root=64, min_edge=16, seed=7)
    want = oracle.MLGrid(n, blocks, cell, np.float64, seed=12734)
    r_want = want.jacobi(11)
    g = od.Grid(n, blocks=blocks, cell=cell, dtype="f64", exec="persistent", hints=1)
    try:
        g.autotune(2)
        for k in (1, 4, 6):
            g.iterate(k)
        r = g.residual()
        assert g.iterations() == 11
        for b in range(len(blocks)):
            assert np.array_equal(g.read_block(b), want.interior(b)), b
    finally:
        g.close()
    assert r == r_want


def test_multires_bc_and_constant_field():
    n, blocks, cell = _two_level()
    c = 0.75
    g = od.Grid(n, blocks=blocks, cell=cell, dtype="f64", exec="fused", bc=(c,) * 6)
    try:
        for b in range(len(blocks)):
            g.write_block(b, np.full(g.block_cells(b)[::-1], c))
        g.iterate(25)
        assert g.residual() == 0.0
        for b in range(len(blocks)):
            assert np.all(g.read_block(b) == c)
    finally:
        g.close()


def test_multires_autotuned_graph_long_run():
    n, blocks, cell = _octree(n=128, root=64, min_edge=16, seed=7)
    g = od.Grid(n, blocks=blocks, cell=cell, dtype="f64", exec="fused", hints=1)
    tile = g.autotune(2)
    g.close()
    _compare(n, blocks, cell, "f64", "graph", 60, tile=tile)


def test_multires_768_octree_full_size():
    # the 768^3 octree (root 128, leaves down to 16, refine probability 0.4)
    # with 16 cells per leaf edge: finest leaves have unit cells
    n, blocks, cell = _octree(n=768, root=128, min_edge=16, seed=12734)
    oracle.set_threads(oracle.max_threads())
    g = od.Grid(n, blocks=blocks, cell=cell, dtype="f64", exec="fused", hints=1)
    tile = g.autotune(2)
    g.close()
    _compare(n, blocks, cell, "f64", "graph", 20, tile=tile)
    _compare(n, blocks, cell, "f64", "persistent", 20, tile=tile)


def test_global_io_refused_for_multires():
    n, blocks, cell = _two_level()
    g = od.Grid(n, blocks=blocks, cell=cell, dtype="f64", exec="fused")
    try:
        with pytest.raises(od.ODError):
            g.read()
        with pytest.raises(od.ODError):
            g.read_points(np.array([0], dtype=np.int64))
    finally:
        g.close()


def test_block_io_roundtrip_uniform_grid():
    g = od.Grid(48, odf=8, dtype="f32", exec="fused")
    try:
        A = g.read_block(3)
        U = g.read()
        # chare 3 of the 2x2x2 split: origin (24, 24, 0)
        assert np.array_equal(A, U[1:25, 25:49, 25:49])
        B = np.arange(A.size, dtype=np.float32).reshape(A.shape)
        g.write_block(3, B)
        assert np.array_equal(g.read_block(3), B)
    finally:
        g.close()
