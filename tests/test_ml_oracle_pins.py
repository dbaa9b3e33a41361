"""Pins of the multi-resolution block oracle (oracle/ml_oracle.c) against
facts that do not come from the oracle itself: the uniform oracle when every
block has unit cells, hand-computed ghost values and updates, a constant
field, linearity, mirror symmetry, and an independent pure-Python brute
force on small layouts."""
import numpy as np
import pytest

import oracle
from oracle import brute
import workloads

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _two_level():
    # coarse half (cell 2) next to four fine 4^3 blocks (cell 1): ratio-2 faces along x
    blocks = [((0, 0, 0), (4, 8, 8)), ((4, 0, 0), (4, 4, 4)), ((4, 4, 0), (4, 4, 4)), ((4, 0, 4), (4, 4, 4)),
              ((4, 4, 4), (4, 4, 4))]
    return (8, 8, 8), blocks, [2, 1, 1, 1, 1]


def _three_level():
    # cells 4, 2 and 1 side by side: ratio-2 and ratio-4 faces along x, y and z
    blocks = [((0, 0, 0), (8, 8, 8)),            # cell 4
              ((8, 0, 0), (4, 4, 4)), ((12, 0, 0), (4, 4, 4)), ((8, 4, 0), (4, 4, 4)), ((12, 4, 0), (4, 4, 4)),
              ((8, 0, 4), (4, 4, 4)), ((12, 0, 4), (4, 4, 4)), ((8, 4, 4), (4, 4, 4)),
              ((12, 4, 4), (4, 4, 4)),            # cell 1 (the rest of x in [8,16) cell 2)
              ((0, 8, 0), (16, 8, 8)),            # cell 2 on top in y
              ((0, 0, 8), (16, 16, 8))]           # cell 4 above in z
    cell = [4, 2, 2, 2, 1, 2, 2, 2, 2, 2, 4]
    return (16, 16, 16), blocks, cell


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_unit_cells_equal_the_uniform_oracle(dtype):
    n = (24, 16, 16)
    blocks = [((0, 0, 0), (8, 16, 16)), ((8, 0, 0), (16, 8, 16)), ((8, 8, 0), (16, 8, 8)), ((8, 8, 8), (16, 8, 8))]
    g = oracle.MLGrid(n, blocks, [1] * 4, dtype, seed=11)
    r = g.jacobi(9)
    U, _, rw = oracle.solve(n, dtype, seed=11, iters=9)
    assert r == rw
    for b, (o, e) in enumerate(blocks):
        want = U[1 + o[2]:1 + o[2] + e[2], 1 + o[1]:1 + o[1] + e[1], 1 + o[0]:1 + o[0] + e[0]]
        assert np.array_equal(g.interior(b), want)


def test_hand_computed_x_interface():
    # coarse block A = one cell of edge 2 at x in [0,2); fine block B (cell 1) at x in [2,4)
    n = (4, 2, 2)
    blocks = [((0, 0, 0), (2, 2, 2)), ((2, 0, 0), (2, 2, 2))]
    g = oracle.MLGrid(n, blocks, [2, 1], np.float64, bc=(1, 0, 0, 0, 0, 0))
    g.block(0)[1, 1, 1] = 0.5
    k, j, i = np.meshgrid(np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    g.block(1)[1:-1, 1:-1, 1:-1] = 1 + i + 2 * j + 4 * k
    g.jacobi(1)
    # A: x- ghost = bc 1, x+ ghost = mean of B's x=0 layer (1, 3, 5, 7) = 4
    assert g.interior(0)[0, 0, 0] == np.float64(5.0) / 6.0
    B = g.interior(1)
    # B(0,0,0): x- ghost = A's value injected (0.5); neighbours 2, 3, 5; y-, z- ghosts 0
    assert B[0, 0, 0] == 1.75
    # B(1,1,1): x- 7, y- 6, z- 4, the rest Dirichlet 0
    assert B[1, 1, 1] == np.float64(17.0) / 6.0


def test_hand_computed_z_interface():
    # coarse block A (cell 2) below a fine block B (cell 1) along z
    n = (2, 2, 4)
    blocks = [((0, 0, 0), (2, 2, 2)), ((0, 0, 2), (2, 2, 2))]
    g = oracle.MLGrid(n, blocks, [2, 1], np.float64, bc=(1, 0, 0, 0, 0, 0))
    g.block(0)[1, 1, 1] = 0.25
    k, j, i = np.meshgrid(np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    g.block(1)[1:-1, 1:-1, 1:-1] = 1 + i + 2 * j + 4 * k
    g.jacobi(1)
    # A's z+ ghost = mean of B's k=0 layer (1, 2, 3, 4) = 2.5; x- ghost = 1
    assert g.interior(0)[0, 0, 0] == np.float64(3.5) / 6.0
    B = g.interior(1)
    # B(0,0,0): x- bc 1, x+ 2, y- 0, y+ 3, z- = A injected 0.25, z+ 5
    assert B[0, 0, 0] == np.float64(11.25) / 6.0


@pytest.mark.parametrize("layout", [_two_level, _three_level])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_brute_force_identity(layout, dtype):
    n, blocks, cell = layout()
    g = oracle.MLGrid(n, blocks, cell, dtype, seed=5)
    r = g.jacobi(3)
    A = brute.ml_init(n, blocks, cell, dtype, 5)
    A, rb = brute.ml_jacobi(n, blocks, cell, A, 3, oracle.DEFAULT_BC)
    assert r == rb
    for b in range(len(blocks)):
        assert np.array_equal(g.interior(b), np.array(A[b], dtype=dtype)[1:-1, 1:-1, 1:-1]), b


@pytest.mark.parametrize("layout", [_two_level, _three_level])
def test_constant_field_stays_fixed(layout):
    n, blocks, cell = layout()
    c = 0.75
    g = oracle.MLGrid(n, blocks, cell, np.float64, bc=(c,) * 6)
    for b in range(len(blocks)):
        g.block(b)[...] = c
    r = g.jacobi(20)
    assert r == 0.0
    for b in range(len(blocks)):
        assert np.all(g.interior(b) == c)


def test_linearity():
    n, blocks, cell = _three_level()
    bc1, bc2 = (1.0, 0, 0.5, 0, 0, 0.25), (0, 2.0, 0, 0, 1.0, 0)
    g1 = oracle.MLGrid(n, blocks, cell, np.float64, seed=1, bc=bc1)
    g2 = oracle.MLGrid(n, blocks, cell, np.float64, seed=2, bc=bc2)
    g3 = oracle.MLGrid(n, blocks, cell, np.float64, seed=1, bc=tuple(a + b for a, b in zip(bc1, bc2)))
    g3.U[:] = g1.U + g2.U
    for g in (g1, g2, g3):
        g.jacobi(15)
    for b in range(len(blocks)):
        assert np.allclose(g3.interior(b), g1.interior(b) + g2.interior(b), rtol=0, atol=1e-13)


def test_mirror_symmetry_in_y():
    # layout closed under y -> ny - y, values and boundaries symmetric: the
    # result stays symmetric (up to the reversed order of face sums)
    n = (16, 16, 8)
    blocks = [((0, 0, 0), (8, 8, 8)), ((0, 8, 0), (8, 8, 8)),
              ((8, 0, 0), (8, 4, 4)), ((8, 0, 4), (8, 4, 4)), ((8, 4, 0), (8, 8, 8)), ((8, 12, 0), (8, 4, 4)),
              ((8, 12, 4), (8, 4, 4))]
    cell = [2, 2, 1, 1, 2, 1, 1]
    g = oracle.MLGrid(n, blocks, cell, np.float64, bc=(1.0, 0.25, 0.5, 0.5, 0, 0))
    for b, ((o, e), h) in enumerate(zip(blocks, cell)):
        A = g.block(b)
        mz, my, mx = A.shape[0] - 2, A.shape[1] - 2, A.shape[2] - 2
        zc = o[2] + (np.arange(mz) + 0.5) * h
        yc = o[1] + (np.arange(my) + 0.5) * h
        xc = o[0] + (np.arange(mx) + 0.5) * h
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        A[1:-1, 1:-1, 1:-1] = np.sin(0.3 * X) + np.cos(0.1 * (Y - n[1] / 2) ** 2) + 0.01 * Z
    g.jacobi(12)
    mirror = {}
    for b, (o, e) in enumerate(blocks):
        mo = (o[0], n[1] - o[1] - e[1], o[2])
        mirror[b] = next(c for c, (o2, e2) in enumerate(blocks) if tuple(o2) == mo and tuple(e2) == tuple(e))
    for b in range(len(blocks)):
        assert np.allclose(g.interior(b), g.interior(mirror[b])[:, ::-1, :], rtol=0, atol=1e-14)


def test_octree_layout_is_accepted_and_fine_leaves_match_unit_resolution():
    # the octree of uneven blocks with 16 cells per leaf edge: finest leaves
    # (edge 16) have unit cells; the layout satisfies the alignment rule
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.4, seed=3)
    cell = [e[0] // 8 for _, e in blocks]
    g = oracle.MLGrid(96, blocks, cell, np.float64, seed=3)
    g.jacobi(2)
    assert np.isfinite(g.U).all()
    assert sum(int(np.prod(g.m[b])) for b in range(len(blocks))) == 8 ** 3 * len(blocks)


def test_misaligned_layout_rejected():
    # a fine block whose tangential extent is not a multiple of the coarse cell
    n = (8, 4, 4)
    blocks = [((0, 0, 0), (4, 4, 4)), ((4, 0, 0), (4, 1, 4)), ((4, 1, 0), (4, 3, 4))]
    g = oracle.MLGrid(n, blocks, [2, 1, 1], np.float64)
    with pytest.raises(ValueError):
        g.jacobi(1)
