"""Jacobi2D (the paper's own workload, Section V): 5-point stencil, bit-exact
against the 2D oracle in every execution mode, and sampled at the paper's
per-GPU size (32768^2 fp64, 100 iterations)."""
import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("odf", [1, 4, 16])
@pytest.mark.parametrize("exec_", ["graph", "persistent", "msgdriven", "per_chare"])
def test_jacobi2d_bit_identical(dtype, odf, exec_):
    n2 = (300, 170)
    bc = (1.0, 0.0, 0.5, 0.25)
    want, _, r_w = oracle.solve2d(n2, DT[dtype], seed=8, iters=20, bc=bc)
    g = od.Grid2D(n2, odf=odf, dtype=dtype, exec=exec_, seed=8, bc=bc)
    try:
        g.iterate(20)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    assert np.array_equal(U, want)
    assert r == r_w


def test_jacobi2d_paper_size_sampled():
    # one GPU's share in the paper's weak scaling: 32768 x 32768, 100 iterations
    n2 = (32768, 32768)
    iters = 100
    g = od.Grid2D(n2, odf=16, dtype="f64", exec="graph", hints=1)
    try:
        g.iterate(iters)
        rng = np.random.default_rng(5)
        pts = [(int(rng.integers(0, 32768)), int(rng.integers(0, 32768))) for _ in range(12)]
        pts += [(0, 0), (32767, 32767), (8191, 8192), (16384, 0)]
        got = g.read_points([j * 32768 + i for (i, j) in pts])
    finally:
        g.close()
    want = oracle.point_values2d(n2, pts, iters, np.float64)
    assert np.array_equal(got, want)


VARIANTS2D = {"f64": [128, 256, 512], "f32": [256, 512, 1024]}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [1, 2, 7, 20])
@pytest.mark.parametrize("exec_", ["fused", "graph"])
def test_jacobi2d_pairs_bit_identical(dtype, iters, exec_):
    # two steps per pass on the (x, z) rows: every compiled row width,
    # ragged tiles, odd counts ending with a single sweep, four boundary values
    n2 = (300, 170)
    bc = (1.0, 0.5, 0.25, 2.0)
    want, _, r_w = oracle.solve2d(n2, DT[dtype], seed=4, iters=iters, bc=bc)
    for tx in VARIANTS2D[dtype]:
        for odf, tz in ((1, 64), (4, 16), (16, 7)):
            g = od.Grid2D(n2, odf=odf, dtype=dtype, exec=exec_, seed=4, bc=bc, tile=(tx, 1, tz), hints=1)
            try:
                assert g.plan()["steps_per_pass"] == 2
                g.iterate(iters)
                r = g.residual()
                U = g.read()
            finally:
                g.close()
            assert np.array_equal(U, want), (tx, odf, tz)
            assert r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n2,odf", [((1, 1), 1), ((2, 3), 1), ((5, 4), 4), ((9, 40), 16), ((130, 3), 4)])
def test_jacobi2d_pairs_tiny(dtype, n2, odf):
    bc = (1.0, 0.5, 0.25, 2.0)
    want, _, r_w = oracle.solve2d(n2, DT[dtype], seed=6, iters=5, bc=bc)
    g = od.Grid2D(n2, odf=odf, dtype=dtype, exec="graph", seed=6, bc=bc,
                  tile=(128 if dtype == "f64" else 256, 1, 8))
    try:
        assert g.plan()["steps_per_pass"] == 2
        g.iterate(5)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    assert np.array_equal(U, want)
    assert r == r_w
