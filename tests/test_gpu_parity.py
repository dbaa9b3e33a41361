"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, bit-exact (0 ULP) in fp64 and fp32.

Sizes span several tiles with ragged tails; every execution mode and a
range of overdecomposition factors must give the oracle's bits.
"""
import os

import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od
import workloads

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}
MODES = ["fused", "graph", "persistent", "msgdriven", "per_chare"]


def _oracle(n, dtype, iters, seed=12734, bc=od.DEFAULT_BC):
    return oracle.solve(n, DT[dtype], seed=seed, iters=iters, bc=bc)


def _run(n, iters, **kw):
    g = od.Grid(n, **kw)
    try:
        g.iterate(iters)
        r = g.residual()
        U = g.read()
        return U, r, g.iterations()
    finally:
        g.close()


def _assert_same(U, want):
    if not np.array_equal(U, want):
        d = np.argwhere(U != want)
        k, j, i = d[0]
        raise AssertionError(f"{len(d)} cells differ; first at padded (k,j,i)=({k},{j},{i}): "
                             f"{U[k, j, i]!r} vs {want[k, j, i]!r}")


def test_device_present():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    props = torch.cuda.get_device_properties(0)
    assert "gfx950" in getattr(props, "gcnArchName", "gfx950")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,odf", [(64, 8), ((37, 21, 19), 8), ((5, 70, 3), 1), ((1, 1, 1), 1)])
def test_init_matches_oracle(dtype, n, odf):
    bc = (1.0, 0.5, 0.25, 0.125, 2.0, 3.0)
    g = od.Grid(n, odf=odf, dtype=dtype, bc=bc, seed=99, exec="fused")
    try:
        U = g.read()
    finally:
        g.close()
    _assert_same(U, oracle.init_field(n, DT[dtype], 99, bc))


@pytest.mark.parametrize("exec_", MODES)
def test_config0_64cubed_fp64_2x2x2_100_iterations(exec_):
    # 64^3 FP64, 2x2x2 chares of 32^3, bc 1 on x-, 100 iterations, 0 ULP
    want, it_w, r_w = _oracle(64, "f64", 100)
    U, r, it = _run(64, 100, odf=8, dtype="f64", exec=exec_)
    _assert_same(U, want)
    assert it == it_w == 100 and r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("odf", [1, 8, 64, 512])
@pytest.mark.parametrize("exec_", ["graph", "persistent", "msgdriven"])
def test_odf_sweep_bit_identical(dtype, odf, exec_):
    want, _, r_w = _oracle(64, dtype, 12)
    U, r, _ = _run(64, 12, odf=odf, dtype=dtype, exec=exec_)
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("odf", [8, 64])
def test_per_chare_baseline_bit_identical(dtype, odf):
    want, _, r_w = _oracle(48, dtype, 7)
    U, r, _ = _run(48, 7, odf=odf, dtype=dtype, exec="per_chare")
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("tile", [None, (16, 8, 5), (64, 4, 7), (32, 16, 64)])
@pytest.mark.parametrize("exec_", ["fused", "msgdriven"])
def test_ragged_tiles_and_uneven_chares(dtype, tile, exec_):
    n = (75, 41, 29)    # uneven chares (first blocks take the remainder), ragged tiles
    if dtype == "f32" and tile is not None and tile[0] == 16:
        tile = (16, 16, 5)
    bc = (1.0, 0.0, 0.5, 0.0, 0.25, 0.0)
    want, _, r_w = _oracle(n, dtype, 9, seed=5, bc=bc)
    U, r, _ = _run(n, 9, odf=27, dtype=dtype, exec=exec_, tile=tile, seed=5, bc=bc)
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_octree_uneven_blocks(dtype):
    blocks = workloads.octree_blocks(n=96, root=32, min_edge=8, p_refine=0.5, seed=7)
    assert len({e[0] for _, e in blocks}) >= 3
    want, _, r_w = _oracle(96, dtype, 10)
    for exec_ in ("graph", "persistent", "msgdriven"):
        U, r, _ = _run(96, 10, blocks=blocks, dtype=dtype, exec=exec_, tile=(16, 16, 8) if dtype == "f64" else (16, 16, 8))
        _assert_same(U, want)
        assert r == r_w


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_linear_field_fixed_point_through_write(dtype):
    n = (40, 33, 24)
    k, j, i = np.meshgrid(np.arange(-1, n[2] + 1), np.arange(-1, n[1] + 1), np.arange(-1, n[0] + 1),
                          indexing="ij")
    L = (3.0 + i - 2.0 * j + 5.0 * k).astype(DT[dtype])
    g = od.Grid(n, odf=8, dtype=dtype, exec="graph")
    try:
        g.write(L)
        assert g.iterations() == 0
        g.iterate(6)
        assert g.residual() == 0.0
        U = g.read()
    finally:
        g.close()
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    _assert_same(U[inner], L[inner])
    assert np.array_equal(U[1:-1, 1:-1, 0], L[1:-1, 1:-1, 0])


def test_index_field_one_sweep_exact():
    # every cell = its global linear index: one sweep's sums expose any wrong
    # ghost source (halo exchange) as a wrong value
    n = (34, 20, 18)
    k, j, i = np.meshgrid(np.arange(n[2] + 2), np.arange(n[1] + 2), np.arange(n[0] + 2), indexing="ij")
    F = ((k * (n[1] + 2) + j) * (n[0] + 2) + i).astype(np.float64)
    want, _ = oracle.sweep(F)
    for exec_, odf in (("fused", 27), ("per_chare", 8), ("msgdriven", 64), ("persistent", 12)):
        g = od.Grid(n, odf=odf, dtype="f64", exec=exec_)
        try:
            g.write(F)
            g.iterate(1)
            U = g.read()
        finally:
            g.close()
        inner = (slice(1, -1), slice(1, -1), slice(1, -1))
        _assert_same(U[inner], want[inner])


def test_read_points_and_iterations():
    n = (30, 20, 10)
    want, _, _ = _oracle(n, "f64", 4)
    g = od.Grid(n, odf=8, dtype="f64", exec="fused")
    try:
        g.iterate(3)
        g.iterate(1)
        assert g.iterations() == 4
        rng = np.random.default_rng(0)
        idx = rng.integers(0, n[0] * n[1] * n[2], size=200)
        vals = g.read_points(idx)
    finally:
        g.close()
    kk, rem = np.divmod(idx, n[0] * n[1])
    jj, ii = np.divmod(rem, n[0])
    assert np.array_equal(vals, want[kk + 1, jj + 1, ii + 1])


def test_zero_iterations_and_errors():
    g = od.Grid(16, odf=8, dtype="f64", exec="graph")
    try:
        g.iterate(0)
        assert g.residual() == 0.0
        with pytest.raises(od.ODError):
            g.iterate(-1)
        with pytest.raises(od.ODError):
            g.read_points([16 ** 3])
    finally:
        g.close()


@pytest.mark.parametrize("exec_", ["graph", "persistent", "msgdriven", "fused"])
def test_split_calls_equal_one_call(exec_):
    # iterating 5 + 8 + 1 equals 14 at once, and the oracle
    want, _, r_w = _oracle(40, "f32", 14)
    g = od.Grid(40, odf=64, dtype="f32", exec=exec_)
    try:
        for k in (5, 8, 1):
            g.iterate(k)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("exec_", ["persistent", "msgdriven", "fused"])
def test_imbalance_does_not_change_results(exec_):
    want, _, r_w = _oracle(48, "f64", 11)
    U, r, _ = _run(48, 11, odf=64, dtype="f64", exec=exec_, imbalance_pct=10, imbalance_max_extra=4)
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("exec_,dtype", [("graph", "f64"), ("persistent", "f32"), ("fused", "f64")])
def test_autotune_keeps_bits(exec_, dtype):
    # tuning picks a tile shape by timing; it must not change a bit, and it
    # must not disturb the field or the residual already computed
    want5, _, r5 = _oracle(64, dtype, 5)
    want, _, r_w = _oracle(64, dtype, 15)
    g = od.Grid(64, odf=64, dtype=dtype, exec=exec_)
    try:
        g.iterate(5)
        assert g.residual() == r5
        tile = g.autotune(iters=1)
        assert g.plan()["tile"] == tuple(tile)
        assert g.residual() == r5
        _assert_same(g.read(), want5)
        g.iterate(10)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("hints", [1])
@pytest.mark.parametrize("exec_", ["graph", "msgdriven", "persistent"])
def test_hints_keep_bits(hints, exec_):
    # bit 0: non-temporal output stores
    want, _, r_w = _oracle((70, 36, 40), "f64", 9, seed=3)
    U, r, _ = _run((70, 36, 40), 9, odf=64, dtype="f64", exec=exec_, hints=hints, seed=3)
    _assert_same(U, want)
    assert r == r_w


@pytest.mark.parametrize("dtype,n,odf,tile,iters", [
    ("f64", 256, 512, (32, 16, 8), 9),              # 4096 tiles over 1536 workgroups
    ("f32", 256, 512, (32, 32, 8), 9),              # 2048 tiles
    ("f64", (200, 136, 72), 64, (32, 16, 4), 12),   # ragged tile depths (4, 4, 4, 4, 2)
    ("f32", (200, 136, 144), 64, (32, 32, 5), 12),  # ragged tile depths (5 x 7, 1)
])
@pytest.mark.parametrize("sched", [0, 16, 32, 2048])
def test_persistent_schedules(dtype, n, odf, tile, iters, sched):
    # fixed stride (0), tiles from per-XCD counters (16), counters with each
    # XCD group's last tiles cut into z-ranges (32), fixed contiguous runs
    # (2048): bits must not change
    want, _, r_want = _oracle(n, dtype, iters)
    g = od.Grid(n, odf=odf, dtype=dtype, exec="persistent", tile=tile, hints=1 | sched)
    try:
        plan = g.plan()
        assert plan["grid_wgs"] % 8 == 0
        if sched == 32:
            assert plan["ntiles"] % 8 == 0
        g.iterate(iters)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    assert r == r_want
    _assert_same(U, want)


def test_library_loaded_before_torch():
    # libod loaded first (a host-only plan), PyTorch afterwards: one HIP
    # runtime must serve both (a second runtime would find no device)
    import subprocess
    import sys
    code = ("import paper_2605_12734_amd as od\n"
            "info = od.host_plan(n=16, odf=1)\n"
            "g = od.Grid(16, odf=1, exec='fused')\n"
            "g.iterate(3)\n"
            "print(g.residual() > 0)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0 and r.stdout.strip().endswith("True"), r.stderr[-2000:]


def test_persistent_timeline():
    # hints bit 3 records, per iteration, when workgroups start it and
    # finish their tiles; the barrier orders them and bits do not change
    want, _, r_want = _oracle(64, "f64", 20)
    g = od.Grid(64, odf=64, dtype="f64", exec="persistent", hints=1 | 8, tile=(16, 8, 8))
    try:
        g.iterate(20)
        r = g.residual()
        U = g.read()
        tl = g.timeline()
    finally:
        g.close()
    assert r == r_want
    _assert_same(U, want)
    assert tl.shape == (20, 4) and tl[0, 0] == 0.0
    assert (tl[:, 0] <= tl[:, 1]).all() and (tl[:, 2] <= tl[:, 3]).all() and (tl[:, 0] <= tl[:, 2]).all()
    # nobody starts iteration i + 1 before the last workgroup finished i
    assert (tl[1:, 0] >= tl[:-1, 3]).all()
