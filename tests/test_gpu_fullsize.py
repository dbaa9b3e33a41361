"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times.

Outputs the oracle cannot compute for the whole grid are checked one by one
(each sampled point's value after t sweeps depends only on cells within
Chebyshev distance t, so the oracle evaluates it on a small sub-box), and
properties that hold at any size are checked on the whole field: identical
bits across execution modes and decompositions at the full iteration
count, and a discrete-harmonic linear field that must stay fixed.
"""
import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od
import workloads

pytestmark = pytest.mark.gpu


def _sample_points(n, count, seed):
    rng = np.random.default_rng(seed)
    pts = [tuple(int(rng.integers(0, m)) for m in n) for _ in range(count)]
    nx, ny, nz = n
    # corners, faces and chare-boundary neighbourhoods
    pts += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny // 2, nz // 2), (nx - 1, 0, nz - 1),
            (31, 31, 31), (32, 32, 32), (31, 32, 33), (nx // 2, ny // 2, 0)]
    return pts


def _lin(pts, n):
    nx, ny, _ = n
    return np.array([(k * ny + j) * nx + i for (i, j, k) in pts], dtype=np.int64)


def _tuned(n, odf, dtype, exec_="graph", hints=1, **kw):
    g = od.Grid(n, odf=odf, dtype=dtype, exec="fused", hints=hints, **kw)
    tile = g.autotune(2)
    g.close()
    return od.Grid(n, odf=odf, dtype=dtype, exec=exec_, tile=tile, hints=hints, **kw)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_512_odf4096_sampled_against_oracle(dtype):
    n = (512, 512, 512)
    iters = 10
    g = _tuned(n, 4096, dtype)
    try:
        g.iterate(iters)
        pts = _sample_points(n, 48, 1)
        got = g.read_points(_lin(pts, n))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64 if dtype == "f64" else np.float32)
    assert np.array_equal(got, want)


def test_512_odf4096_one_full_step_sampled_against_oracle():
    # the benchmark's step as timed: 200 iterations, graph form, autotuned
    # tile; a few points the oracle evaluates on their domain of dependence
    # (up to 401^3 cells each)
    n = (512, 512, 512)
    iters = 200
    pts = [(0, 0, 0), (511, 511, 511), (31, 32, 480), (256, 255, 256), (5, 300, 40)]
    g = _tuned(n, 4096, "f64")
    try:
        g.iterate(iters)
        got = g.read_points(_lin(pts, n))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("tile", [(32, 32, 16), (32, 16, 32)])
def test_512_fp32_persistent_full_grid_sampled(tile):
    # a cooperative grid as large as the device holds (the static-stride
    # persistent kernel at its capped occupancy): every workgroup must be
    # resident for the device-wide barrier to complete
    n = (512, 512, 512)
    iters = 10
    g = od.Grid(n, odf=4096, dtype="f32", exec="persistent", tile=tile, hints=1)
    try:
        assert g.plan()["grid_wgs"] >= 1024
        g.iterate(iters)
        pts = _sample_points(n, 24, 3)
        got = g.read_points(_lin(pts, n))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float32)
    assert np.array_equal(got, want)


def test_512_odf4096_full_iterations_identical_across_modes():
    # 200 iterations: graph (bench launch configuration) = persistent =
    # message-driven = fused with another tile = ODF 8
    n = 512
    g = _tuned(n, 4096, "f64", "graph")
    try:
        g.iterate(200)
        ref = g.read()
        r_ref = g.residual()
    finally:
        g.close()
    assert np.isfinite(ref).all()
    for kw in (dict(odf=4096, exec="persistent"), dict(odf=4096, exec="msgdriven"),
               dict(odf=4096, exec="fused", tile=(32, 8, 16)), dict(odf=8, exec="graph", tile=(64, 8, 32))):
        g = od.Grid(n, dtype="f64", hints=1, **kw)
        try:
            g.iterate(200)
            U = g.read()
            r = g.residual()
        finally:
            g.close()
        assert r == r_ref, kw
        assert np.array_equal(U, ref), kw


def test_512_linear_field_fixed_full_size():
    n = (512, 512, 512)
    k, j, i = np.meshgrid(np.arange(-1, 513), np.arange(-1, 513), np.arange(-1, 513), indexing="ij",
                          sparse=True)
    L = (7.0 + i + 2.0 * j - 3.0 * k).astype(np.float64)
    g = _tuned(n, 4096, "f64")
    try:
        g.write(np.broadcast_to(L, (514, 514, 514)))
        g.iterate(200)
        assert g.residual() == 0.0
        U = g.read()
    finally:
        g.close()
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.array_equal(U[inner], np.broadcast_to(L, (514, 514, 514))[inner])


@pytest.mark.parametrize("exec_", ["msgdriven", "persistent"])
def test_1024_odf32768_imbalance_sampled(exec_):
    n = (1024, 1024, 1024)
    iters = 12
    g = od.Grid(n, odf=32768, dtype="f64", exec=exec_, tile=(32, 16, 32), hints=1, imbalance_pct=10,
                imbalance_max_extra=4)
    try:
        g.iterate(iters)
        pts = _sample_points(n, 32, 2)
        got = g.read_points(_lin(pts, n))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("odf", [8, 64])
def test_1024_few_chares_imbalance_msgdriven_sampled(odf):
    # the benchmark's message-driven configuration under imbalance with few
    # chares: every chare spread over all XCD groups, tiles of depth 32
    n = (1024, 1024, 1024)
    iters = 12
    g = od.Grid(n, odf=odf, dtype="f64", exec="msgdriven", tile=(64, 16, 32), hints=1, imbalance_pct=10,
                imbalance_max_extra=4)
    try:
        g.iterate(iters)
        pts = _sample_points(n, 32, 4)
        pts += [(511, 511, 511), (512, 512, 512), (255, 767, 256)]
        got = g.read_points(_lin(pts, n))
    finally:
        g.close()
    want = oracle.point_values(n, pts, iters, np.float64)
    assert np.array_equal(got, want)


def test_768_octree_sampled_graph_persistent_msgdriven():
    blocks = workloads.octree_blocks(n=768, root=128, min_edge=16, p_refine=0.4, seed=12734)
    n = (768, 768, 768)
    iters = 12
    pts = _sample_points(n, 32, 3)
    want = oracle.point_values(n, pts, iters, np.float64)
    for exec_ in ("graph", "persistent", "msgdriven"):
        g = od.Grid(768, blocks=blocks, dtype="f64", exec="fused", hints=1)
        tile = g.autotune(2)
        g.close()
        g = od.Grid(768, blocks=blocks, dtype="f64", exec=exec_, tile=tile, hints=1)
        try:
            g.iterate(iters)
            got = g.read_points(_lin(pts, n))
        finally:
            g.close()
        assert np.array_equal(got, want), exec_


def test_served_384_request_matches_oracle():
    from paper_2605_12734_amd.serving import Server
    q = dict(n=384, dtype="f64", odf=64, tol=1e-6, max_iters=30, check_every=10, seed=77)
    want, it, r = oracle.solve(384, np.float64, seed=77, iters=30, tol=1e-6, check_every=10)
    with Server(arena_bytes=3 << 30, max_slots=4) as srv:
        t = srv.submit(**q)
        res = srv.wait(t, timeout=300)
        field = srv.fetch(t)
    assert res["iters"] == it and res["residual"] == r
    assert np.array_equal(field, want)


def test_served_384_request_survives_yields():
    # small requests arriving while a 384^3 solve runs end its scheduling
    # epochs early (queued tasks dropped, counters rebuilt at the next
    # launch); every result must still be the oracle's, bit for bit
    import time
    from paper_2605_12734_amd.serving import Server
    big = dict(n=384, dtype="f64", odf=64, tol=1e-6, max_iters=60, check_every=10, seed=78)
    small = [dict(n=20 + 3 * i, dtype=("f32", "f64")[i % 2], odf=(1, 8)[i % 2], tol=1e-4, max_iters=120,
                  check_every=(5, 0, 1)[i % 3], seed=90 + i) for i in range(6)]
    with Server(arena_bytes=3 << 30, max_slots=8) as srv:
        tb = srv.submit(**big)
        ts = []
        for q in small:
            time.sleep(0.004)
            ts.append(srv.submit(**q))
        res = srv.wait(tb, timeout=300)
        field = srv.fetch(tb)
        smalls = [(srv.wait(t, timeout=300), srv.fetch(t)) for t in ts]
        epochs = srv.stats()["epochs"]
    want, it, r = oracle.solve(384, np.float64, seed=78, iters=60, tol=1e-6, check_every=10)
    assert res["iters"] == it and res["residual"] == r
    assert np.array_equal(field, want)
    for q, (rs, f) in zip(small, smalls):
        dt = np.float32 if q["dtype"] == "f32" else np.float64
        w, i2, r2 = oracle.solve(q["n"], dt, seed=q["seed"], iters=q["max_iters"], tol=q["tol"],
                                 check_every=q["check_every"])
        assert rs["iters"] == i2 and rs["residual"] == r2, q
        assert np.array_equal(f, w), q
    assert epochs >= 2


def test_served_two_384_requests_cursor_mode_with_yields():
    # two 384^3 fp64 solves put 6912 tiles in a launch (at least 4 per
    # workgroup: the serving scheduler claims ready tiles from per-XCD
    # cursors); small requests arriving meanwhile end epochs early
    import time
    from paper_2605_12734_amd.serving import Server
    big = [dict(n=384, dtype="f64", odf=64, tol=1e-6, max_iters=40, check_every=10, seed=83 + i) for i in range(2)]
    small = [dict(n=24 + 5 * i, dtype=("f64", "f32")[i % 2], odf=(8, 1)[i % 2], tol=1e-4, max_iters=90,
                  check_every=(0, 3)[i % 2], seed=95 + i) for i in range(4)]
    with Server(arena_bytes=6 << 30, max_slots=8) as srv:
        tb = [srv.submit(**q) for q in big]
        ts = []
        for q in small:
            time.sleep(0.004)
            ts.append(srv.submit(**q))
        got = [(srv.wait(t, timeout=300), srv.fetch(t)) for t in tb + ts]
    for q, (res, field) in zip(big + small, got):
        dt = np.float32 if q["dtype"] == "f32" else np.float64
        w, it, r = oracle.solve(q["n"], dt, seed=q["seed"], iters=q["max_iters"], tol=q["tol"],
                                check_every=q["check_every"])
        assert res["iters"] == it and res["residual"] == r, q
        assert np.array_equal(field, w), q


@pytest.mark.parametrize("exec_", ["persistent", "msgdriven"])
def test_device_wait_bound_reports_timeout(exec_):
    # a 1 ns bound on every device-side wait: the launch's barriers and
    # queues give up (every workgroup leaves normally) and the host sees
    # OD_ETIMEDOUT instead of a result; od_write makes the grid usable
    g = od.Grid(256, odf=512, dtype="f64", exec=exec_, tile=(32, 16, 32), hints=1, wait_s=1e-9)
    try:
        g.iterate(50)
        with pytest.raises(od.ODError) as ei:
            g.residual()
        assert ei.value.status == -110
        with pytest.raises(od.ODError) as ei:
            g.read_points([0, 1, 2])
        assert ei.value.status == -110
    finally:
        g.close()
    # nothing is left behind on the device: a grid with the default bound
    # right after it is exact
    n = (64, 64, 64)
    want, _, r_w = oracle.solve(n, np.float64, seed=3, iters=9)
    g = od.Grid(n, odf=8, dtype="f64", exec=exec_, seed=3)
    try:
        g.iterate(9)
        assert g.residual() == r_w
        assert np.array_equal(g.read(), want)
    finally:
        g.close()


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 5, 1), (2, 1, 3), (3, 3, 1)])
@pytest.mark.parametrize("exec_", ["fused", "persistent", "msgdriven", "per_chare", "graph"])
def test_degenerate_tiny_grids(n, exec_):
    want, _, r_w = oracle.solve(n, np.float64, seed=5, iters=7)
    g = od.Grid(n, odf=1, dtype="f64", exec=exec_, seed=5)
    try:
        g.iterate(7)
        r = g.residual()
        U = g.read()
    finally:
        g.close()
    assert np.array_equal(U, want) and r == r_w
