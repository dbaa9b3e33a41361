"""Autotuned tiles and schedules keep the bits: the tuner times candidates
on the grid itself (persistent: one sweep per launch into the spare parity;
message-driven: real steps with the state saved and restored), so a tuned
grid must continue exactly where it was and give the oracle's result."""
import numpy as np
import pytest

import oracle
import paper_2605_12734_amd as od

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}


def _check(n, dtype, g, iters_before, iters_after):
    want, _, r_want = oracle.solve(n, DT[dtype], seed=12734, iters=iters_before + iters_after)
    g.iterate(iters_after)
    assert g.iterations() == iters_before + iters_after
    assert g.residual() == r_want
    U = g.read()
    assert np.array_equal(U, want), int((U != want).sum())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,odf", [(256, 512), ((150, 90, 70), 27)])
def test_persistent_autotune_keeps_bits(dtype, n, odf):
    g = od.Grid(n, odf=odf, dtype=dtype, exec="persistent", hints=1)
    try:
        g.iterate(3)
        g.autotune(1)
        plan = g.plan()
        assert plan["schedule"] in (1, 2, 3, 4) and plan["grid_wgs"] > 0
        _check(n, dtype, g, 3, 9)
    finally:
        g.close()


@pytest.mark.parametrize("dtype,n,odf", [("f64", 128, 64), ("f32", (96, 80, 64), 512)])
def test_msgdriven_autotune_restores_state(dtype, n, odf):
    g = od.Grid(n, odf=odf, dtype=dtype, exec="msgdriven", hints=1)
    try:
        g.iterate(5)
        g.autotune(1)
        plan = g.plan()
        assert plan["schedule"] & 3 in (1, 2) and (plan["schedule"] >> 2) & 3 in (1, 2)
        _check(n, dtype, g, 5, 7)
    finally:
        g.close()


@pytest.mark.parametrize("claim", [64, 128])
@pytest.mark.parametrize("pub", [512, 1024])
def test_msgdriven_forced_schedules(claim, pub):
    n = 128
    g = od.Grid(n, odf=512, dtype="f64", exec="msgdriven", hints=1 | claim | pub, tile=(16, 8, 8))
    try:
        plan = g.plan()
        assert plan["schedule"] == (1 if claim == 64 else 2) | ((1 if pub == 512 else 2) << 2)
        _check(n, "f64", g, 0, 11)
    finally:
        g.close()
