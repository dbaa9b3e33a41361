"""od_create_static: the grid whose descriptors and device state live in the
library's static per-GPU array (for callers that cannot allocate device
memory).  Through the C ABI, its results must equal od_create's bit for bit,
on two grids made one after the other on the same GPU, the second smaller;
the first is then superseded and refused."""
import ctypes

import numpy as np
import pytest

import paper_2605_12734_amd as od
from paper_2605_12734_amd import _binding as B
from paper_2605_12734_amd._binding import check

pytestmark = pytest.mark.gpu

ITERS = 23


def _field_bytes(kw):
    p = od._PlanHandle(**kw)
    try:
        return od.plan_info(p.h)["field_bytes"]
    finally:
        p.close()


def _make_static(kw):
    import torch

    cfg, keep = od.make_config(**kw)
    nbytes = _field_bytes(kw)
    fields = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    check(B.lib().od_create_static(ctypes.byref(cfg), ctypes.c_void_p(st.cuda_stream),
                                   ctypes.c_void_p(fields.data_ptr()), nbytes, ctypes.byref(h)), "od_create_static")
    return h, fields, keep


def _results(h, kw, iters):
    L = B.lib()
    check(L.od_iterate(h, iters), "od_iterate")
    r = ctypes.c_double()
    check(L.od_residual(h, ctypes.byref(r)), "od_residual")
    nx, ny, nz = od._dims(kw["n"])
    dt = np.float64 if kw.get("dtype", "f64") == "f64" else np.float32
    U = np.empty((nz + 2, ny + 2, nx + 2), dtype=dt)
    check(L.od_read(h, U.ctypes.data_as(ctypes.c_void_p), U.nbytes), "od_read")
    return U, r.value


def _reference(kw, iters):
    g = od.Grid(**kw)
    try:
        g.iterate(iters)
        return g.read(), g.residual()
    finally:
        g.close()


PAIRS = [
    (dict(n=96, odf=27, dtype="f64", exec="persistent"), dict(n=40, odf=8, dtype="f64", exec="persistent")),
    (dict(n=(70, 50, 33), odf=12, dtype="f32", exec="fused"), dict(n=(21, 17, 9), odf=8, dtype="f32", exec="fused")),
    (dict(n=64, odf=64, dtype="f64", exec="msgdriven"), dict(n=24, odf=8, dtype="f64", exec="msgdriven")),
    (dict(n=48, odf=8, dtype="f64", exec="persistent", imbalance_pct=25, imbalance_max_extra=2),
     dict(n=16, odf=1, dtype="f32", exec="fused")),
]


@pytest.mark.parametrize("first,second", PAIRS)
def test_static_grid_matches_od_create(first, second):
    L = B.lib()
    h1, f1, k1 = _make_static(first)
    try:
        U1, r1 = _results(h1, first, ITERS)
        W1, q1 = _reference(first, ITERS)
        assert r1 == q1 and np.array_equal(U1, W1), first
        # the second, smaller grid reuses the same array
        h2, f2, k2 = _make_static(second)
        try:
            U2, r2 = _results(h2, second, ITERS + 4)
            W2, q2 = _reference(second, ITERS + 4)
            assert r2 == q2 and np.array_equal(U2, W2), second
            # the first grid is superseded: refused, not run on stale state
            assert L.od_iterate(h1, 1) == B.OD_EINVAL
            assert b"superseded" in L.od_last_error()
        finally:
            check(L.od_destroy(h2), "od_destroy")
    finally:
        check(L.od_destroy(h1), "od_destroy")
