"""The C-ABI library loads and exports every symbol include/*.h declares;
host-side argument checks (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**\s*(od_[A-Za-z0-9_]+)\s*\(",
                             src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("od_create", "od_iterate", "od_residual", "od_submit", "od_poll", "od_read", "od_write",
                 "od_workspace_bytes", "od_destroy", "od_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2605_12734_amd import _binding
    L = _binding.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the Python binding covers the whole surface
    assert set(_declared_functions()) <= set(_binding.SIGNATURES)


def test_config_default_and_version():
    from paper_2605_12734_amd import _binding as B
    cfg = B.od_config()
    B.lib().od_config_default(ctypes.byref(cfg))
    assert tuple(cfg.n) == (64, 64, 64) and cfg.odf == 8 and cfg.dtype == B.OD_F64
    assert tuple(cfg.bc) == (1.0, 0, 0, 0, 0, 0) and cfg.seed == 12734
    assert cfg.wait_s == 0.0 and not cfg.block_cell
    assert b"gfx950" in B.lib().od_version()


@pytest.mark.parametrize("kw,code", [
    (dict(n=(0, 4, 4)), -22),
    (dict(n=8, odf=0), -22),
    (dict(n=4, odf=125), -22),            # 5 chares along a 4-cell dimension
    (dict(n=8, dtype="f64", tile=(24, 8, 8)), -22),   # not a compiled tile variant
    (dict(n=8, exec="per_chare", blocks=[((0, 0, 0), (8, 8, 8))]), -22),
    (dict(n=8, blocks=[((0, 0, 0), (8, 8, 4))]), -22),             # does not cover
    (dict(n=8, blocks=[((0, 0, 0), (8, 8, 8)), ((0, 0, 0), (8, 8, 8))]), -22),   # overlap / over-cover
    (dict(n=8, imbalance_pct=150), -22),
    (dict(n=8, wait_s=-1.0), -22),
    (dict(n=8, wait_s=float("nan")), -22),
])
def test_invalid_configs_rejected(kw, code):
    import paper_2605_12734_amd as od
    with pytest.raises(od.ODError) as ei:
        od.workspace_bytes(**kw)
    assert ei.value.status == code


def test_workspace_grows_with_grid_and_is_aligned():
    import paper_2605_12734_amd as od
    a = od.workspace_bytes(n=32, odf=8)
    b = od.workspace_bytes(n=64, odf=8)
    assert b > 7 * a // 2
    # two fp64 parities of 64^3 at least
    assert b >= 2 * 8 * 64 ** 3 and b % 256 == 0


def test_device_calls_refuse_host_only_handle():
    import paper_2605_12734_amd as od
    from paper_2605_12734_amd import _binding as B
    p = od._PlanHandle(n=16, odf=8)
    try:
        assert B.lib().od_iterate(p.h, 1) == B.OD_EINVAL
        r = ctypes.c_double()
        assert B.lib().od_residual(p.h, ctypes.byref(r)) == B.OD_EINVAL
    finally:
        p.close()


def test_launch_overlap_host_checks():
    # argument checks run before any device call
    from paper_2605_12734_amd import _binding as B
    L = B.lib()
    assert L.od_launch_overlap_bytes(0) == 0
    assert L.od_launch_overlap_bytes(10) == 256 + 40
    res = B.od_overlap_result()
    assert L.od_launch_overlap(None, 0, 10, 1, 1, 1, ctypes.byref(res)) == -22
    assert L.od_launch_overlap(ctypes.c_void_p(256), 1 << 20, 10, 11, 1, 1, ctypes.byref(res)) == -22


def test_request_arrival_stamp():
    # the arrival stamp is part of the request record and is checked on the
    # host (od_request_bytes validates without a server or a GPU)
    from paper_2605_12734_amd import _binding as B
    from paper_2605_12734_amd.serving import make_request
    names = [f for f, _ in B.od_request._fields_]
    assert names[-1] == "t_arrival" and B.od_request.t_arrival.offset == 96
    assert [f for f, _ in B.od_info._fields_][-1] == "t_arrival"
    L = B.lib()
    out = ctypes.c_size_t()
    r = make_request(16, "f64", odf=8, t_arrival=-1.0)
    assert L.od_request_bytes(ctypes.byref(r), ctypes.byref(out)) == -22
    r = make_request(16, "f64", odf=8, t_arrival=float("nan"))
    assert L.od_request_bytes(ctypes.byref(r), ctypes.byref(out)) == -22
    r = make_request(16, "f64", odf=8, t_arrival=12.5)
    assert L.od_request_bytes(ctypes.byref(r), ctypes.byref(out)) == 0 and out.value > 0


def test_create_static_host_checks():
    # refused before any device work: a form that allocates when it first
    # iterates, and control state beyond the static array's 16 MiB
    from paper_2605_12734_amd import _binding as B
    import paper_2605_12734_amd as od
    L = B.lib()
    h = ctypes.c_void_p()
    cfg, keep = od.make_config(n=32, odf=8, exec="graph")
    assert L.od_create_static(ctypes.byref(cfg), None, ctypes.c_void_p(256), 1 << 30, ctypes.byref(h)) == -22
    cfg, keep = od.make_config(n=32, odf=8, exec="per_chare")
    assert L.od_create_static(ctypes.byref(cfg), None, ctypes.c_void_p(256), 1 << 30, ctypes.byref(h)) == -22
    p = od._PlanHandle(n=64, odf=8, exec="fused")
    info = od.plan_info(p.h)
    p.close()
    assert info["field_bytes"] > 0 and info["control_bytes"] > 0
    assert info["field_bytes"] + info["control_bytes"] == od.workspace_bytes(n=64, odf=8, exec="fused")
    big, keep2 = od.make_config(n=1024, odf=64 ** 3, exec="fused")   # 262144 chares: 32 MiB of tiles
    assert L.od_create_static(ctypes.byref(big), None, ctypes.c_void_p(256), 1 << 40, ctypes.byref(h)) == -12
    assert b"static array holds" in L.od_last_error()
    assert not h.value


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,odf", [(384, 1), (384, 8), (384, 64), (300, 27)])
def test_largest_serving_requests_fit_a_slot(dtype, n, odf):
    # the serving kernel runs tasks of one step: a request's dependency
    # lists reach one cell, so the largest request sizes fit a slot's
    # tile and dependency tables (checked on the host, no GPU)
    from paper_2605_12734_amd.serving import request_bytes

    assert request_bytes(n=n, dtype=dtype, odf=odf, tol=1e-6, max_iters=2000) > 0
