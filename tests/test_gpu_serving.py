"""Serving: independent solves admitted under a memory budget and run
together by the message-driven scheduler.  Every result (field, iteration
count, residual) must equal the oracle's solve with the same stopping rule,
bit for bit, whether the solve ran alone or in the mix."""
import time

import numpy as np
import pytest

import oracle
from paper_2605_12734_amd import ODError
from paper_2605_12734_amd.serving import Server, control_bytes, request_bytes

pytestmark = pytest.mark.gpu

DT = {"f64": np.float64, "f32": np.float32}

MIX = [
    dict(n=16, dtype="f64", odf=8, tol=1e-5, max_iters=400, check_every=10, seed=11),
    dict(n=23, dtype="f32", odf=1, tol=1e-3, max_iters=300, check_every=7, seed=12),
    dict(n=40, dtype="f64", odf=64, tol=1e-6, max_iters=60, check_every=10, seed=13),   # hits the cap
    dict(n=12, dtype="f32", odf=8, tol=1e-4, max_iters=500, check_every=1, seed=14),
    dict(n=33, dtype="f64", odf=27, tol=0.0, max_iters=45, check_every=0, seed=15),     # no checks
    dict(n=9, dtype="f64", odf=1, tol=1e-9, max_iters=1000, check_every=25, seed=16),
]


def _oracle(req):
    return oracle.solve(req["n"], DT[req["dtype"]], seed=req["seed"], iters=req["max_iters"],
                        tol=req["tol"], check_every=req["check_every"])


def _check(res, field, req):
    want, it, r = _oracle(req)
    assert res["state"] == "done"
    assert res["iters"] == it, (req, res["iters"], it)
    assert res["residual"] == r, (req, res["residual"], r)
    assert field.dtype == want.dtype and np.array_equal(field, want), req


def test_mix_matches_oracle_and_alone():
    with Server(arena_bytes=512 << 20, max_slots=16) as srv:
        # odd requests carry an arrival stamp taken before submission; the
        # others arrive at their submit time
        t_arr = time.monotonic() - 0.25
        tickets = [srv.submit(**q, t_arrival=t_arr if i % 2 else 0.0) for i, q in enumerate(MIX)]
        mixed = []
        for i, (t, q) in enumerate(zip(tickets, MIX)):
            res = srv.wait(t)
            field = srv.fetch(t)
            _check(res, field, q)
            assert res["t_arrival"] <= res["t_submit"] <= res["t_admit"] <= res["t_done"]
            if i % 2:
                assert res["t_arrival"] == t_arr
            else:
                assert res["t_arrival"] == res["t_submit"]
            mixed.append((res, field))
    # each request alone on a fresh server gives the same bits
    for q, (res_m, field_m) in zip(MIX[:3], mixed[:3]):
        with Server(arena_bytes=256 << 20, max_slots=4) as srv:
            t = srv.submit(**q)
            res = srv.wait(t)
            field = srv.fetch(t)
        assert res["iters"] == res_m["iters"] and res["residual"] == res_m["residual"]
        assert np.array_equal(field, field_m)


def test_staggered_arrivals_join_running_work():
    # requests arriving while others run are admitted into later epochs
    reqs = [dict(n=30, dtype="f64", odf=8, tol=0.0, max_iters=400, check_every=0, seed=21 + i) for i in range(3)]
    reqs += [dict(n=14, dtype="f32", odf=1, tol=1e-4, max_iters=800, check_every=5, seed=31 + i) for i in range(3)]
    with Server(arena_bytes=512 << 20, max_slots=8) as srv:
        tickets = []
        for q in reqs:
            tickets.append(srv.submit(**q))
            time.sleep(0.002)
        for t, q in zip(tickets, reqs):
            res = srv.wait(t)
            _check(res, srv.fetch(t), q)


def test_budget_admission_limits_residency():
    q = dict(n=36, dtype="f64", odf=8, tol=0.0, max_iters=150, check_every=0)
    need = request_bytes(**q)
    # control region + room for two solves only
    with Server(arena_bytes=control_bytes(4) + 2 * need + 4096, max_slots=4) as srv:
        tickets = [srv.submit(**q, seed=40 + i) for i in range(5)]
        peak = 0
        t0 = time.monotonic()
        while time.monotonic() - t0 < 60:
            a, _ = srv.counts()
            peak = max(peak, a)
            if all(srv.poll(t) is not None for t in tickets):
                break
            time.sleep(5e-4)
        assert peak <= 2
        admits = []
        for i, t in enumerate(tickets):
            res = srv.wait(t)
            admits.append(res["t_admit"])
            _check(res, srv.fetch(t), dict(q, seed=40 + i))
        # FIFO admission
        assert admits == sorted(admits)


def test_request_errors():
    with Server(arena_bytes=128 << 20, max_slots=2) as srv:
        with pytest.raises(ODError) as ei:
            srv.submit(n=1000, dtype="f64", odf=1)     # cannot ever fit the arena
        assert ei.value.status in (-12, -22)
        with pytest.raises(ODError) as ei:
            srv.submit(n=0, dtype="f64")
        assert ei.value.status == -22
        with pytest.raises(ODError) as ei:
            srv.submit(n=8, dtype="f64", odf=1000)
        assert ei.value.status == -22
        t = srv.submit(n=10, dtype="f64", odf=1, tol=0.0, max_iters=20, check_every=0)
        res = srv.wait(t)
        assert res["iters"] == 20
        with pytest.raises(ODError):
            srv.poll(t + 1000)


def test_close_with_work_in_flight():
    # closing the server stops running epochs promptly, cancels what is
    # unfinished and still completes the copy-out of finished solves
    srv = Server(arena_bytes=512 << 20, max_slots=8)
    try:
        q = dict(n=10, dtype="f64", odf=1, tol=0.0, max_iters=20, check_every=0, seed=1)
        small = srv.submit(**q)
        for i in range(3):
            srv.submit(n=64, dtype="f64", odf=8, tol=0.0, max_iters=10**6, check_every=0, seed=2 + i)
        res = srv.wait(small)
        _check(res, srv.fetch(small), q)
        # the retire thread books its time just after the result is published
        t0 = time.monotonic()
        while srv.stats()["retire_s"] == 0.0 and time.monotonic() - t0 < 5.0:
            time.sleep(1e-3)
        assert srv.stats()["retire_s"] > 0.0
    finally:
        t0 = time.monotonic()
        srv.close()
        assert time.monotonic() - t0 < 30.0
