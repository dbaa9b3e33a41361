"""Serving front end: independent Jacobi solves admitted under a device
memory budget and run concurrently by libod's message-driven scheduler
(od_server_* in include/od.h).  PyTorch provides the arena (device memory)
and the stream; admission, scheduling and completion run in libod."""
from __future__ import annotations

import ctypes
import time
from typing import Optional

import numpy as np

from . import _binding as B
from ._binding import ODError, check, lib

STATES = {0: "queued", 1: "running", 2: "done", 3: "canceled"}
DEFAULT_BC = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def make_request(n: int, dtype: str = "f64", odf: int = 1, tol: float = 1e-6, max_iters: int = 2000,
                 check_every: int = 10, seed: int = 12734, bc=DEFAULT_BC, t_arrival: float = 0.0) -> B.od_request:
    """t_arrival: arrival time on time.monotonic()'s clock (CLOCK_MONOTONIC,
    the server's clock); 0 = the submit time."""
    r = B.od_request()
    r.n = int(n)
    r.dtype = B.OD_F64 if dtype in ("f64", np.float64) else B.OD_F32
    r.odf = int(odf)
    r.tol = float(tol)
    r.max_iters = int(max_iters)
    r.check_every = int(check_every)
    r.seed = int(seed) & (2**64 - 1)
    for i in range(6):
        r.bc[i] = float(bc[i])
    r.t_arrival = float(t_arrival)
    return r


def request_bytes(**kw) -> int:
    r = make_request(**kw)
    out = ctypes.c_size_t()
    check(lib().od_request_bytes(ctypes.byref(r), ctypes.byref(out)), "od_request_bytes")
    return int(out.value)


def control_bytes(max_slots: int) -> int:
    out = ctypes.c_size_t()
    check(lib().od_server_control_bytes(int(max_slots), ctypes.byref(out)), "od_server_control_bytes")
    return int(out.value)


class Server:
    def __init__(self, arena_bytes: int, max_slots: int = 64, device: str = "cuda:0", stream=None):
        import torch

        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().od_server_create(ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                         int(max_slots), ctypes.byref(h)), "od_server_create")
        self.h = h
        self.meta = {}

    def submit(self, n: int, dtype: str = "f64", **kw) -> int:
        r = make_request(n, dtype, **kw)
        t = ctypes.c_uint64()
        check(lib().od_submit(self.h, ctypes.byref(r), ctypes.byref(t)), "od_submit")
        self.meta[int(t.value)] = (int(n), np.float64 if r.dtype == B.OD_F64 else np.float32)
        return int(t.value)

    def poll(self, ticket: int) -> Optional[dict]:
        """Info dict when finished, None while queued or running."""
        info = B.od_info()
        s = lib().od_poll(self.h, int(ticket), ctypes.byref(info))
        if s == B.OD_ENOTREADY:
            return None
        check(s, "od_poll")
        return {"state": STATES.get(info.state, info.state), "iters": info.iters, "residual": info.residual,
                "t_arrival": info.t_arrival, "t_submit": info.t_submit, "t_admit": info.t_admit,
                "t_done": info.t_done}

    def wait(self, ticket: int, timeout: float = 120.0, interval: float = 1e-3) -> dict:
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"request {ticket} not finished after {timeout} s")
            time.sleep(interval)

    def fetch(self, ticket: int) -> np.ndarray:
        n, dt = self.meta[ticket]
        out = np.empty((n + 2, n + 2, n + 2), dtype=dt)
        check(lib().od_fetch(self.h, int(ticket), out.ctypes.data, out.nbytes), "od_fetch")
        del self.meta[ticket]
        return out

    def set_hints(self, hints: int, seed: int = 12734) -> None:
        """Kernel hints of later scheduling epochs (4: schedule check)."""
        check(lib().od_server_set_hints(self.h, int(hints), int(seed) & (2**64 - 1)), "od_server_set_hints")

    def counts(self) -> tuple:
        a, q = ctypes.c_int32(), ctypes.c_int32()
        check(lib().od_server_step(self.h, ctypes.byref(a), ctypes.byref(q)), "od_server_step")
        return int(a.value), int(q.value)

    def stats(self) -> dict:
        """Time accounting: epochs, seconds in epochs, admission and idle
        (worker thread), retirement (retire thread, overlapping epochs)."""
        st = B.od_server_stats()
        check(lib().od_server_stats_get(self.h, ctypes.byref(st)), "od_server_stats_get")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self) -> None:
        if getattr(self, "h", None):
            check(lib().od_server_destroy(self.h), "od_server_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
