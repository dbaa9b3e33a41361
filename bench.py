"""Benchmark: overdecomposed 3D 7-point Jacobi on one MI355X.

Headline workload (one "step" = one pass of the whole hot path): a 512^3
fp64 interior split into 4096 chares of 32^3, 200 Jacobi iterations with the
halo exchange fused into the sweep, graph-captured, autotuned tile, residual
of the last sweep read back.  value = GLUP/s (10^9 lattice-site updates/s).

Prints ONE JSON line: the headline, the roofline of the sweep kernel (its
average launch time measured live with HIP events on the grid's stream),
the measured HBM ceilings (copy, read-only, write-only), and, by default,
every other part of the metric:
  odf_sweep        512^3 fp64 and fp32, ODF 8..4096: batched (graph-captured
                   fused launches), batched persistent (one cooperative launch),
                   message-driven (dependency-counting scheduler) and
                   per-chare launches, each with its roofline fraction
  amr_octree_768   768^3 fp64 octree of uneven blocks, 500 iterations:
                   graph-captured and persistent, plus the multi-resolution
                   reading (ghost fill by injection / averaging)
  imbalance_1024   1024^3 fp64, ODF 8..32768, 10% of chares re-run 1-4 times
                   per step: message-driven scheduler vs both bulk-synchronous
                   forms
  serving          Poisson stream of independent solves at 10..2000 /s under a
                   200 GB budget: p50/p99 of t_done - t_arrival, solves/s,
                   aggregate GLUP/s
and the CPU oracle on a bounded sample of the headline workload.

Optional legs: --jacobi2d (the paper's 2D workload, 32768^2 fp64), --launch
(launch-overlap microbenchmark).  --quick skips the default extra legs.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the fused sweeps' source: the prefetch-depth and halo-load
    settings and everything from the tile geometry to the end of k_sweep2
    (edits elsewhere in kernels.hip leave measured traffic valid)."""
    with open(os.path.join(ROOT, "paper_2605_12734_amd", "csrc", "kernels.hip")) as f:
        src = f.read()
    a = src.index("#ifndef OD_PREFETCH")
    b = src.index("namespace od {", a)
    c = src.index("#ifndef OD_MERGED_HALO")
    d = src.index("// Synchronisation between workgroups", c)
    h = hashlib.sha256()
    h.update(src[a:b].encode())
    h.update(src[c:d].encode())
    return h.hexdigest()[:16]


# Kernel whose device time the roofline divides by, per execution form (the
# persistent and message-driven forms run every iteration in one launch:
# their time per iteration is used).
KERNEL_OF_EXEC = {
    "graph": "k_sweep (fused 7-point sweep + halo pack/exchange/unpack)",
    "fused": "k_sweep (fused 7-point sweep + halo pack/exchange/unpack)",
    "per_chare": "k_sweep per chare + k_pack_b + k_unpack (time per iteration)",
    "persistent": "k_persistent (time per iteration)",
    "msgdriven": "k_msgdriven (time per iteration)",
}


def load_traffic(key: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(key)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


SCHEDULES = {1: "stride", 2: "counters", 3: "counters+guided-tail", 4: "runs"}


def msg_tile(tile):
    """Message-driven tile from a tuned fused tile: z extent at most 32."""
    return (tile[0], tile[1], min(tile[2], 32))


def msgdriven_tile(n, odf, dtype, fused_tile, iters=20,
                   shapes=((32, 16, 32), (32, 32, 32), (64, 16, 64), (32, 32, 64)), **kw):
    """The message-driven grid's tile: its dependency lists are built for
    the tiles it is created with, so instead of retiling one grid, short
    runs on grids of a few shapes (the fused grid's tuned tile with z <= 32,
    the tuned tile itself, then `shapes`) pick the fastest, outside any
    timed run; `kw` are further grid settings (the imbalance draw).  Tasks
    of two steps favour deeper tiles than tasks of one step did."""
    import paper_2605_12734_amd as od

    cands = []
    for t in (msg_tile(fused_tile), tuple(fused_tile)) + tuple(tuple(x) for x in shapes):
        if t not in cands:
            cands.append(t)
    best, best_s = cands[0], float("inf")
    for t in cands:
        try:
            g = od.Grid(n, odf=odf, dtype=dtype, exec="msgdriven", tile=t, hints=1, **kw)
        except od.ODError:
            continue
        try:
            g.iterate(4)
            s = min(g.time_iterate(iters) for _ in range(2))
        finally:
            g.close()
        if s < best_s:
            best, best_s = t, s
    return best


def make_grid(n, odf=None, blocks=None, dtype="f64", exec_="graph", tile=None, hints=1, autotune=True, **kw):
    import paper_2605_12734_amd as od

    if autotune and tile is None and exec_ in ("graph", "fused", "persistent"):
        g = od.Grid(n, odf=odf or 1, blocks=blocks, dtype=dtype, exec=exec_, hints=hints, **kw)
        g.autotune(TUNE_ITERS)
        return g
    if autotune and tile is None and exec_ in ("msgdriven", "per_chare"):
        # these modes take the shape tuned on a fused grid of the same
        # decomposition; message-driven tasks are tiles, so their z extent
        # is capped at 32 (deep tiles leave too few tasks to overlap)
        t = od.Grid(n, odf=odf or 1, blocks=blocks, dtype=dtype, exec="fused", hints=hints)
        tile = msg_tile(t.autotune(TUNE_ITERS)) if exec_ == "msgdriven" else t.autotune(TUNE_ITERS)
        t.close()
    return od.Grid(n, odf=odf or 1, blocks=blocks, dtype=dtype, exec=exec_, tile=tile, hints=hints, **kw)


def timed(g, iters, steps, warmup):
    """Wall and device time of `steps` x od_iterate(iters) after `warmup`."""
    import torch

    for _ in range(warmup):
        g.iterate(iters)
    g.residual()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(g.stream)
    for _ in range(steps):
        g.iterate(iters)
    ev1.record(g.stream)
    r = g.residual()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return {"wall_s": t1 - t0, "dev_s": ev0.elapsed_time(ev1) * 1e-3, "residual": r}


# passes timed per autotune candidate (2 measured within a few percent of
# noise; 6 separates candidates that close)
TUNE_ITERS = 6


def pass_gbps(plan, launch_s):
    """Algorithmic GB/s of the grid's own pass: the bytes one pass must move
    (one sweep, or a pair of steps where the grid runs two steps per pass)
    over the pass's device time; launch_s is the time per iteration."""
    return plan["bytes_per_pass"] / (launch_s * plan["steps_per_pass"]) / 1e9


def grid_leg(n, odf, dtype, exec_, iters, steps, warmup, tile=None, **kw):
    g = make_grid(n, odf=odf, dtype=dtype, exec_=exec_, tile=tile, **kw)
    try:
        plan = g.plan()
        t = timed(g, iters, steps, warmup)
    finally:
        g.close()
    lups = plan["interior"] * iters * steps
    t.update({"plan": plan, "glups": lups / t["wall_s"] / 1e9, "launch_s": t["dev_s"] / (iters * steps)})
    return t


def cpu_baseline(n, dtype, target_s=15.0, max_iters=200, chunk=10):
    """The oracle on this host's cores, on a bounded sample of the timed
    job (max_iters iterations: the steps x iterations the GPU ran): one call
    of as many iterations as take about target_s seconds, at the marginal
    rate of two short calls (chunk and 2 * chunk iterations; each call also
    copies the field once).  The one-thread rate is marginal too: two calls
    of 1 and 3 iterations, their difference over 2 iterations (the copy and
    first touch cancel out)."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    nt = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.set_threads(nt)
    U = oracle.init_field(n, np.float64 if dtype == "f64" else np.float32, 12734)
    oracle.jacobi(U, 1)                       # first touch, thread start-up
    t = time.perf_counter()
    oracle.jacobi(U, chunk)
    ta = time.perf_counter() - t
    t = time.perf_counter()
    oracle.jacobi(U, 2 * chunk)
    tb = time.perf_counter() - t
    per = max((tb - ta) / chunk, 1e-6)
    over = max(ta - chunk * per, 0.0)
    done = max(1, min(max_iters, int((target_s - over) / per)))
    t0 = time.perf_counter()
    oracle.jacobi(U, done)
    dt = time.perf_counter() - t0
    cores = int(oracle.max_threads())
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.jacobi(U, 1)
    d1 = time.perf_counter() - t1
    t1 = time.perf_counter()
    oracle.jacobi(U, 3)
    d3 = time.perf_counter() - t1
    per1 = max((d3 - d1) / 2, 1e-6)
    oracle.set_threads(nt)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(n ** 3 * done / dt / 1e9, 3), "unit": "GLUP/s", "cores": cores, "kind": "oracle",
            "sample": f"{n}^3 {dtype} undecomposed, {done} of the timed job's {max_iters} iterations "
                      f"({dt:.1f} s), same seed/bc",
            "single_thread_value": round(n ** 3 / per1 / 1e9, 4),
            "single_thread_sample": f"marginal rate of 1- and 3-iteration calls ({d1:.1f} s, {d3:.1f} s)",
            "cpu_model": model}


def odf_sweep(n, iters, persistent=True):
    """Per dtype and ODF: graph-captured fused launches (tile autotuned),
    the persistent cooperative form (tile and schedule autotuned on its own
    kernel), the message-driven form (the fastest of a few tiles in short
    runs, see msgdriven_tile), per-chare launches (the graph's tile).  Each
    batched form's roofline fraction divides the algorithmic bytes per
    iteration by its own kernel time per iteration (HIP events)."""
    rows = []
    for dtype in ("f64", "f32"):
        for odf in (8, 64, 512, 4096):
            b = grid_leg(n, odf, dtype, "graph", iters, 2, 1)
            tile = b["plan"]["tile"]
            bp = b["plan"]["bytes_per_iter"]
            k = round(odf ** (1 / 3))
            gb = pass_gbps(b["plan"], b["launch_s"])
            row = {"dtype": dtype, "odf": odf, "block": n // k, "tile": list(tile),
                   "batched_steps_per_pass": b["plan"]["steps_per_pass"],
                   "batched_glups": round(b["glups"], 2),
                   "batched_hbm_gbps": round(gb, 1),
                   "batched_frac": round(gb / PEAK_HBM_GBPS, 4),
                   "batched_step_bytes_frac": round(bp / b["launch_s"] / 1e9 / PEAK_HBM_GBPS, 4)}
            if persistent:
                # tile and schedule tuned on the persistent kernel itself
                q = grid_leg(n, odf, dtype, "persistent", iters, 2, 1)
                gq = pass_gbps(q["plan"], q["launch_s"])
                row.update({"persistent_tile": list(q["plan"]["tile"]),
                            "persistent_schedule": SCHEDULES.get(q["plan"]["schedule"], q["plan"]["schedule"]),
                            "persistent_steps_per_pass": q["plan"]["steps_per_pass"],
                            "persistent_glups": round(q["glups"], 2),
                            "persistent_hbm_gbps": round(gq, 1),
                            "persistent_frac": round(gq / PEAK_HBM_GBPS, 4),
                            "persistent_step_bytes_frac": round(bp / q["launch_s"] / 1e9 / PEAK_HBM_GBPS, 4),
                            "persistent_us_per_iter": round(q["launch_s"] * 1e6, 2),
                            "persistent_grid_wgs": q["plan"]["grid_wgs"]})
                m = grid_leg(n, odf, dtype, "msgdriven", iters, 2, 1, tile=msgdriven_tile(n, odf, dtype, tile))
                gm = pass_gbps(m["plan"], m["launch_s"])
                row.update({"msgdriven_tile": list(m["plan"]["tile"]),
                            "msgdriven_steps_per_pass": m["plan"]["steps_per_pass"],
                            "msgdriven_glups": round(m["glups"], 2),
                            "msgdriven_hbm_gbps": round(gm, 1),
                            "msgdriven_frac": round(gm / PEAK_HBM_GBPS, 4),
                            "msgdriven_grid_wgs": m["plan"]["grid_wgs"]})
            pc_iters = 10 if odf <= 64 else (4 if odf <= 512 else 2)
            p = grid_leg(n, odf, dtype, "per_chare", pc_iters, 1, 1, tile=tile)
            row.update({"per_chare_glups": round(p["glups"], 3),
                        "per_chare_ms_per_iter": round(p["wall_s"] / pc_iters * 1e3, 2),
                        "speedup_batched_vs_per_chare": round(b["glups"] / p["glups"], 1)})
            if persistent:
                row["speedup_persistent_vs_per_chare"] = round(row["persistent_glups"] / p["glups"], 1)
            log("odf sweep:", row)
            rows.append(row)
    return rows


def amr_leg(iters=500, multires_only=False):
    import workloads

    blocks = workloads.octree_blocks(n=768, root=128, min_edge=16, p_refine=0.4, seed=12734)
    out = {"blocks": len(blocks), "edges": sorted({e[0] for _, e in blocks})}
    for exec_ in () if multires_only else ("graph", "persistent"):
        g = make_grid(768, blocks=blocks, dtype="f64", exec_=exec_)
        try:
            plan = g.plan()
            t = timed(g, iters, 1, 1)
        finally:
            g.close()
        bp = plan["bytes_per_iter"]
        gb = pass_gbps(plan, t["dev_s"] / iters)
        out[exec_] = {"glups": round(plan["interior"] * iters / t["wall_s"] / 1e9, 2),
                      "steps_per_pass": plan["steps_per_pass"],
                      "hbm_gbps": round(gb, 1),
                      "frac": round(gb / PEAK_HBM_GBPS, 4),
                      "step_bytes_frac": round(bp * iters / t["dev_s"] / 1e9 / PEAK_HBM_GBPS, 4),
                      "tile": list(plan["tile"]), "tiles": plan["ntiles"], "iters": iters}
        log("amr:", exec_, out[exec_])
    # multi-resolution reading: the same octree, 16 cells per leaf edge
    # (finest leaves unit cells), resolution-change faces filled by
    # injection / face averaging before every sweep
    cell = [e[0] // 16 for _, e in blocks]
    # graph: the ghost fill and the sweep as two kernels per iteration;
    # persistent: both in one cooperative launch, a barrier after each
    for exec_ in ("graph", "persistent"):
        g = make_grid(768, blocks=blocks, dtype="f64", exec_=exec_, cell=cell)
        try:
            plan = g.plan()
            t = timed(g, iters, 1, 1)
        finally:
            g.close()
        bp = plan["bytes_per_iter"]
        key = "multires_" + exec_
        out[key] = {"cells": plan["interior"], "glups": round(plan["interior"] * iters / t["wall_s"] / 1e9, 2),
                    "hbm_gbps": round(bp * iters / t["dev_s"] / 1e9, 1),
                    "frac": round(bp * iters / t["dev_s"] / 1e9 / PEAK_HBM_GBPS, 4),
                    "tile": list(plan["tile"]), "tiles": plan["ntiles"], "iters": iters}
        log("amr: multires", exec_, out[key])
    return out


def imbalance_leg(iters=1000, odfs=(8, 64, 512, 4096, 32768)):
    """Each form with its own tile: the fused autotuner's (the persistent
    form takes the same), and for the message-driven form the fastest of
    short runs under the same imbalance (msgdriven_tile over the fused tile,
    its z <= 32 cut, (32,16,32) and (64,16,64))."""
    rows = []
    imb = {"imbalance_pct": 10, "imbalance_max_extra": 4}
    for odf in odfs:
        row = {"odf": odf, "block": 1024 // round(odf ** (1 / 3))}
        tile = mtile = None
        for exec_ in ("fused", "persistent", "msgdriven"):
            if exec_ == "msgdriven":
                mtile = msgdriven_tile(1024, odf, "f64", tile, iters=40, shapes=((32, 16, 32), (64, 16, 64)), **imb)
            g = make_grid(1024, odf=odf, dtype="f64", exec_=exec_,
                          tile=mtile if exec_ == "msgdriven" else tile, **imb)
            try:
                tile = tile or g.plan()["tile"]
                plan = g.plan()
                t = timed(g, iters, 1, 0)
            finally:
                g.close()
            row[exec_ + "_glups"] = round(plan["interior"] * iters / t["wall_s"] / 1e9, 2)
            row[exec_ + "_s"] = round(t["wall_s"], 3)
        row["tile_bsp"] = list(tile)
        row["tile_msgdriven"] = list(mtile)
        row["msgdriven_vs_bsp_launches"] = round(row["msgdriven_glups"] / row["fused_glups"], 3)
        row["msgdriven_vs_bsp_barrier"] = round(row["msgdriven_glups"] / row["persistent_glups"], 3)
        log("imbalance:", row)
        rows.append(row)
    return rows


def jacobi2d_leg(n=32768, iters=100, odfs=(1, 4, 16, 64, 256, 1024)):
    """The paper's Jacobi2D workload on one GPU's share: n^2 fp64, 5-point,
    `iters` iterations, batched (graph) vs per-chare launches per ODF."""
    import paper_2605_12734_amd as od

    rows = []
    for odf in odfs:
        t = od.Grid2D(n, odf=odf, dtype="f64", exec="fused", hints=1)
        try:
            tile = t.autotune(TUNE_ITERS)
        finally:
            t.close()
        row = {"n": n, "odf": odf, "tile": list(tile)}
        for exec_, it, steps in (("graph", iters, 2), ("per_chare", 10 if odf <= 64 else 4, 1)):
            g = od.Grid2D(n, odf=odf, dtype="f64", exec=exec_, tile=tile, hints=1)
            try:
                plan = g.plan()
                tm = timed(g, it, steps, 1)
            finally:
                g.close()
            glups = plan["interior"] * it * steps / tm["wall_s"] / 1e9
            row[exec_ + "_glups"] = round(glups, 2)
            if exec_ == "graph":
                gbps = pass_gbps(plan, tm["dev_s"] / (it * steps))
                row["graph_steps_per_pass"] = plan["steps_per_pass"]
                row["graph_hbm_gbps"] = round(gbps, 1)
                row["graph_frac"] = round(gbps / PEAK_HBM_GBPS, 4)
                row["graph_step_bytes_frac"] = round(
                    plan["bytes_per_iter"] * it * steps / tm["dev_s"] / 1e9 / PEAK_HBM_GBPS, 4)
                row["graph_ms_per_100_iters"] = round(tm["wall_s"] / (it * steps) * 100 * 1e3, 2)
        row["speedup_batched_vs_per_chare"] = round(row["graph_glups"] / row["per_chare_glups"], 1)
        log("jacobi2d:", row)
        rows.append(row)
    return rows


def launch_leg(totals=(1 << 18, 1 << 20), kernels=(1, 2, 4, 8, 16, 32, 64, 256, 1024), works=(0, 20000)):
    """Launch-overlap microbenchmark: the same work split over more kernels,
    all released at once from a stream gate (device makespan vs ODF; work 0
    isolates the per-kernel device cost)."""
    import paper_2605_12734_amd as od

    overlap = []
    for work in works:
        for total in totals:
            base = None
            for nk in kernels:
                best = None
                for _ in range(3):
                    r = od.launch_overlap(total, nk, work=work)
                    best = r if best is None or r["makespan_us"] < best["makespan_us"] else best
                base = base or best["makespan_us"]
                row = {"work": work, "threads": total, "kernels": nk, "streams": best["nstreams"],
                       "makespan_us": round(best["makespan_us"], 1), "host_us": round(best["host_us"], 1),
                       "enqueue_us": round(best["enqueue_us"], 1),
                       "makespan_vs_1_kernel": round(best["makespan_us"] / base, 3)}
                log("launch overlap:", row)
                overlap.append(row)
    return {"overlap": overlap}


def serving_leg(rates=(10, 30, 100, 300, 1000, 2000), count=128, arena_gb=200.0):
    import torch

    from paper_2605_12734_amd.serving import Server

    free = torch.cuda.mem_get_info()[0]
    arena = int(min(arena_gb * 1e9, free * 0.85)) // 256 * 256
    out = []
    # one server (one arena) for every arrival rate: the arena is most of HBM
    with Server(arena_bytes=arena, max_slots=min(count, 256)) as srv:
        for rate in rates:
            out.append(_serve_rate(srv, rate, count))
    return out


def _serve_rate(srv, rate, count):
    """Submit a seeded Poisson stream at its arrival times; every request
    carries its scheduled arrival time (t_arrival, the server's monotonic
    clock), so latency = t_done - t_arrival counts any delay before
    od_submit.  Finished fields are fetched by a second thread, so the
    submitting loop only plans and submits."""
    import queue
    import threading

    import numpy as np

    import workloads

    reqs = workloads.serving_requests(rate, count, seed=12734 + int(rate))
    st0 = srv.stats()
    fetch_q: "queue.Queue" = queue.Queue()
    fetch_err = []

    def fetcher():
        while True:
            t = fetch_q.get()
            if t is None:
                return
            try:
                srv.fetch(t)
            except Exception as ex:   # reported after the run
                fetch_err.append(repr(ex))

    th = threading.Thread(target=fetcher, daemon=True)
    th.start()
    t0 = time.monotonic()
    tickets = {}
    lag = []
    pending = list(reqs)
    done = {}
    try:
        while pending or len(done) < len(reqs):
            now = time.monotonic()
            while pending and t0 + pending[0]["t_arrival"] <= now:
                q = pending.pop(0)
                ta = t0 + q["t_arrival"]
                tk = srv.submit(q["n"], q["dtype"], odf=q["odf"], tol=q["tol"], max_iters=q["max_iters"],
                                check_every=q["check_every"], seed=q["seed"], t_arrival=ta)
                tickets[tk] = q
                now = time.monotonic()
                lag.append(now - ta)
            for t in list(tickets):
                if t in done:
                    continue
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
                    fetch_q.put(t)
            if pending and not any(t not in done for t in tickets):
                time.sleep(max(0.0, min(0.002, t0 + pending[0]["t_arrival"] - time.monotonic())))
            else:
                time.sleep(2e-4)
    finally:
        fetch_q.put(None)
        th.join()
    if fetch_err:
        raise RuntimeError("serving fetch failed: " + fetch_err[0])
    lat = np.array([done[t]["t_done"] - done[t]["t_arrival"] for t in tickets])
    first = min(r["t_arrival"] for r in done.values())
    last = max(r["t_done"] for r in done.values())
    lups = sum(q["n"] ** 3 * done[t]["iters"] for t, q in tickets.items())
    lag = np.array(lag)
    row = {"rate": rate, "requests": count, "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
           "solves_per_s": round(count / (last - first), 2), "glups": round(lups / (last - first) / 1e9, 2),
           "mean_iters": round(float(np.mean([r["iters"] for r in done.values()])), 1),
           "submit_lag_ms": {"p50": round(float(np.percentile(lag, 50)) * 1e3, 3),
                             "p99": round(float(np.percentile(lag, 99)) * 1e3, 3),
                             "max": round(float(lag.max()) * 1e3, 3)}}
    st1 = srv.stats()
    wall = time.monotonic() - t0
    row["worker"] = {k: round(st1[k] - st0[k], 3) for k in ("epochs", "epoch_s", "admit_s", "retire_s", "idle_s")}
    row["worker"]["wall_s"] = round(wall, 3)
    log("serving:", row)
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=200, help="Jacobi iterations per step")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--odf", type=int, default=4096)
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--exec", default="graph")
    ap.add_argument("--tile", default=None, help="tx,ty,tz (default: autotuned)")
    ap.add_argument("--hints", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="headline, ceilings and CPU baseline only")
    ap.add_argument("--no-sweep", action="store_true", help="skip the ODF sweep")
    ap.add_argument("--no-ceilings", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-imbalance", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--imb-iters", type=int, default=1000)
    ap.add_argument("--amr-iters", type=int, default=500)
    ap.add_argument("--amr", action="store_true", help="with --quick: run the octree leg too")
    ap.add_argument("--amr-multires-only", action="store_true",
                    help="octree leg: only the multi-resolution grid")
    ap.add_argument("--jacobi2d", action="store_true")
    ap.add_argument("--launch", action="store_true")
    ap.add_argument("--serving-count", type=int, default=128)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "one GPU's share of chares only: a single-GPU benchmark; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import paper_2605_12734_amd as od

    t_start = time.monotonic()
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    log(f"bench: {args.n}^3 {args.dtype} odf {args.odf} {args.exec}, {args.iters} iterations/step, "
        f"warmup {args.warmup}, steps {args.steps}")
    leg = grid_leg(args.n, args.odf, args.dtype, args.exec, args.iters, args.steps, args.warmup, tile,
                   hints=args.hints)
    plan = leg["plan"]
    bytes_per_iter = plan["bytes_per_iter"]
    spp = plan["steps_per_pass"]
    achieved = pass_gbps(plan, leg["launch_s"])
    s = 8 if args.dtype == "f64" else 4
    strict = 2 * s * plan["interior"] / leg["launch_s"] / 1e9
    log(f"bench: {leg['glups']:.1f} GLUP/s, {leg['launch_s'] * 1e6:.1f} us/iteration, {spp} step(s) per pass, "
        f"{achieved:.0f} GB/s algorithmic, tile {plan['tile']}")

    ceil = None if args.no_ceilings else od.hbm_ceilings(4 << 30, iters=8)
    if ceil:
        log("bench: ceilings", ceil)

    k = round(plan["nchares"] ** (1 / 3))
    workload = (f"{args.n}^3 {args.dtype} odf{plan['nchares']} tile{'x'.join(map(str, plan['tile']))} "
                f"hints{args.hints} steps{spp}")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4),
            "traffic": load_traffic(workload) if args.exec in ("graph", "fused") else None,
            "kernel": (("k_persistent2 (every pass of two fused 7-point steps in one cooperative launch; "
                        "time per pass)" if args.exec == "persistent"
                        else "k_sweep2 (two fused 7-point steps per pass + halo reads)") if spp == 2
                       else KERNEL_OF_EXEC.get(args.exec, args.exec)),
            "steps_per_launch": spp,
            "alg_bytes_per_launch": plan["bytes_per_pass"],
            "avg_launch_us": round(leg["launch_s"] * spp * 1e6, 2),
            # the method's per-step bytes s(2N+G) over the time per step: with
            # two steps per pass the first step's traffic is never incurred
            "step_bytes_per_iter": bytes_per_iter,
            "step_bytes_frac": round(bytes_per_iter / leg["launch_s"] / 1e9 / PEAK_HBM_GBPS, 4),
            "strict_frac_2s_per_lup": round(strict / PEAK_HBM_GBPS, 4)}
    if ceil:
        roof.update({"copy_ceiling_gbps": ceil["copy_gbps"], "read_ceiling_gbps": ceil["read_gbps"],
                     "write_ceiling_gbps": ceil["write_gbps"],
                     "frac_of_copy_ceiling": round(achieved / ceil["copy_gbps"], 4)})
    out = {
        "metric": "GLUP/s at 512^3 fp64, ODF 4096 (batched: graph-captured fused sweeps); ODF sweep batched "
                  "(graph, persistent) vs per-chare; HBM GB/s vs roofline; octree, imbalance and serving "
                  "p50/p99 legs",
        "value": round(leg["glups"], 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(leg["wall_s"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic: SplitMix64 U[0,1) interior, Dirichlet 1 on x-, 0 elsewhere",
        "config": {"workload": f"{args.n}^3 {args.dtype} 7-point Jacobi, {plan['nchares']} chares of "
                               f"{args.n // k}^3, {args.iters} iterations per step, exec={args.exec}",
                   "odf": plan["nchares"], "iters_per_step": args.iters, "tile": list(plan["tile"]),
                   "exec": args.exec, "hints": args.hints},
        "roofline": roof,
        "residual": leg["residual"],
    }
    if ceil:
        out["hbm_ceilings"] = ceil
    legs = []
    if not args.no_sweep and not args.quick:
        legs.append(("odf_sweep", lambda: odf_sweep(args.n, args.iters)))
    if (args.amr or not args.quick) and not args.no_amr:
        legs.append(("amr_octree_768", lambda: amr_leg(args.amr_iters, args.amr_multires_only)))
    if not args.quick and not args.no_imbalance:
        legs.append(("imbalance_1024", lambda: imbalance_leg(args.imb_iters)))
    if not args.quick and not args.no_serving:
        legs.append(("serving", lambda: serving_leg(count=args.serving_count)))
    if args.jacobi2d:
        legs.append(("jacobi2d_32768", jacobi2d_leg))
    if args.launch:
        legs.append(("launch", launch_leg))
    leg_s = {}
    for name, fn in legs:
        t0 = time.monotonic()
        out[name] = fn()
        leg_s[name] = round(time.monotonic() - t0, 1)
        log(f"bench: leg {name} done in {leg_s[name]} s")
    t0 = time.monotonic()
    out["cpu_baseline"] = (None if args.no_cpu_baseline
                           else cpu_baseline(args.n, args.dtype, max_iters=args.iters * args.steps))
    leg_s["cpu_baseline"] = round(time.monotonic() - t0, 1)
    leg_s["total"] = round(time.monotonic() - t_start, 1)
    out["leg_seconds"] = leg_s
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
