"""Continuous-batching request loop for gas-kinetic solves on one GPU.

Each request is a solve (a Case) that runs until its residual has fallen by `tol`
relative to its first step (max over fields of res_m / res_first_m) or until
`max_steps`.  The server keeps every admitted solve's state on the device and advances
all of them together with the persistent batch kernels (a captured graph of several
steps; admissions and retirements rewrite the batch table in place).  Requests are admitted in
arrival order (or, with order="shortest", smallest expected work first: cells x step
cap) whenever a batch slot and enough HBM (the solve's workspace footprint) are free and
the cells already in the batch do not saturate the GPU (`sat_cells`: past that point a
further member only shares the GPU, lengthening every member's time without adding
throughput); new solves are initialised on a separate stream so that their set-up overlaps
the running batch.  For comparison `run_fifo` serves the same trace one solve at a time
with the plain per-solve loop.

Latency of a request = completion time - arrival time (wall clock, arrivals replayed in
real time from the trace).

Both loops advance their work in quanta of steps sized to about `target_s` of GPU time
(from the measured time of the previous quantum, at least `quantum` steps), so that the
per-quantum host work (reading the states back, admitting, retiring) stays a small
fraction of the GPU time.  A solve stops on the device, at the end of the step where its
residual has fallen by `tol` (the request's tolerance, set as the solve's res_tol) or at
its step cap, so a quantum that overshoots a solve's end costs no work and no steps (the
kernels pass a stopped solve), only up to one quantum of detection delay; its steps and
final state are those of the solve run alone, whatever the quanta.
"""
from __future__ import annotations

import collections
import time

import numpy as np


def _converged(res, res_first, steps, tol, max_steps, nv):
    """The device's stopping rule (residual fall by tol after step 2, or the step cap),
    evaluated on the host from a solve's residuals."""
    if steps >= max_steps:
        return True
    r0 = np.asarray(res_first[:nv])
    r = np.asarray(res[:nv])
    mask = r0 > 0
    if steps < 2 or not np.any(mask):
        return False
    return float(np.max(r[mask] / r0[mask])) <= tol


def _next_quantum(q, gpu_ms, quantum, target_s, q_max=4000):
    """Steps of the next quantum: about target_s of GPU time at the last measured rate."""
    if gpu_ms <= 0.0:
        return q
    per_step = gpu_ms * 1e-3 / q
    return int(min(q_max, max(quantum, target_s / per_step)))


def _summary(lat, cell_updates, makespan, n):
    lat = np.asarray(lat)
    return {
        "requests": n,
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_latency_s": float(np.mean(lat)) if len(lat) else None,
        "makespan_s": makespan,
        "throughput_req_s": n / makespan if makespan > 0 else None,
        "cell_updates_per_s": cell_updates / makespan if makespan > 0 else None,
    }


def run_batched(requests, make_case, hbm_budget=64 << 30, capacity=64, quantum=20, keep_fields=False,
                device="cuda:0", target_s=0.004, log=None, sat_cells=None, order="arrival", graph_steps=16):
    """Serve `requests` (dicts with id, arrival [s], max_steps, tol) with continuous
    batching.  Returns (summary, per-request records).  `log(msg)`, if given, is called
    every 16 completions.

    Each iteration enqueues the next `quantum` steps of the running batch first, then does
    the host work (building and initialising newly arrived solves on their own stream)
    while those steps run, then synchronises, retires finished solves and admits the new
    ones by rewriting the batch table in place.  The steps replay a graph of `graph_steps`
    captured steps (quanta are rounded up to whole replays)."""
    import torch

    from . import gks as G
    torch.cuda.set_device(device)
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    if sat_cells is None:
        sat_cells = 8192 * cus          # ~2M cells: a few waves of tiles on every CU
    run_stream = torch.cuda.Stream(device=device)
    init_stream = torch.cuda.Stream(device=device)
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    queue = collections.deque()
    active = []          # (req, solver, bytes) being stepped by the batch
    records = {}
    used = 0
    batch = None
    classes = set()
    cell_updates = 0
    q = quantum
    ndone = 0
    cells_in = 0         # cells of the active and staged solves
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    while pending or queue or active:
        t = now()
        while pending and pending[0]["arrival"] <= t:
            queue.append(pending.popleft())
        if active:
            q = -(-q // graph_steps) * graph_steps       # whole replays of the captured steps
            ev0.record(run_stream)
            batch.step(q)                                # GPU works while the host admits
            ev1.record(run_stream)
        staged = []
        while queue and len(active) + len(staged) < capacity:
            if order == "shortest":
                req = min(queue, key=lambda r: make_case(r).ncells * r["max_steps"])
            else:
                req = queue[0]
            case = make_case(req)
            case.res_tol = float(req["tol"])            # the device stops the solve there
            nbytes = G.gks_workspace_bytes(G.config_from_case(case))
            if (used + nbytes > hbm_budget or cells_in + case.ncells > sat_cells) and (active or staged):
                break                                    # wait for memory or GPU room
            queue.remove(req)
            cells_in += case.ncells
            with torch.cuda.stream(init_stream):
                solver = G.Solver(case, device=device, stream=init_stream)
            used += nbytes
            staged.append((req, solver, nbytes))
            records[req["id"]] = {"id": req["id"], "arrival": req["arrival"], "admitted": now(),
                                  "cells": case.ncells, "family": req.get("family"), "bytes": nbytes}
        retired = False
        if active:
            st = batch.status()                          # synchronises the run stream
            q = _next_quantum(q, ev0.elapsed_time(ev1), quantum, target_s)
            keep = []
            tnow = now()
            for i, item in enumerate(active):
                req, solver, nbytes = item
                steps, state = int(st["steps"][i]), int(st["state"][i])
                if state != 0 or _converged(st["res"][i], st["res_first"][i], steps, req["tol"],
                                            req["max_steps"], solver.case.nvar):
                    rec = records[req["id"]]
                    rec.update(done=tnow, latency=tnow - req["arrival"], steps=steps, state=state)
                    cell_updates += steps * rec["cells"]
                    if keep_fields:
                        rec["fields"] = solver.fields("cons")
                    solver.close()
                    used -= nbytes
                    cells_in -= rec["cells"]
                    retired = True
                    ndone += 1
                    if log is not None and ndone % 16 == 0:
                        log(f"batched: {ndone}/{len(requests)} done at {tnow:.1f} s, quantum {q}")
                else:
                    keep.append(item)
            active = keep
        if staged or retired:
            active = active + staged
            members = [s for _, s, _ in active]
            new_classes = {(s.case.dim, s.case.precision) for s in members}
            if batch is None:
                batch = G.Batch(members, capacity=capacity, device=device, stream=run_stream)
                for kind in (1, 2):
                    batch.set_launch(kind, 8 * cus, 0)
                for kind in (3, 4):
                    batch.set_launch(kind, 16 * cus, 64)
                batch.set_launch(0, 8 * cus, 0)
                batch.set_launch(5, 8 * cus, 0)
                batch.capture(steps=graph_steps)
                classes = new_classes
            else:
                batch.set_members(members)
                if not new_classes <= classes:           # a new kernel class joins: recapture
                    classes = classes | new_classes
                    batch.capture(steps=graph_steps)
        if not active and pending and not queue:
            time.sleep(max(0.0, min(0.05, pending[0]["arrival"] - now())))
    makespan = now()
    if batch is not None:
        batch.close()
    lat = [r["latency"] for r in records.values()]
    return _summary(lat, cell_updates, makespan, len(records)), records


def run_fifo(requests, make_case, quantum=20, keep_fields=False, device="cuda:0", target_s=0.004, log=None):
    """The same trace served one solve at a time with the plain per-solve loop."""
    import torch

    from . import gks as G
    torch.cuda.set_device(device)
    reqs = sorted(requests, key=lambda r: r["arrival"])
    records = {}
    cell_updates = 0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    for req in reqs:
        wait = req["arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        case = make_case(req)
        case.res_tol = float(req["tol"])                # the device stops the solve there
        s = G.Solver(case, device=device)
        q = quantum
        steps = 0
        while True:
            ev0.record()
            s.step(q)
            ev1.record()
            r = s.residual()                             # synchronises
            stopped = r["steps"] < steps + q             # the device stopped it within the quantum
            q = _next_quantum(q, ev0.elapsed_time(ev1), quantum, target_s)
            steps = r["steps"]
            if stopped or _converged(r["res"], r["res_first"], steps, req["tol"], req["max_steps"], case.nvar):
                break
        tnow = time.perf_counter() - t0
        rec = {"id": req["id"], "arrival": req["arrival"], "done": tnow, "latency": tnow - req["arrival"],
               "steps": steps, "cells": case.ncells, "family": req.get("family")}
        if keep_fields:
            rec["fields"] = s.fields("cons")
        cell_updates += steps * case.ncells
        s.close()
        records[req["id"]] = rec
        if log is not None and len(records) % 16 == 0:
            log(f"fifo: {len(records)}/{len(reqs)} done at {tnow:.1f} s")
    makespan = time.perf_counter() - t0
    lat = [r["latency"] for r in records.values()]
    return _summary(lat, cell_updates, makespan, len(records)), records
