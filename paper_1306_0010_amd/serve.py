"""Continuous batching of independent radiation-hydrodynamics solves on one GPU.

Requests arrive over time, each with its own grid, opacity, reduced speed of light and
number of gas steps. Between two batch steps the server admits waiting requests in
arrival order while two limits allow it: the device-memory budget (the sum of
``rhd_footprint_bytes`` of the admitted solves) and the number of slots. For each
admitted request it creates a handle, uploads the state and adds the handle to the
batch. Every batch step advances each active solve by one gas step (``rhd_batch_step``);
the radiation subcycles of all solves share launches over a packed tile list. A solve
that has taken its steps is copied back, removed and destroyed, which frees its memory
and slot for the next admission.

Latency is measured from a request's arrival to its result on the host. Synthesising a
request's initial state on the host is not counted: the clock stops while it runs, as
if the client had sent a ready state.

``serve_concurrent`` serves the same stream with the same admission rule, but each
admitted solve keeps its own handle and stream: the server advances the active solves one
gas step each in turn, so the steps of different solves run on the device at the same
time and a solve with few subcycles is not held back by one with many.

``serve_native`` hands the same stream to the native server (``rhd_server_*``): the
client only submits each request at its arrival and a few client threads collect the
results, while the server's own worker thread admits, batches, steps and retires the
solves. The initial
states are synthesised before the clock starts.

``serve_serial`` runs the same requests one at a time with one handle each, for
comparison.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import (RHD_KERNELS_TILED, RhdError, Server, Solver, params_from_spec, rhd_batch_add,
               rhd_batch_create, rhd_batch_destroy, rhd_batch_remove, rhd_batch_step,
               rhd_batch_sync, rhd_footprint_bytes)


class _Clock:
    """Wall clock that can be paused for work that is not the server's."""

    def __init__(self):
        self.t0 = time.perf_counter()
        self.excluded = 0.0

    def now(self):
        return time.perf_counter() - self.t0 - self.excluded

    def exclude(self, fn):
        t = time.perf_counter()
        out = fn()
        self.excluded += time.perf_counter() - t
        return out


def _percentiles(lat):
    a = np.sort(np.asarray(lat, dtype=np.float64))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def serve_batched(requests, make_problem, budget_bytes=16 << 30, max_slots=64, tile_rows=8,
                  zchunk=8, keep_results=False):
    """Serve ``requests`` (dicts with 'id', 'arrival' in seconds, 'steps') with
    continuous batching. ``make_problem(req)`` returns the problem dict (spec, state,
    chat). Returns a summary dict and, with keep_results, the final states by id."""
    order = [dict(r) for r in sorted(requests, key=lambda r: r["arrival"])]
    clock = _Clock()
    batch = rhd_batch_create(max_slots, tile_rows, zchunk)
    waiting = list(order)
    active = []  # dicts: req, solver, footprint, steps_done, cells
    used = 0
    lat, results, zone_updates, peak_active, steps_taken = {}, {}, 0, 0, 0
    try:
        while waiting or active:
            now = clock.now()
            # admission in arrival order, by memory budget and slots
            while waiting and waiting[0]["arrival"] <= now and len(active) < max_slots:
                req = waiting[0]
                if "_problem" not in req:
                    req["_problem"] = clock.exclude(lambda: make_problem(req))
                pb = req["_problem"]
                fp = rhd_footprint_bytes(params_from_spec(pb["spec"]))
                if used + fp > budget_bytes and active:
                    break
                waiting.pop(0)
                del req["_problem"]
                s = Solver(pb["spec"])
                s.set_state(pb["state"])
                rhd_batch_add(batch, s.h, pb["chat"])
                used += fp
                active.append({"req": req, "solver": s, "fp": fp, "done": 0,
                               "cells": int(np.prod(s.shape))})
                peak_active = max(peak_active, len(active))
            if not active:
                # idle until the next arrival
                wait = waiting[0]["arrival"] - clock.now()
                if wait > 0:
                    time.sleep(wait)
                continue
            nsub, _ = rhd_batch_step(batch)
            steps_taken += 1
            for a, ns in zip(active, nsub):
                a["done"] += 1
                zone_updates += a["cells"] * ns
            finished = [a for a in active if a["done"] >= a["req"]["steps"]]
            for a in finished:
                out = a["solver"].get_state()  # waits for the batch's stream
                lat[a["req"]["id"]] = clock.now() - a["req"]["arrival"]
                if keep_results:
                    results[a["req"]["id"]] = out
                rhd_batch_remove(batch, a["solver"].h)
                a["solver"].close()
                used -= a["fp"]
                active.remove(a)
        rhd_batch_sync(batch)
    finally:
        for a in active:
            rhd_batch_remove(batch, a["solver"].h)
            a["solver"].close()
        rhd_batch_destroy(batch)
    elapsed = clock.now()
    p50, p99 = _percentiles(list(lat.values()))
    summary = {"mode": "batched", "requests": len(lat), "zone_updates": zone_updates,
               "elapsed_s": elapsed, "zone_updates_per_s": zone_updates / elapsed,
               "p50_latency_s": p50, "p99_latency_s": p99, "peak_active": peak_active,
               "batch_steps": steps_taken, "budget_bytes": budget_bytes, "max_slots": max_slots}
    return summary, results


def serve_concurrent(requests, make_problem, budget_bytes=16 << 30, max_slots=16,
                     variant=None, keep_results=False):
    """Serve ``requests`` with continuous batching over independent handles, one stream
    each. Between rounds the server admits waiting requests in arrival order while the
    memory budget and the slot count allow; in each round every active solve computes its
    step size (which waits for its own previous step only) and enqueues one gas step.
    Returns a summary dict and, with keep_results, the final states by id."""
    order = [dict(r) for r in sorted(requests, key=lambda r: r["arrival"])]
    clock = _Clock()
    waiting = list(order)
    active = []  # dicts: req, solver, fp, done, cells, chat
    used = 0
    lat, results, zone_updates, peak_active, steps_taken = {}, {}, 0, 0, 0
    try:
        while waiting or active:
            now = clock.now()
            while waiting and waiting[0]["arrival"] <= now and len(active) < max_slots:
                req = waiting[0]
                if "_problem" not in req:
                    req["_problem"] = clock.exclude(lambda: make_problem(req))
                pb = req["_problem"]
                fp = rhd_footprint_bytes(params_from_spec(pb["spec"]))
                if used + fp > budget_bytes and active:
                    break
                waiting.pop(0)
                del req["_problem"]
                s = Solver(pb["spec"])
                if variant is not None:
                    s.set_kernel_variant(*variant)
                s.set_state(pb["state"])
                used += fp
                active.append({"req": req, "solver": s, "fp": fp, "done": 0, "chat": pb["chat"],
                               "cells": int(np.prod(s.shape))})
                peak_active = max(peak_active, len(active))
            if not active:
                wait = waiting[0]["arrival"] - clock.now()
                if wait > 0:
                    time.sleep(wait)
                continue
            for a in list(active):
                dt, ns = a["solver"].suggest_dt(a["chat"])
                a["solver"].step(dt, a["chat"], ns)
                a["done"] += 1
                steps_taken += 1
                zone_updates += a["cells"] * ns
                if a["done"] >= a["req"]["steps"]:
                    out = a["solver"].get_state()  # waits for this solve's stream
                    lat[a["req"]["id"]] = clock.now() - a["req"]["arrival"]
                    if keep_results:
                        results[a["req"]["id"]] = out
                    a["solver"].close()
                    used -= a["fp"]
                    active.remove(a)
    finally:
        for a in active:
            a["solver"].close()
    elapsed = clock.now()
    p50, p99 = _percentiles(list(lat.values()))
    summary = {"mode": "concurrent", "requests": len(lat), "zone_updates": zone_updates,
               "elapsed_s": elapsed, "zone_updates_per_s": zone_updates / elapsed,
               "p50_latency_s": p50, "p99_latency_s": p99, "peak_active": peak_active,
               "gas_steps": steps_taken, "budget_bytes": budget_bytes, "max_slots": max_slots}
    return summary, results


def serve_native(requests, make_problem, budget_bytes=16 << 30, max_slots=64, tile_rows=8,
                 zchunk=8, keep_results=False, collectors=4):
    """Serve ``requests`` through the native server. A request's latency runs from its
    arrival to the moment the server holds its final state in host memory (its
    ``t_done``). The calling thread submits each request at its arrival; ``collectors``
    client threads wait for the results and copy them out meanwhile, as separate clients
    would (a single thread that also copies every result out falls behind the server).
    Returns a summary dict and, with keep_results, the final states by id."""
    order = sorted(requests, key=lambda r: r["arrival"])
    problems = {r["id"]: make_problem(r) for r in order}
    lat, results = {}, {}

    def collect(srv, rid, req, late):
        info = srv.wait(rid)
        out, _, rc = srv.fetch(rid)
        if rc:
            raise RhdError(rc, f"request {req['id']} failed")
        return req["id"], late + info["t_done"] - info["t_submit"], info["zone_updates"], out

    with Server(budget_bytes, max_slots, tile_rows, zchunk) as srv, \
            ThreadPoolExecutor(max_workers=max(1, collectors)) as pool:
        t0 = time.perf_counter()
        futures = []
        for req in order:
            wait = req["arrival"] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            pb = problems[req["id"]]
            late = (time.perf_counter() - t0) - req["arrival"]
            rid = srv.submit(pb["spec"], pb["state"], pb["chat"], req["steps"])
            futures.append(pool.submit(collect, srv, rid, req, late))
        submitted = time.perf_counter() - t0
        zone_updates = 0
        for f in futures:  # in submission order; the first failure is raised
            i, latency, zu, out = f.result()
            lat[i] = latency
            zone_updates += zu
            if keep_results:
                results[i] = out
        elapsed = time.perf_counter() - t0
        st = srv.stats()
    p50, p99 = _percentiles(list(lat.values()))
    summary = {"mode": "native_server", "requests": len(lat), "zone_updates": zone_updates,
               "elapsed_s": elapsed, "zone_updates_per_s": zone_updates / elapsed,
               "p50_latency_s": p50, "p99_latency_s": p99, "peak_active": st["peak_running"],
               "batch_steps": st["rounds"], "peak_bytes": st["peak_bytes"],
               "budget_bytes": budget_bytes, "max_slots": max_slots,
               "last_submission_s": submitted}
    return summary, results


def serve_serial(requests, make_problem, keep_results=False, variant=None):
    """Serve the same requests one at a time, one handle each, in arrival order."""
    order = sorted(requests, key=lambda r: r["arrival"])
    clock = _Clock()
    lat, results, zone_updates = {}, {}, 0
    for req in order:
        wait = req["arrival"] - clock.now()
        if wait > 0:
            time.sleep(wait)
        pb = clock.exclude(lambda: make_problem(req))
        with Solver(pb["spec"]) as s:
            if variant is not None:
                s.set_kernel_variant(*variant)
            s.set_state(pb["state"])
            cells = int(np.prod(s.shape))
            for _ in range(req["steps"]):
                dt, ns = s.suggest_dt(pb["chat"])
                s.step(dt, pb["chat"], ns)
                zone_updates += cells * ns
            out = s.get_state()
        lat[req["id"]] = clock.now() - req["arrival"]
        if keep_results:
            results[req["id"]] = out
    elapsed = clock.now()
    p50, p99 = _percentiles(list(lat.values()))
    summary = {"mode": "one_at_a_time", "requests": len(lat), "zone_updates": zone_updates,
               "elapsed_s": elapsed, "zone_updates_per_s": zone_updates / elapsed,
               "p50_latency_s": p50, "p99_latency_s": p99}
    return summary, results


DEFAULT_VARIANT = (RHD_KERNELS_TILED, 8, 8)
