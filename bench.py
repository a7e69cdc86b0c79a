#!/usr/bin/env python3
"""Throughput of the gray M1 radiation-hydrodynamics hot path on one MI355X.

Headline: the 256^3 concentrated-source grid (outflow faces, static gas with a Gaussian
core of peak density 1e3 and sigma = 8 cells, emissivity j = 1 in the central 4^3 cells,
kappa_F = 1.2766 so that the core column is ~50, chat = c = 1, mixed precision). One
benchmark step is one radiation-only gas step of 10 Van Leer subcycles (each a predictor
and a corrector launch) followed by the FP64 ledger with its non-finite check; the
default 20 timed steps are the workload's 200 subcycles, from its initial state. The
state stays resident in HBM; nothing is copied to the host inside the timed region.

Prints one JSON line: the radiation zone-update rate (cells x subcycles per second); the
roofline of the dominant kernel from HIP-event timings of its launches inside a timed
pass of its own: its algorithmic HBM bytes against the 8 TB/s peak, with its FP32 VALU
lane-slot rate beside it; the FP64 CPU oracle timed on a bounded sample of the same input
on the host's cores. Extra keys hold the coupled operator-split step on the 128^3 linear
box, the 256^3 dusty shell over its 100 gas steps, the served batch of 512 requests with
its p50/p99 latencies, and the paper's own test problems.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "radiation zone-updates/s + % HBM peak; p50/p99 latency of batched solves"
HBM_PEAK_GBS = 8000.0
# FP32 VALU lane slots per second without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz (an FMA is one slot; a reciprocal or square root takes two: dependent chains of
# v_rcp/v_sqrt/v_rsq_f32 interleaved with FMAs run at 1/2.9 of the FMA-only rate on
# gfx950, i.e. about 1.9 slots each)
VALU_PEAK_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12
# published MI355X FP32 vector peak (packed FMA: 4 flops per lane and clock)
FP32_PEAK_TFLOPS = 157.3
KERNEL_SOURCES = ("paper_1306_0010_amd/csrc/rhd_device.hpp", "paper_1306_0010_amd/csrc/rhd_tile.hpp")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic.json")
# tile shapes (rows, z chunk) of the corrector and the gas stages for the two grid sizes
# on MI355X (the FP32 predictor takes 4-row tiles of at most 11 planes): at 128^3 the one
# rhd_autotune picked; at 256^3 the fastest corrector of a sweep of rows 4-16 x chunks
# 8-256: 16 x 64, one block per CU (277-281 us; 8 x 16 and 8 x 32 take 283-288, 16 x 16
# 299; at 4 rows its unrolled plane loop spills and takes 343 us)
TILE_C2 = (8, 8)
TILE_C3 = (16, 64)


def algorithmic_bytes_per_cell(kernel, spec, has_j, kappa_field):
    """Bytes a kernel must move per cell it processes if every field is read and written
    exactly once (see the data layout notes of the repository). es is 4 in mixed
    precision, 8 in FP64."""
    es = 4 if spec["precision"] == "mixed" else 8
    beta = spec["beta_tau"]
    absorb = spec["exchange"] == "absorb_only"
    gas_fields = 4 if spec["isothermal"] else 5
    frozen = 1 + (3 if beta else 0) + (1 if has_j else 0) + ((2 if absorb else 1) if kappa_field else 0)
    table = {
        "rad_predict": 4 + frozen + 4,            # U^m + frozen gas in, U^{m+1/2} out
        "rad_correct": 4 + 4 + frozen + 4,        # U^{m+1/2}, U^m, frozen gas in, U^{m+1} out
        "exchange": 6 + (1 if kappa_field else 0) + 2,
        "gas_predict": gas_fields + 4 + (1 if kappa_field else 0) + gas_fields,
        "gas_correct": 2 * gas_fields + 4 + (1 if kappa_field else 0) + gas_fields + 8,
        "gas_source_correct": 4 + 4 + gas_fields + 4 + (1 if kappa_field else 0) + gas_fields,
        "ledger": 9,
        "vmax": 6 + (1 if kappa_field else 0),
    }
    return table[kernel] * es


def algorithmic_slots_per_cell(kernel, spec, has_j):
    """FP32 VALU lane slots the arithmetic of one radiation stage takes per cell, counted
    from its formulas: every add, multiply, FMA, min, max, median and compare is one slot,
    a reciprocal or (reciprocal) square root two. Closure of one state along one
    direction: 31 + 4 transcendentals; HLL flux: 24 + 1; MC slope: 7 per field; face
    states: 8 per direction; divergence: 24; update (E_r, F with theta damping, floor and
    clamp): 35 + 1, plus 19 + 1 for the O(beta tau) terms, 2 for an emissivity and 9 + 1
    for absorption-only damping."""
    T = 2
    closure_state = 14 + 3 * T  # reduced flux, s, 3/(2+s), chat/s, (s-1)/3
    closure_dir = 17 + 1 * T    # physical flux and the two extreme eigenvalues
    hll = 24 + 1 * T
    update = 35 + 1 * T + (19 + T if spec["beta_tau"] else 0) + (2 if has_j else 0) \
        + (9 + T if spec["exchange"] == "absorb_only" else 0)
    div = 24
    if kernel == "rad_predict":
        return closure_state + 3 * closure_dir + 3 * hll + div + update
    if kernel == "rad_correct":
        return 3 * (4 * 7 + 8) + 6 * (closure_state + closure_dir) + 3 * hll + div + update
    return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, tile):
    """HBM bytes per launch from the committed hardware-counter record, if it was taken
    on the kernel sources as they are now and with the same tile shape; None otherwise."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    wl = rec.get("kernels", {}).get(workload, {})
    if tuple(wl.get("tile", ())) != tuple(tile):
        return None
    entry = wl.get(kernel)
    return None if entry is None else entry.get("bytes_per_launch")


def kernel_table(timing, spec, has_j, kappa_field):
    kernels = {}
    total = sum(v["total_ms"] for v in timing.values())
    for name, t in timing.items():
        if t["calls"] == 0:
            continue
        avg_ms = t["total_ms"] / t["calls"]
        b = algorithmic_bytes_per_cell(name, spec, has_j, kappa_field) * t["cells"]
        k = {"calls": t["calls"], "avg_us": 1e3 * avg_ms, "share": t["total_ms"] / max(1e-30, total),
             "cells_per_launch": t["cells"], "algorithmic_GBps": b / (avg_ms * 1e-3) / 1e9}
        sl = algorithmic_slots_per_cell(name, spec, has_j)
        if sl is not None:
            k["algorithmic_Tslots_per_s"] = sl * t["cells"] / (avg_ms * 1e-3) / 1e12
            k["slots_per_cell"] = sl
        kernels[name] = k
    return kernels


def roofline(kernels, spec, has_j, kappa_field, workload, tile):
    """The dominant radiation kernel: its algorithmic HBM bandwidth (bytes it must move
    per cell x cells per launch / average launch time) against the 8 TB/s peak, with the
    measured HBM traffic per launch when the counters were taken on the current kernel
    sources. Its FP32 VALU lane-slot rate stands beside it: non-packed slots (an FMA is one
    slot, a reciprocal or square root two) against 256 CUs x 64 lanes x 2.4 GHz =
    39.3 T slots/s, and, as an upper bound in flops (every slot an FMA of 2 flops),
    against the published 157.3 TFLOP/s FP32 peak (which counts packed FMAs)."""
    rad = {k: v for k, v in kernels.items() if k.startswith("rad_")}
    dom = max(rad, key=lambda k: rad[k]["share"])
    k = rad[dom]
    bpc = algorithmic_bytes_per_cell(dom, spec, has_j, kappa_field)
    traffic = measured_traffic(dom, workload, tile)
    slots = k["algorithmic_Tslots_per_s"]
    return {"bound": "hbm", "achieved": k["algorithmic_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": k["algorithmic_GBps"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": dom, "avg_us": k["avg_us"], "bytes_per_cell": bpc,
            "cells_per_launch": k["cells_per_launch"],
            "algorithmic_bytes_per_launch": bpc * k["cells_per_launch"],
            "traffic_over_algorithmic": None if traffic is None
            else traffic / (bpc * k["cells_per_launch"]),
            "valu": {"unit": "T lane-slots/s", "achieved": slots,
                     "slots_per_cell": k["slots_per_cell"],
                     "peak_nonpacked": VALU_PEAK_TSLOTS, "frac_nonpacked": slots / VALU_PEAK_TSLOTS,
                     "flops_upper_bound_TFLOPs": 2.0 * slots,
                     "published_fp32_peak_TFLOPs": FP32_PEAK_TFLOPS,
                     "frac_of_published_upper_bound": 2.0 * slots / FP32_PEAK_TFLOPS}}


MARSHAK_N = (32, 128, 512, 2048)
MARSHAK_TAU = (1.0, 10.0, 100.0)


def marshak_schedule(ri, n, tau_end):
    """Steps and face states of the Marshak problem (Sec. 4.1.3, eps = 1, chi in
    [0, 100]) on n cells up to tau_end: the boundary states are inputs, computed before
    any clock starts."""
    pb = ri.marshak_problem(n)
    dt = pb["dt"]
    steps = int(math.ceil(tau_end / dt - 1e-9))
    hs = [min(dt, tau_end - k * dt) for k in range(steps)]
    bvals = [ri.marshak_boundary(k * dt + 0.5 * hs[k]) for k in range(steps)]
    return pb, hs, bvals


def marshak_timing(P, ri, stream):
    """The paper's own timing benchmark (Sec. 4.2): wall time of the 1D Marshak wave to
    tau = 1, 10 and 100 for n = 32 ... 2048 cells, FP64 (mixed precision at 2048 as
    well), state resident on the device, one gas step of nsub = 1 per CFL step, boundary
    states precomputed; best of two runs. Two drivers: the whole sequence in one rhd_run
    call (fused 1D launches) and one rhd_set_boundary + rhd_step call per step."""
    import numpy as np
    import torch
    rows = []
    for prec in ("fp64", "mixed"):
        for n in (MARSHAK_N if prec == "fp64" else MARSHAK_N[-1:]):
            pb0 = ri.marshak_problem(n, precision=prec)
            sched = {tau: marshak_schedule(ri, n, tau) for tau in MARSHAK_TAU}
            for tau in MARSHAK_TAU:
                _, hs, bvals = sched[tau]
                hs_a = np.asarray(hs, dtype=np.float64)
                ns_a = np.ones(len(hs), dtype=np.int32)
                bv_a = np.asarray(bvals, dtype=np.float64)
                for driver in ("rhd_run", "rhd_step"):
                    el = float("inf")
                    for _ in range(2):  # best of two: the first run pays one-time costs
                        with P.Solver(pb0["spec"], stream=stream.cuda_stream) as s:
                            s.set_state(pb0["state"])
                            if driver == "rhd_run":  # allocate the step tables untimed
                                s.run(hs_a[:1], ns_a[:1], 1.0, bv_a[:1])
                                s.set_state(pb0["state"])
                            s.sync()
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            if driver == "rhd_run":
                                s.run(hs_a, ns_a, 1.0, bv_a)
                            else:
                                for h, bv in zip(hs, bvals):
                                    s.set_boundary(bv)
                                    s.step(h, 1.0, 1)
                            s.sync()
                            el = min(el, time.perf_counter() - t0)
                            u0 = float(s.get_state()["Er"][0, 0, 0])
                    rows.append({"n": n, "tau": tau, "precision": prec, "driver": driver,
                                 "steps": len(hs), "seconds": el,
                                 "us_per_step": 1e6 * el / len(hs),
                                 "zone_updates_per_s": n * len(hs) / el, "u_first_cell": u0})
    return {"workload": "marshak_wave_1d", "tau": list(MARSHAK_TAU), "n": list(MARSHAK_N),
            "rows": rows}


def cpu_baseline_marshak(ri, max_zone_updates=5e6):
    """The FP64 oracle (as it stands, one thread) on the same Marshak runs, except those
    of more than max_zone_updates (2048 cells to tau = 100: ~13 s alone)."""
    import oracle
    rows = []
    for n in MARSHAK_N:
        for tau in MARSHAK_TAU:
            pb, hs, bvals = marshak_schedule(ri, n, tau)
            if n * len(hs) > max_zone_updates:
                continue
            spec, st = dict(pb["spec"]), pb["state"]
            t0 = time.perf_counter()
            for h, bv in zip(hs, bvals):
                spec["bvals"] = bv
                st, _ = oracle.step(spec, st, h, 1.0, 1)
            el = time.perf_counter() - t0
            rows.append({"n": n, "tau": tau, "steps": len(hs), "seconds": el,
                         "zone_updates_per_s": n * len(hs) / el,
                         "u_first_cell": float(st["Er"][0, 0, 0])})
    return {"kind": "oracle", "cores": 1, "rows": rows}


def pulse_timing(P, ri, stream, n=512):
    """The advection of a radiation pulse (Sec. 4.3.2) at the paper's 512 cells to
    t = 2w/v, in FP64: the advected and the static run, with and without the O(beta tau)
    terms, each gas step at the CFL step the GPU suggests with its subcycles. Reports
    time per run and per gas step, and the largest relative differences of density and
    gas temperature between the advected and the static run (the paper's measure)."""
    import numpy as np
    import torch
    rows, finals = [], {}
    for beta_tau in (True, False):
        for advected in (True, False):
            pb = ri.pulse_problem(n, advected=advected, beta_tau=beta_tau)
            spec, chat = pb["spec"], pb["chat"]
            with P.Solver(spec, stream=stream.cuda_stream) as s:
                s.set_state(pb["state"])
                s.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                t, steps, subs = 0.0, 0, 0
                while t < pb["t_end"] * (1.0 - 1e-12):
                    dt, ns = s.suggest_dt(chat)
                    dt = min(dt, pb["t_end"] - t)
                    s.step(dt, chat, ns)
                    t += dt
                    steps += 1
                    subs += ns
                s.sync()
                el = time.perf_counter() - t0
                st, diag = s.get_state(), s.diagnostics()
            finals[(beta_tau, advected)] = (pb, st)
            rows.append({"workload": pb["name"], "gas_steps": steps, "subcycles": subs,
                         "seconds": el, "us_per_gas_step": 1e6 * el / steps,
                         "zone_subcycles_per_s": n * subs / el, "nonfinite": diag["nonfinite"]})
    errors = {}
    for beta_tau in (True, False):
        (pa, sa), (ps, ss) = finals[(beta_tau, True)], finals[(beta_tau, False)]
        Ta = ri.gas_temperature(pa["spec"], sa)[0, 0]
        Ts = ri.gas_temperature(ps["spec"], ss)[0, 0]
        key = "with_beta_tau" if beta_tau else "without_beta_tau"
        errors[key] = {"rho": float(np.max(np.abs(sa["rho"][0, 0] / ss["rho"][0, 0] - 1.0))),
                       "T_gas": float(np.max(np.abs(Ta / Ts - 1.0)))}
    return {"cells": n, "precision": "fp64", "rows": rows, "max_rel_error": errors,
            "paper_bounds": {"with_beta_tau": 0.066, "without_beta_tau": 0.077}}


def cpu_baseline_pulse(ri, n=512, gas_steps=100):
    """The FP64 oracle on the first gas steps of the advected pulse (a bounded sample)."""
    import oracle
    pb = ri.pulse_problem(n, advected=True, beta_tau=True)
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    subs = 0
    t0 = time.perf_counter()
    for _ in range(gas_steps):
        dt, ns, _ = oracle.suggest_dt(spec, st, chat)
        st, _ = oracle.step(spec, st, dt, chat, ns)
        subs += ns
    el = time.perf_counter() - t0
    return {"kind": "oracle", "cores": 1,
            "sample": f"{n} cells, the first {gas_steps} gas steps ({subs} subcycles)",
            "zone_subcycles_per_s": n * subs / el, "seconds": el}


def shell_timing(P, ri, stream, n=128, every=0.005):
    """The expanding-shell test of Sec. 4.3.6 at the paper's 128^3 octant to t = 0.124
    (the shell reaches 2 r0), mixed precision, for chat/a0 = 860, 430 and 215: time of
    the stepping (the sampling of <r> and <v_r> every `every` is outside the clock), gas
    steps and subcycles, and the largest relative errors of <r> and <v_r> against the
    trajectory of Eqs. radshell:odepos and radshell:odevel next to the paper's."""
    import torch
    paper = {860: (0.031, 0.070), 430: (0.053, 0.13), 215: (0.085, 0.23)}
    rows = []
    for chat in (860, 430, 215):
        pb = ri.shell_expansion_problem(n, chat_over_a0=float(chat), precision="mixed")
        spec = pb["spec"]
        samples = [(0.0,) + ri.shell_moments(spec, pb["state"], pb["r"])]
        with P.Solver(spec, stream=stream.cuda_stream) as s:
            s.set_state(pb["state"])
            s.sync()
            torch.cuda.synchronize()
            t, nxt, steps, subs, el = 0.0, every, 0, 0, 0.0
            while t < pb["t_end"] * (1 - 1e-12):
                t0 = time.perf_counter()
                while t < nxt * (1 - 1e-12):
                    dt, ns = s.suggest_dt(pb["chat"])
                    dt = min(dt, nxt - t)
                    s.step(dt, pb["chat"], ns)
                    t += dt
                    steps += 1
                    subs += ns
                s.sync()
                el += time.perf_counter() - t0
                samples.append((t,) + ri.shell_moments(spec, s.get_state(), pb["r"]))
                nxt = min(nxt + every, pb["t_end"])
            diag = s.diagnostics()
        er, ev = ri.shell_errors(pb["M0"], samples)
        rows.append({"workload": pb["name"], "chat_over_a0": chat, "gas_steps": steps,
                     "subcycles": subs, "seconds": el, "zone_subcycles_per_s": n ** 3 * subs / el,
                     "max_rel_error_r": er, "max_rel_error_vr": ev,
                     "paper_max_rel_error_r": paper[chat][0], "paper_max_rel_error_vr": paper[chat][1],
                     "final_r": samples[-1][1], "nonfinite": diag["nonfinite"]})
    return {"cells": [n, n, n], "precision": "mixed", "rows": rows}


def cpu_baseline_shell(ri, n=32, gas_steps=2):
    """The FP64 oracle on the first gas steps of the shell test at 32^3 (a bounded sample)."""
    import oracle
    pb = ri.shell_expansion_problem(n, precision="fp64")
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    subs = 0
    t0 = time.perf_counter()
    for _ in range(gas_steps):
        dt, ns, _ = oracle.suggest_dt(spec, st, chat)
        st, _ = oracle.step(spec, st, dt, chat, ns)
        subs += ns
    el = time.perf_counter() - t0
    return {"kind": "oracle", "cores": 1,
            "sample": f"{n}^3 cells, the first {gas_steps} gas steps ({subs} subcycles)",
            "zone_subcycles_per_s": n ** 3 * subs / el, "seconds": el}


def box_fp64_timing(P, ri, stream, n=128, steps=5, warmup=2):
    """The headline box in FP64 throughout (state, stencils, exchange, ledger) on the
    tiled kernels (8 rows x 8 planes): zone-updates/s over `steps` gas steps."""
    import torch
    pb = ri.c2_linear_box(n, precision="fp64")
    spec, chat = pb["spec"], pb["chat"]
    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, 8, 8)
        s.set_state(pb["state"])

        def one():
            dt, ns = s.suggest_dt(chat)
            s.step(dt, chat, ns)
            return ns

        for _ in range(warmup):
            one()
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sub = sum(one() for _ in range(steps))
        s.sync()
        el = time.perf_counter() - t0
    return {"workload": pb["name"], "precision": "fp64", "steps": steps,
            "ms_per_step": 1e3 * el / steps, "zone_updates_per_s": n ** 3 * sub / el}


def shadow_timing(P, ri, stream, crossings=10.0):
    """The shadow test of Sec. 4.1.1 at the paper's 280 x 80 cells for 10 horizontal
    light-crossing times, without and with emission, in mixed precision and FP64, in one
    rhd_run call each; the radiation temperature at the right boundary, behind the
    cloud (y < 0.045) and above it (y > 0.09), shows the shadow."""
    import numpy as np
    import torch
    rows = []
    for emission, precision in ((False, "mixed"), (True, "mixed"), (False, "fp64"),
                                (True, "fp64")):
        pb = ri.shadow_problem(280, 80, emission=emission, precision=precision)
        spec, dt, chat = pb["spec"], pb["dt"], pb["chat"]
        steps = int(math.ceil(crossings * pb["crossing"] / dt))
        with P.Solver(spec, stream=stream.cuda_stream) as s:
            s.set_state(pb["state"])
            s.set_boundary(spec["bvals"])
            s.sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run(np.full(steps, dt), np.ones(steps, dtype=np.int32), chat)
            s.sync()
            el = time.perf_counter() - t0
            st, diag = s.get_state(), s.diagnostics()
        y = (np.arange(spec["ny"]) + 0.5) * spec["dy"]
        Tr = ri.radiation_temperature(st["Er"][0, :, -1]) / pb["T1"]
        cells = spec["nx"] * spec["ny"]
        rows.append({"workload": pb["name"], "precision": precision, "steps": steps,
                     "seconds": el,
                     "us_per_step": 1e6 * el / steps, "zone_updates_per_s": cells * steps / el,
                     "T_rad_over_T1_shadow": float(np.mean(Tr[y < 0.045])),
                     "T_rad_over_T1_lit": float(np.mean(Tr[y > 0.09])),
                     "nonfinite": diag["nonfinite"]})
    return {"grid": [280, 80], "crossings": crossings, "rows": rows}


def cpu_baseline_shadow(ri, steps=2000):
    """The FP64 oracle on the shadow problem at 56 x 16 cells (a bounded sample)."""
    import oracle
    pb = ri.shadow_problem(56, 16, emission=True)
    t0 = time.perf_counter()
    oracle.step(pb["spec"], pb["state"], pb["dt"], pb["chat"], 1, steps=steps)
    el = time.perf_counter() - t0
    return {"kind": "oracle", "cores": 1, "sample": f"56x16 cells, {steps} steps, with emission",
            "zone_updates_per_s": 56 * 16 * steps / el, "seconds": el}


def host_info():
    """Cores and CPU model of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def oracle_threads(fn, jobs, threads):
    """Run fn(job) for every job on `threads` Python threads; the oracle's entry points
    are ctypes calls, which release the GIL, so the threads run on separate cores.
    Returns the wall time."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(fn, jobs))
    return time.perf_counter() - t0


def cpu_baseline_c3(ri, cut=64, subcycles=20, max_threads=16):
    """The FP64 oracle (as it stands) on a bounded sample of the headline workload: the
    central cut^3 cells of the 256^3 concentrated-source input (the core and the
    emitting cells, outflow faces), one radiation-only gas step of `subcycles`
    subcycles. Timed once on one thread, then with one copy of the same sample per
    thread on up to max_threads threads (the host's CPU share)."""
    import numpy as np
    import oracle
    pb = ri.c3_point_source(256, precision="fp64")
    n = pb["spec"]["nx"]
    lo = (n - cut) // 2
    sl = (slice(lo, lo + cut),) * 3
    spec = dict(pb["spec"], nx=cut, ny=cut, nz=cut, precision="fp64")
    st = {k: (np.ascontiguousarray(v[sl]) if isinstance(v, np.ndarray) else v)
          for k, v in pb["state"].items()}
    dt = pb["dt"] * subcycles
    info = host_info()
    threads = max(1, min(max_threads, info["usable_cpus"]))

    def one(_):
        oracle.step(spec, st, dt, pb["chat"], subcycles)

    el1 = oracle_threads(one, [0], 1)
    elp = oracle_threads(one, list(range(threads)), threads)
    zu = cut ** 3 * subcycles
    return {"value": threads * zu / elp, "unit": "zone-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"central {cut}^3 cells of the 256^3 concentrated-source input (core and "
                      f"emitting cells, outflow faces), {subcycles} radiation subcycles, FP64; one "
                      f"copy per thread on {threads} threads ({elp:.1f} s wall), and one thread "
                      f"alone ({el1:.1f} s)",
            "single_core_value": zu / el1, **info}


def cpu_baseline_c4(ri, cut=48, gas_steps=3, max_threads=16):
    """The FP64 oracle (as it stands) on a bounded sample of the dusty shell: a cut^3
    block of the 256^3 input centred on the shell where it crosses the +x axis (dense
    lognormal shell and ambient gas, outflow faces), `gas_steps` full operator-split gas
    steps at chat = 20 v_max(t=0) with the oracle's CFL subcycle counts. Timed once on
    one thread, then with one copy per thread on up to max_threads threads."""
    import numpy as np
    import oracle
    pb = ri.c4_dusty_shell(256, precision="fp64")
    n = pb["spec"]["nx"]
    xc = int(round((0.3 + 0.5) * n - 0.5))
    lo_x, lo_yz = xc - cut // 2, (n - cut) // 2
    sl = (slice(lo_yz, lo_yz + cut), slice(lo_yz, lo_yz + cut), slice(lo_x, lo_x + cut))
    spec = dict(pb["spec"], nx=cut, ny=cut, nz=cut, precision="fp64")
    st0 = {k: (np.ascontiguousarray(v[sl]) if isinstance(v, np.ndarray) and v.ndim == 3 else v)
           for k, v in pb["state"].items()}
    chat = pb["chat_over_vmax"] * oracle.suggest_dt(spec, st0, 1.0)[2]
    info = host_info()
    threads = max(1, min(max_threads, info["usable_cpus"]))
    subs = []

    def one(_):
        st, ns_all = st0, []
        for _ in range(gas_steps):
            dt, ns, _ = oracle.suggest_dt(spec, st, chat)
            st, _ = oracle.step(spec, st, dt, chat, ns)
            ns_all.append(ns)
        subs.append(sum(ns_all))

    el1 = oracle_threads(one, [0], 1)
    elp = oracle_threads(one, list(range(threads)), threads)
    zu = cut ** 3 * subs[0]
    return {"value": threads * zu / elp, "unit": "zone-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"a {cut}^3 block of the 256^3 dusty-shell input centred on the shell at "
                      f"x = +0.3 (outflow faces), {gas_steps} gas steps at chat = "
                      f"{chat:.3g} ({subs[0]} radiation subcycles in all), FP64; one copy per "
                      f"thread on {threads} threads ({elp:.1f} s wall), and one thread alone "
                      f"({el1:.1f} s)",
            "gas_step_zone_updates_per_s": threads * cut ** 3 * gas_steps / elp,
            "single_core_value": zu / el1, **info}


def cpu_baseline_c5(ri, pert, requests=16, nz_slab=8, max_threads=16):
    """The FP64 oracle (as it stands) on a bounded sample of the served stream: its
    first `requests` requests (the same seeded boxes and perturbations as the GPU's
    stream), each cut to its first nz_slab z-planes as a periodic slab and advanced by
    one gas step (exchange, gas VL, its CFL radiation subcycles, correction). One
    request per thread on up to max_threads threads; the rate is all zone-updates over
    the wall time."""
    import numpy as np
    import oracle
    reqs = ri.c5_requests(count=requests)
    info = host_info()
    threads = max(1, min(max_threads, info["usable_cpus"], requests))
    done = {}

    def one(r):
        pb = ri.c5_problem(r, precision="fp64", perturbations=pert[r["id"]])
        nz = min(nz_slab, r["nz"])
        spec = dict(pb["spec"], nz=nz, precision="fp64")
        st = {k: (np.ascontiguousarray(v[:nz]) if isinstance(v, np.ndarray) and v.ndim == 3 else v)
              for k, v in pb["state"].items()}
        dt, ns, _ = oracle.suggest_dt(spec, st, pb["chat"])
        t0 = time.perf_counter()
        oracle.step(spec, st, dt, pb["chat"], ns)
        done[r["id"]] = (r["nx"] * r["ny"] * nz * ns, time.perf_counter() - t0)

    el = oracle_threads(one, reqs, threads)
    zu = sum(v[0] for v in done.values())
    return {"value": zu / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"the stream's first {requests} requests, each its first {nz_slab} z-planes "
                      f"as a periodic slab, one gas step with its CFL subcycles, FP64; one "
                      f"request per thread on {threads} threads ({el:.1f} s wall)",
            "per_thread_value": zu / sum(v[1] for v in done.values()), **info}


def cpu_baseline_c2(pb, nz_slab=32):
    """The FP64 oracle (single thread, as it stands) on a bounded sample of the 128^3
    box: its first nz_slab z-planes as a periodic slab, one full gas step with its CFL
    subcycles."""
    import oracle
    import numpy as np
    spec = dict(pb["spec"], nz=nz_slab, precision="fp64")
    st = {k: (np.ascontiguousarray(v[:nz_slab]) if isinstance(v, np.ndarray) else v)
          for k, v in pb["state"].items()}
    dt, ns, _ = oracle.suggest_dt(spec, st, pb["chat"])
    t0 = time.perf_counter()
    oracle.step(spec, st, dt, pb["chat"], ns)
    el = time.perf_counter() - t0
    cells = spec["nx"] * spec["ny"] * spec["nz"]
    return {"value": cells * ns / el, "unit": "zone-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one gas step (exchange, gas VL, {ns} radiation subcycles, correction) on "
                      f"a {spec['nx']}x{spec['ny']}x{nz_slab} periodic slab cut from the same "
                      f"128^3 input, FP64, {el:.1f} s"}


def c3_headline(P, ri, stream, steps, warmup, nsub, tune, graph=False):
    """The concentrated-source grid (256^3): `warmup` untimed steps, then the initial
    state again and `steps` timed steps of `nsub` radiation subcycles each (rhd_step of
    a radiation-only gas step: nsub x [predictor, corrector], then the FP64 ledger),
    bracketed by device synchronisations. A second pass of the same steps with HIP-event
    timing of every launch gives the per-kernel averages."""
    import torch
    pb = ri.c3_point_source(256)
    spec, chat = pb["spec"], pb["chat"]
    dt_gas = pb["dt"] * nsub
    ncell = spec["nx"] * spec["ny"] * spec["nz"]
    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_state(pb["state"])
        if tune:
            tile = s.autotune(chat, pb["dt"], 3) + ("autotune",)
        else:
            tile = (P.RHD_KERNELS_TILED,) + TILE_C3 + ("fixed",)
            s.set_kernel_variant(*tile[:3])
        s.set_graph(graph)
        for _ in range(warmup):
            s.step(dt_gas, chat, nsub)
        s.set_state(pb["state"])
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step(dt_gas, chat, nsub)
        s.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diag = s.diagnostics()
        s.set_state(pb["state"])
        P.rhd_set_timing(s.h, 1)
        for _ in range(steps):
            s.step(dt_gas, chat, nsub)
        s.sync()
        timing = P.rhd_get_timing(s.h)
        P.rhd_set_timing(s.h, 0)
    kernels = kernel_table(timing, spec, True, False)
    rl = roofline(kernels, spec, True, False, pb["name"], tile[1:3])
    sub_bytes = sum(algorithmic_bytes_per_cell(k, spec, True, False) * kernels[k]["cells_per_launch"]
                    for k in ("rad_predict", "rad_correct"))
    sub_us = kernels["rad_predict"]["avg_us"] + kernels["rad_correct"]["avg_us"]
    return {"pb": pb, "elapsed": el, "zone_updates": ncell * nsub * steps, "diag": diag,
            "kernels": kernels, "roofline": rl, "tile": tile,
            "subcycle": {"us": sub_us, "algorithmic_bytes": sub_bytes,
                         "algorithmic_GBps": sub_bytes / (sub_us * 1e-6) / 1e9,
                         "zone_updates_per_s_from_kernels": ncell / (sub_us * 1e-6)}}


def c2_measurement(P, ri, stream, steps=10, warmup=3, precision="mixed", n=128):
    """The coupled operator-split step on the 128^3 periodic linear-perturbation box
    (CFL step with one v_max read per gas step, FP64 exchange, gas Van Leer, 20 radiation
    subcycles, gas source correction, FP64 ledger): `steps` gas steps after `warmup`,
    then a pass with per-kernel HIP-event timing."""
    import torch
    pb = ri.c2_linear_box(n, precision=precision)
    spec, chat = pb["spec"], pb["chat"]
    ncell = spec["nx"] * spec["ny"] * spec["nz"]
    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_state(pb["state"])
        s.set_kernel_variant(P.RHD_KERNELS_TILED, *TILE_C2)

        def one():
            dt, ns = s.suggest_dt(chat)
            s.step(dt, chat, ns)
            return ns

        for _ in range(warmup):
            one()
        s.set_state(pb["state"])
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sub = sum(one() for _ in range(steps))
        s.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diag = s.diagnostics()
        s.set_state(pb["state"])
        P.rhd_set_timing(s.h, 1)
        for _ in range(steps):
            one()
        s.sync()
        timing = P.rhd_get_timing(s.h)
        P.rhd_set_timing(s.h, 0)
    kernels = kernel_table(timing, spec, False, False)
    return {"workload": pb["name"], "grid": [n, n, n], "precision": precision,
            "gas_steps": steps, "subcycles_per_step": sub / steps,
            "value": ncell * sub / el, "unit": "zone-updates/s",
            "gas_step_zone_updates_per_s": ncell * steps / el, "ms_per_gas_step": 1e3 * el / steps,
            "roofline": roofline(kernels, spec, False, False, pb["name"], TILE_C2), "kernels": kernels,
            "kernel_ms_per_step": sum(t["total_ms"] for t in timing.values()) / steps,
            "nonfinite": diag["nonfinite"], "cache_note": "the 128^3 working set (~80 MB) fits "
            "in the 256 MB memory-side cache: its HBM figures are cache-resident"}


def c4_measurement(P, ri, stream, steps, over=20.0):
    """The dusty-shell grid (256^3, isothermal gas, outflow faces, radiative equilibrium,
    lognormal shell and a central source). chat is held fixed through the run (Sec. 3.2),
    at `over` times the largest v_max of a pilot run of the same `steps` gas steps, which
    itself holds chat at `over` times the initial v_max: the source accelerates the gas,
    so v_max grows through the run. The timed run then takes `steps` CFL-limited gas steps
    with nsub = ceil(chat / v_max) subcycles each from the initial state, the state
    resident on the device; one v_max read per gas step."""
    import torch
    pb = ri.c4_dusty_shell(256)
    spec = pb["spec"]
    ncell = spec["nx"] * spec["ny"] * spec["nz"]

    def run(s, chat, record):
        vmax, nsubs = [], []
        for _ in range(steps):
            dt, ns = s.suggest_dt(chat)
            if record:
                vmax.append(s.diagnostics()["vmax"])
            s.step(dt, chat, ns)
            nsubs.append(ns)
        return vmax, nsubs

    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, *TILE_C3)
        s.set_state(pb["state"])
        s.suggest_dt(1.0)
        v0 = s.diagnostics()["vmax"]
        chat0 = over * v0
        t0 = time.perf_counter()
        pilot_v, pilot_n = run(s, chat0, True)
        pilot_s = time.perf_counter() - t0
        chat = over * max(pilot_v)
        s.set_state(pb["state"])
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, nsubs = run(s, chat, False)
        s.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diag = s.diagnostics()
        # the v_max trajectory of the timed run, outside the clock
        s.set_state(pb["state"])
        vmax, _ = run(s, chat, True)
        s.sync()
    sub = sum(nsubs)
    ratio = [chat / v for v in vmax]
    return {"workload": pb["name"], "grid": [spec["nx"], spec["ny"], spec["nz"]],
            "gas_steps": steps, "chat": chat,
            "chat_choice": f"{over:g} x the largest v_max of a {steps}-step pilot run at "
                           f"chat = {over:g} x v_max(t=0) = {chat0:.4g} (pilot: v_max from "
                           f"{pilot_v[0]:.4g} to {max(pilot_v):.4g}, mean nsub "
                           f"{sum(pilot_n) / steps:.1f}, {pilot_s:.1f} s)",
            "subcycles": sub, "subcycles_per_step": sub / steps, "nsub_min": min(nsubs),
            "nsub_max": max(nsubs), "chat_over_vmax_min": min(ratio),
            "chat_over_vmax_max": max(ratio), "value": ncell * sub / el,
            "unit": "zone-updates/s", "gas_step_zone_updates_per_s": ncell * steps / el,
            "elapsed_s": el, "nonfinite": diag["nonfinite"],
            "tile": {"tile_rows": TILE_C3[0], "zchunk": TILE_C3[1]}}


def progress(msg):
    """A progress line on stderr; stdout carries only the result line."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def c5_prepare(count, workers):
    """The seeded perturbations of the served stream's requests, synthesised on `workers`
    processes forked before anything touches the GPU (each request's two random-phase
    fields take up to a second at 192^3)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    import rhd_inputs as ri
    reqs = ri.c5_requests(count=count)
    t0 = time.perf_counter()
    ctx = multiprocessing.get_context("fork")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        pert = dict(zip((r["id"] for r in reqs), ex.map(ri.c5_perturbations, reqs, chunksize=4)))
    return pert, time.perf_counter() - t0


SERVE_MODES = ("one_at_a_time", "native_server", "batched", "concurrent")


def serving(count, load, pert, modes=("one_at_a_time", "native_server"), heavy_load=1.6):
    """The served-batch workload: a stream of independent periodic boxes (32^3..192^3,
    kappa log-uniform in [1, 1e3], chat/a0 in [5, 50], 20 gas steps each). The
    one-at-a-time capacity is measured first with every request queued at t = 0; the
    Poisson arrivals are then scaled so that the offered load is ``load`` times that
    capacity, and the same stream is served in each mode: one at a time (one handle and
    stream per request, in arrival order), through the native server (continuous
    batching over packed tile lists), and, when asked, with the Python batching loops
    (packed tiles, or concurrent per-solve streams). The capacity of each served mode
    (every request queued at t = 0) follows, and the native server serves the stream
    once more at ``heavy_load`` times the one-at-a-time capacity."""
    import rhd_inputs as ri
    from paper_1306_0010_amd import serve

    reqs = ri.c5_requests(count=count, load=load)

    def make(r):
        return ri.c5_problem(r, perturbations=pert[r["id"]], compact=True)

    fns = {"one_at_a_time": lambda rs: serve.serve_serial(rs, make, variant=serve.DEFAULT_VARIANT),
           "native_server": lambda rs: serve.serve_native(rs, make),
           "batched": lambda rs: serve.serve_batched(rs, make),
           "concurrent": lambda rs: serve.serve_concurrent(rs, make,
                                                           variant=serve.DEFAULT_VARIANT)}
    at_zero = [dict(r, arrival=0.0) for r in reqs]
    cap, _ = fns["one_at_a_time"](at_zero)
    service = cap["elapsed_s"] / count
    progress(f"serving: one-at-a-time capacity measured ({cap['elapsed_s']:.1f} s)")
    timed = [dict(r, arrival=r["arrival"] * service) for r in reqs]
    out = {"requests": count, "offered_load": load,
           "one_at_a_time_capacity_requests_per_s": 1.0 / service,
           "total_zone_updates": cap["zone_updates"]}
    for m in modes:
        out[m], _ = fns[m](timed)
        progress(f"serving: {m} stream done ({out[m]['elapsed_s']:.1f} s)")
    base = out["one_at_a_time"]["zone_updates_per_s"] if "one_at_a_time" in out else None
    capacity = {"one_at_a_time": cap["zone_updates_per_s"]}
    for m in modes:
        if m == "one_at_a_time":
            continue
        if base:
            out[f"{m}_over_one_at_a_time_zone_updates"] = out[m]["zone_updates_per_s"] / base
        c, _ = fns[m](at_zero)
        capacity[m] = c["zone_updates_per_s"]
        progress(f"serving: {m} capacity measured ({c['elapsed_s']:.1f} s)")
    out["capacity_zone_updates_per_s"] = capacity
    if "native_server" in modes and heavy_load:
        # the same stream, arriving faster: the native server's latencies nearer its
        # capacity
        faster = [dict(r, arrival=r["arrival"] * load / heavy_load) for r in timed]
        h, _ = fns["native_server"](faster)
        out["native_server_heavier_load"] = dict(h, offered_load=heavy_load)
        progress(f"serving: native_server at {heavy_load:g}x load done ({h['elapsed_s']:.1f} s)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps of the headline (10 radiation subcycles each)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nsub", type=int, default=10,
                    help="radiation subcycles per headline step (default 10)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the served-batch measurement (0 skips it)")
    ap.add_argument("--serve-load", type=float, default=1.2,
                    help="offered load as a multiple of the one-at-a-time capacity")
    ap.add_argument("--serve-modes", default="one_at_a_time,native_server",
                    help="comma-separated served modes: " + ", ".join(SERVE_MODES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-marshak", action="store_true",
                    help="skip the timings of the paper's own test problems (Marshak wave, "
                         "shadow, pulse advection, expanding shell)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the tile shapes by timing the candidates (rhd_autotune) instead "
                         "of the shapes the tuner picked for these grids before")
    ap.add_argument("--c4-steps", type=int, default=100,
                    help="gas steps of the 256^3 dusty-shell measurement (0 skips it)")
    ap.add_argument("--no-c2", action="store_true", help="skip the 128^3 coupled box")
    ap.add_argument("--only", choices=("marshak", "shadow", "pulse", "shell", "c2", "c4", "c5"),
                    help="run only this workload's timing and print its record (for "
                         "profiling one workload)")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: the headline's subcycle loop replays a captured HIP graph")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the headline (no CPU baseline) and print its line")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once "
                         "(device to device): the reference dispatch for scaling hardware "
                         "byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: a run on several GPUs is "
                                   "not implemented (the one-GPU path is --gpus 1)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import rhd_inputs as ri

    # host-only work first, before anything touches the GPU: the oracle baseline of the
    # headline, and the served stream's inputs (synthesised on forked processes)
    only = args.only or args.headline_only
    cpu = None
    if not args.no_cpu_baseline and not only:
        cpu = cpu_baseline_c3(ri)
        progress(f"oracle timed on the headline sample ({cpu['cores']} threads)")
    pert = None
    modes = [m for m in args.serve_modes.split(",") if m]
    for m in modes:
        if m not in SERVE_MODES:
            raise SystemExit(f"unknown served mode {m!r}")
    if args.serve_requests > 0 and (not only or args.only == "c5"):
        pert, el = c5_prepare(args.serve_requests, max(1, min(16, host_info()["usable_cpus"])))
        progress(f"served stream synthesised ({el:.1f} s)")

    import torch

    import paper_1306_0010_amd as P

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.only:
        fn = {"marshak": marshak_timing, "shadow": shadow_timing, "pulse": pulse_timing,
              "shell": shell_timing, "c2": c2_measurement,
              "c4": lambda P_, ri_, st_: c4_measurement(P_, ri_, st_, args.c4_steps),
              "c5": lambda P_, ri_, st_: serving(args.serve_requests, args.serve_load, pert,
                                                 modes)}[args.only]
        print(json.dumps({args.only: fn(P, ri, stream)}), flush=True)
        return

    if args.copy_calibration_mib > 0:
        # two reference dispatches of known size: a device-to-device copy and an
        # elementwise kernel reading one buffer and writing another
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    hl = c3_headline(P, ri, stream, args.steps, args.warmup, args.nsub, args.autotune, args.graph)
    progress(f"headline timed ({hl['elapsed']:.3f} s)")
    pb, tile = hl["pb"], hl["tile"]
    spec = pb["spec"]
    value = hl["zone_updates"] / hl["elapsed"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * hl["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "f32 state and stencils, f64 ledger (no exchange in this workload)",
        "data": "synthetic",
        "config": {"workload": pb["name"], "grid": [spec["nx"], spec["ny"], spec["nz"]],
                   "precision": "mixed", "chat": pb["chat"], "c": spec["c_light"],
                   "kappa_F": 1.2766, "subcycles_per_step": args.nsub,
                   "subcycles_timed": args.nsub * args.steps,
                   "kernels": {"variant": "tiled" if tile[0] == P.RHD_KERNELS_TILED else "other",
                               "tile_rows": tile[1], "zchunk": tile[2], "picked_by": tile[3]}},
        "roofline": hl["roofline"],
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["kernels"] = hl["kernels"]
    out["subcycle"] = hl["subcycle"]
    out["diagnostics"] = {k: hl["diag"][k] for k in ("nonfinite", "rad_fclamp", "rad_efloor")}
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return
    if not args.no_c2:
        out["c2_linear_box"] = c2_measurement(P, ri, stream)
        progress("128^3 coupled box timed")
        out["box_fp64"] = box_fp64_timing(P, ri, stream)
        progress("128^3 box in FP64 timed")
    if args.c4_steps > 0:
        out["c4_dusty_shell"] = c4_measurement(P, ri, stream, args.c4_steps)
        progress("256^3 dusty shell timed")
    if pert is not None:
        out["serving"] = serving(args.serve_requests, args.serve_load, pert, modes)
        if not args.no_cpu_baseline:
            out["serving"]["cpu_baseline"] = cpu_baseline_c5(ri, pert)
            progress("oracle timed on the served stream's sample")
        del pert
    if not args.no_marshak:
        out["marshak"] = marshak_timing(P, ri, stream)
        progress("Marshak wave timed")
        out["shadow"] = shadow_timing(P, ri, stream)
        progress("shadow test timed")
        out["pulse"] = pulse_timing(P, ri, stream)
        progress("pulse advection timed")
        out["shell"] = shell_timing(P, ri, stream)
        progress("expanding shell timed")
    if not args.no_cpu_baseline:
        if not args.no_c2:
            out["c2_linear_box"]["cpu_baseline"] = cpu_baseline_c2(ri.c2_linear_box(128))
        if args.c4_steps > 0:
            out["c4_dusty_shell"]["cpu_baseline"] = cpu_baseline_c4(ri)
        if not args.no_marshak:
            out["marshak"]["cpu_baseline"] = cpu_baseline_marshak(ri)
            out["shadow"]["cpu_baseline"] = cpu_baseline_shadow(ri)
            out["pulse"]["cpu_baseline"] = cpu_baseline_pulse(ri)
            out["shell"]["cpu_baseline"] = cpu_baseline_shell(ri)
        progress("oracle timed on the other workloads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
