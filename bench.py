#!/usr/bin/env python3
"""Throughput of the operator-split gray M1 radiation-hydrodynamics step on one MI355X.

One benchmark step is one pass of the whole hot path on the 128^3 periodic
linear-perturbation box (rho = P = E_r = 1, kappa = 10, chat = 20 a0, c = 1e4 a0,
seeded random-phase perturbations of RMS 1e-4), mixed precision:
  radiation-modified CFL time step (synchronises once to read v_max)
  -> FP64 implicit energy exchange -> gas Van Leer predictor and corrector
  -> nsub (= 20 here) radiation Van Leer subcycles -> second-order gas source
  correction -> FP64 ledger with non-finite check.
The state stays resident in HBM; nothing is copied to the host inside the timed
region except the one v_max value per step.

Prints one JSON line: the radiation zone-update rate (cells x subcycles per second),
the roofline of the dominant kernel from HIP-event timings of its launches inside the
timed region (against the FP32 VALU roof, which bounds it, with its algorithmic HBM
bandwidth beside it), the same for 200 subcycles of the 256^3 concentrated-source grid,
full gas steps of the 256^3 dusty shell, the served-batch latencies, and the FP64 CPU oracle timed on a bounded sample of the
same input.
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
KERNEL_SOURCES = ("paper_1306_0010_amd/csrc/rhd_device.hpp", "paper_1306_0010_amd/csrc/rhd_tile.hpp")
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic.json")
# tile shapes (rows, z chunk) that rhd_autotune picked for the two grids on MI355X
TILE_C2 = (8, 8)
TILE_C3 = (8, 16)


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


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed hardware-counter record, if it was taken
    on the kernel sources as they are now; None otherwise."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    entry = rec.get("kernels", {}).get(workload, {}).get(kernel)
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


def roofline(kernels, spec, has_j, kappa_field, workload):
    """The dominant kernel against the FP32 VALU roof (it is bound by arithmetic), with
    its algorithmic HBM bandwidth beside it."""
    rad = {k: v for k, v in kernels.items() if k.startswith("rad_")}
    dom = max(rad, key=lambda k: rad[k]["share"])
    k = rad[dom]
    bpc = algorithmic_bytes_per_cell(dom, spec, has_j, kappa_field)
    traffic = measured_traffic(dom, workload)
    return {"bound": "alu", "achieved": k["algorithmic_Tslots_per_s"], "peak": VALU_PEAK_TSLOTS,
            "unit": "TFLOP/s", "frac": k["algorithmic_Tslots_per_s"] / VALU_PEAK_TSLOTS,
            "traffic": traffic, "kernel": dom, "avg_us": k["avg_us"],
            "slots_per_cell": k["slots_per_cell"], "cells_per_launch": k["cells_per_launch"],
            "unit_note": "FP32 VALU lane slots (non-packed; reciprocal/square root = 2)",
            "hbm_algorithmic": {"achieved_GBps": k["algorithmic_GBps"], "peak_GBps": HBM_PEAK_GBS,
                                "frac": k["algorithmic_GBps"] / HBM_PEAK_GBS,
                                "bytes_per_cell": bpc}}


MARSHAK_N = (32, 128, 512, 2048)
MARSHAK_TAU = (1.0, 10.0, 100.0)


def marshak_schedule(ri, n, tau_end):
    """Steps and face states of the Marshak problem (Sec. 4.2.3, eps = 1, chi in
    [0, 100]) on n cells up to tau_end: the boundary states are inputs, computed before
    any clock starts."""
    pb = ri.marshak_problem(n)
    dt = pb["dt"]
    steps = int(math.ceil(tau_end / dt - 1e-9))
    hs = [min(dt, tau_end - k * dt) for k in range(steps)]
    bvals = [ri.marshak_boundary(k * dt + 0.5 * hs[k]) for k in range(steps)]
    return pb, hs, bvals


def marshak_timing(P, ri, stream):
    """The paper's own timing benchmark (Sec. 4.3): wall time of the 1D Marshak wave to
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
    """The advection of a radiation pulse (Sec. 4.2.5) at the paper's 512 cells to
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
    """The expanding-shell test of Sec. 4.4.2 at the paper's 128^3 octant to t = 0.124
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
    """The shadow test of Sec. 4.2.1 at the paper's 280 x 80 cells for 10 horizontal
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


def cpu_baseline(pb, nz_slab=32):
    """The FP64 oracle (single thread, as it stands) on a bounded sample of the same
    input: the first nz_slab z-planes of the 128^3 box as a periodic slab, one full
    gas step with its CFL subcycles."""
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


def c3_measurement(P, ri, stream, subcycles, tune):
    """The concentrated-source grid (256^3, outflow, static gas with a Gaussian core,
    central emitting cells, chat = c = 1): one call of `subcycles` radiation subcycles
    with the state resident on the device, per-kernel HIP-event timing inside it."""
    import torch
    pb = ri.c3_point_source(256)
    spec, chat = pb["spec"], pb["chat"]
    dt_rad = pb["dt"]
    ncell = spec["nx"] * spec["ny"] * spec["nz"]
    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_state(pb["state"])
        if tune:
            tile = s.autotune(chat, dt_rad, 3) + ("autotune",)
        else:
            tile = (P.RHD_KERNELS_TILED,) + TILE_C3 + ("fixed",)
            s.set_kernel_variant(*tile[:3])
        s.step(dt_rad * 4, chat, 4)  # warm-up
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(dt_rad * subcycles, chat, subcycles)
        s.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diag = s.diagnostics()
        # per-kernel HIP-event timing in a pass of its own
        P.rhd_set_timing(s.h, 1)
        nt = min(subcycles, 50)
        s.step(dt_rad * nt, chat, nt)
        s.sync()
        timing = P.rhd_get_timing(s.h)
    kernels = kernel_table(timing, spec, True, False)
    out = {"workload": pb["name"], "grid": [spec["nx"], spec["ny"], spec["nz"]],
           "subcycles": subcycles, "value": ncell * subcycles / el, "unit": "zone-updates/s",
           "elapsed_s": el, "roofline": roofline(kernels, spec, True, False, pb["name"]),
           "kernels": {k: v for k, v in kernels.items() if k.startswith("rad_")},
           "nonfinite": diag["nonfinite"]}
    out["kernels_choice"] = {"tile_rows": tile[1], "zchunk": tile[2], "picked_by": tile[3]}
    return out


def c4_measurement(P, ri, stream, steps):
    """The dusty-shell grid (256^3, isothermal gas, outflow faces, radiative equilibrium,
    lognormal shell and a central source, chat = 20 v_max at t = 0): `steps` full gas
    steps with CFL-limited subcycles, the state resident on the device."""
    import torch
    pb = ri.c4_dusty_shell(256)
    spec = pb["spec"]
    ncell = spec["nx"] * spec["ny"] * spec["nz"]
    with P.Solver(spec, stream=stream.cuda_stream) as s:
        s.set_state(pb["state"])
        s.suggest_dt(1.0)
        chat = pb["chat_over_vmax"] * s.diagnostics()["vmax"]
        s.set_kernel_variant(P.RHD_KERNELS_TILED, *TILE_C3)
        dt, ns = s.suggest_dt(chat)
        s.step(dt, chat, ns)  # warm-up step
        s.sync()
        torch.cuda.synchronize()
        sub = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            dt, ns = s.suggest_dt(chat)
            s.step(dt, chat, ns)
            sub += ns
        s.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        diag = s.diagnostics()
    return {"workload": pb["name"], "grid": [spec["nx"], spec["ny"], spec["nz"]], "gas_steps": steps,
            "subcycles_per_step": sub / steps, "chat": chat, "value": ncell * sub / el,
            "unit": "zone-updates/s", "gas_step_zone_updates_per_s": ncell * steps / el,
            "elapsed_s": el, "nonfinite": diag["nonfinite"],
            "tile": {"tile_rows": TILE_C3[0], "zchunk": TILE_C3[1]}}


def progress(msg):
    """A progress line on stderr; stdout carries only the result line."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serving(count, load):
    """The served-batch workload: a stream of independent periodic boxes (32^3..192^3,
    kappa log-uniform in [1, 1e3], chat/a0 in [5, 50], 20 gas steps each). The
    one-at-a-time capacity is measured first with every request queued at t = 0; the
    Poisson arrivals are then scaled so that the offered load is ``load`` times that
    capacity, and the same stream is served with packed-tile batching, with concurrent
    per-solve streams, through the native server and one at a time. The capacity of each
    mode (all requests queued at t = 0) closes the measurement."""
    import rhd_inputs as ri
    from paper_1306_0010_amd import serve

    reqs = ri.c5_requests(count=count, load=load)
    problems = {}  # each request's initial state is synthesised once and reused

    def make(r):
        if r["id"] not in problems:
            problems[r["id"]] = ri.c5_problem(r)
        return problems[r["id"]]

    at_zero = [dict(r, arrival=0.0) for r in reqs]
    cap, _ = serve.serve_serial(at_zero, make, variant=serve.DEFAULT_VARIANT)
    service = cap["elapsed_s"] / count
    progress(f"serving: one-at-a-time capacity measured ({cap['elapsed_s']:.1f} s)")
    timed = [dict(r, arrival=r["arrival"] * service) for r in reqs]
    batched, _ = serve.serve_batched(timed, make)
    progress("serving: batched stream done")
    concurrent, _ = serve.serve_concurrent(timed, make, variant=serve.DEFAULT_VARIANT)
    progress("serving: concurrent stream done")
    native, _ = serve.serve_native(timed, make)
    progress("serving: native-server stream done")
    serial, _ = serve.serve_serial(timed, make, variant=serve.DEFAULT_VARIANT)
    progress("serving: one-at-a-time stream done")
    # capacity: every request queued at t = 0
    cap_b, _ = serve.serve_batched(at_zero, make)
    cap_c, _ = serve.serve_concurrent(at_zero, make, variant=serve.DEFAULT_VARIANT)
    cap_n, _ = serve.serve_native(at_zero, make)
    progress("serving: capacities measured")
    capacity = {m: c["zone_updates_per_s"] for m, c in
                (("batched", cap_b), ("concurrent", cap_c), ("native_server", cap_n),
                 ("one_at_a_time", cap))}
    return {"requests": count, "offered_load": load,
            "one_at_a_time_capacity_requests_per_s": 1.0 / service,
            "batched": batched, "concurrent": concurrent, "native_server": native,
            "one_at_a_time": serial,
            "batched_over_one_at_a_time_zone_updates": batched["zone_updates_per_s"]
            / serial["zone_updates_per_s"],
            "concurrent_over_one_at_a_time_zone_updates": concurrent["zone_updates_per_s"]
            / serial["zone_updates_per_s"],
            "native_server_over_one_at_a_time_zone_updates": native["zone_updates_per_s"]
            / serial["zone_updates_per_s"],
            "capacity_zone_updates_per_s": capacity}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed")
    ap.add_argument("--n", type=int, default=128, help="grid side of the box (default 128)")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests in the served-batch measurement (0 skips it; 512 is the "
                         "full stream)")
    ap.add_argument("--serve-load", type=float, default=1.2,
                    help="offered load as a multiple of the one-at-a-time capacity")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-marshak", action="store_true",
                    help="skip the timings of the paper's own test problems (Marshak wave, "
                         "shadow, pulse advection, expanding shell)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the tile shapes by timing the candidates (rhd_autotune) instead "
                         "of the shapes the tuner picked for these grids before")
    ap.add_argument("--c3-subcycles", type=int, default=200,
                    help="radiation subcycles of the 256^3 point-source measurement (0 skips it)")
    ap.add_argument("--c4-steps", type=int, default=5,
                    help="gas steps of the 256^3 dusty-shell measurement (0 skips it)")
    ap.add_argument("--only", choices=("marshak", "shadow", "pulse", "shell"),
                    help="run only this test problem's timing and print its record (for "
                         "profiling one workload)")
    ap.add_argument("--c3-only", action="store_true",
                    help="run only the 256^3 point-source measurement and print its line")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once "
                         "(device to device): the reference dispatch for scaling hardware "
                         "byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: a multi-GPU run is not "
                                   "implemented (the one-GPU path is --gpus 1)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1306_0010_amd as P
    import rhd_inputs as ri

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.only:
        fn = {"marshak": marshak_timing, "shadow": shadow_timing, "pulse": pulse_timing,
              "shell": shell_timing}[args.only]
        print(json.dumps({args.only: fn(P, ri, stream)}), flush=True)
        return

    if args.c3_only:
        print(json.dumps(c3_measurement(P, ri, stream, max(1, args.c3_subcycles),
                                        args.autotune)), flush=True)
        return

    pb = ri.c2_linear_box(args.n, precision=args.precision)
    spec, chat = pb["spec"], pb["chat"]
    ncell = spec["nx"] * spec["ny"] * spec["nz"]
    solver = P.Solver(spec, stream=stream.cuda_stream)
    solver.set_state(pb["state"])
    h = solver.h

    def one_step():
        dt, ns = solver.suggest_dt(chat)
        solver.step(dt, chat, ns)
        return ns

    if args.autotune:
        dt0, ns0 = solver.suggest_dt(chat)
        tile = solver.autotune(chat, dt0 / ns0, 3) + ("autotune",)
    else:
        tile = (P.RHD_KERNELS_TILED,) + TILE_C2 + ("fixed",)
        solver.set_kernel_variant(*tile[:3])

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

    for _ in range(args.warmup):
        one_step()
    solver.sync()
    torch.cuda.synchronize()

    subcycles = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        subcycles += one_step()
    torch.cuda.synchronize()
    solver.sync()
    elapsed = time.perf_counter() - t0
    diag = solver.diagnostics()
    timing = {}
    if not args.no_kernel_timing:
        # per-kernel HIP-event timing in a pass of its own, so that the event records
        # do not sit between the kernels of the timed region
        P.rhd_set_timing(h, 1)
        for _ in range(args.steps):
            one_step()
        solver.sync()
        timing = P.rhd_get_timing(h)
        P.rhd_set_timing(h, 0)
    solver.close()
    progress(f"headline workload timed ({elapsed:.2f} s)")

    value = ncell * subcycles / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64",
        "dtype_detail": ("f32 state and stencils, f64 energy exchange and ledger"
                         if args.precision == "mixed" else "f64 throughout"),
        "data": "synthetic",
        "config": {"workload": pb["name"], "grid": [spec["nx"], spec["ny"], spec["nz"]],
                   "precision": args.precision, "chat": chat, "c": spec["c_light"],
                   "kappa": 10.0, "subcycles_per_step": subcycles / args.steps,
                   "gas_step_zone_updates_per_s": ncell * args.steps / elapsed},
    }

    out["config"]["kernels"] = {"variant": "tiled" if tile[0] == P.RHD_KERNELS_TILED else "per_cell",
                                "tile_rows": tile[1], "zchunk": tile[2], "picked_by": tile[3]}
    if timing:
        kernels = kernel_table(timing, spec, False, False)
        out["roofline"] = roofline(kernels, spec, False, False, pb["name"])
        out["kernels"] = kernels
        out["kernel_ms_per_step"] = sum(t["total_ms"] for t in timing.values()) / args.steps

    if args.precision == "mixed" and args.n == 128:
        out["box_fp64"] = box_fp64_timing(P, ri, stream)
        progress("FP64 box timed")

    out["diagnostics"] = {k: diag[k] for k in ("nonfinite", "rad_fclamp", "rad_efloor",
                                               "gas_rhofloor", "gas_pfloor", "exch_theta1",
                                               "exch_bisect", "newton_max")}
    if args.c3_subcycles > 0 and args.precision == "mixed":
        out["c3_point_source"] = c3_measurement(P, ri, stream, args.c3_subcycles, args.autotune)
        progress("256^3 point source timed")
    if args.c4_steps > 0 and args.precision == "mixed":
        out["c4_dusty_shell"] = c4_measurement(P, ri, stream, args.c4_steps)
        progress("256^3 dusty shell timed")
    if args.serve_requests > 0:
        out["serving"] = serving(args.serve_requests, args.serve_load)
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
        out["cpu_baseline"] = cpu_baseline(pb)
        progress("oracle timed on the host")
        if not args.no_marshak:
            out["marshak"]["cpu_baseline"] = cpu_baseline_marshak(ri)
            out["shadow"]["cpu_baseline"] = cpu_baseline_shadow(ri)
            out["pulse"]["cpu_baseline"] = cpu_baseline_pulse(ri)
            out["shell"]["cpu_baseline"] = cpu_baseline_shell(ri)
            progress("oracle timed on the Marshak wave, the shadow, pulse and shell tests")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
