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
timed region, and the FP64 CPU oracle timed on a bounded sample of the same input.
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


def cpu_baseline(pb, nz_slab=16):
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


def serving(count, load):
    """The served-batch workload: a stream of independent periodic boxes (32^3..192^3,
    kappa log-uniform in [1, 1e3], chat/a0 in [5, 50], 20 gas steps each). The
    one-at-a-time capacity is measured first with every request queued at t = 0; the
    Poisson arrivals are then scaled so that the offered load is ``load`` times that
    capacity, and the same stream is served with continuous batching and one at a time."""
    import rhd_inputs as ri
    from paper_1306_0010_amd import serve

    reqs = ri.c5_requests(count=count, load=load)
    make = lambda r: ri.c5_problem(r)
    at_zero = [dict(r, arrival=0.0) for r in reqs]
    cap, _ = serve.serve_serial(at_zero, make, variant=serve.DEFAULT_VARIANT)
    service = cap["elapsed_s"] / count
    timed = [dict(r, arrival=r["arrival"] * service) for r in reqs]
    batched, _ = serve.serve_batched(timed, make)
    serial, _ = serve.serve_serial(timed, make, variant=serve.DEFAULT_VARIANT)
    return {"requests": count, "offered_load": load,
            "one_at_a_time_capacity_requests_per_s": 1.0 / service,
            "batched": batched, "one_at_a_time": serial,
            "batched_over_one_at_a_time_zone_updates": batched["zone_updates_per_s"]
            / serial["zone_updates_per_s"]}


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
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before the timed region, copy a buffer of this many MiB once "
                         "(device to device): the reference dispatch for scaling hardware "
                         "byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: a multi-GPU run is not "
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

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        one_step()
    solver.sync()
    torch.cuda.synchronize()

    if not args.no_kernel_timing:
        P.rhd_set_timing(h, 1)
    subcycles = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        subcycles += one_step()
    torch.cuda.synchronize()
    solver.sync()
    elapsed = time.perf_counter() - t0
    timing = P.rhd_get_timing(h) if not args.no_kernel_timing else {}
    diag = solver.diagnostics()
    solver.close()

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

    if timing:
        kernels = {}
        for name, t in timing.items():
            if t["calls"] == 0:
                continue
            avg_ms = t["total_ms"] / t["calls"]
            b = algorithmic_bytes_per_cell(name, spec, False, False) * t["cells"]
            kernels[name] = {"calls": t["calls"], "avg_us": 1e3 * avg_ms,
                             "share": t["total_ms"] / max(1e-30, sum(v["total_ms"] for v in timing.values())),
                             "algorithmic_GBps": b / (avg_ms * 1e-3) / 1e9}
        dom = max(kernels, key=lambda k: kernels[k]["share"])
        achieved = kernels[dom]["algorithmic_GBps"]
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "kernel": dom, "avg_us": kernels[dom]["avg_us"],
                           "bytes_per_cell": algorithmic_bytes_per_cell(dom, spec, False, False)}
        out["kernels"] = kernels
        out["gpu_time_share_ms_per_step"] = sum(t["total_ms"] for t in timing.values()) / args.steps

    out["diagnostics"] = {k: diag[k] for k in ("nonfinite", "rad_fclamp", "rad_efloor",
                                               "gas_rhofloor", "gas_pfloor", "exch_theta1",
                                               "exch_bisect", "newton_max")}
    if args.serve_requests > 0:
        out["serving"] = serving(args.serve_requests, args.serve_load)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
