"""The 3D linear-perturbation box judged in perturbation space (Sec. 4.3.4).

Its perturbations are 1e-4 of a uniform background, so errors stated against the
background (the bar of the other parity tests) say little about them. Here:

- GPU against the FP64 oracle on the same recipe at 32^3, 10 CFL gas steps of 20
  subcycles, each field's error measured against the field's own departure from the
  background: sum |d_gpu - d_oracle| / sum |d_oracle| for d = rho - 1, E_r - 1,
  E - E(0) (gas energy), and the momentum and the radiation flux against their own
  magnitudes (both vanish in the background).
  Mixed precision: FP32 stores rho = 1 + 1e-4 x to a spacing of 1.2e-7, i.e. 6e-8
  rounding, which is 6e-4 of a perturbation of 1e-4. Over ~400 stages of rounding a
  random walk grows to sqrt(400) x 6e-4 ~ 1.2e-2: the bar is 2e-2 for rho, E and the
  momentum. E_r is another matter: the stiff exchange (eta = c rho kappa dt ~ 1e3 per
  gas step) locks the gas temperature to the radiation, whose share of E + (c/chat) E_r
  is 500 times the gas's, so after a few steps E_r departs from 1 by at most ~3e-7, a
  few FP32 spacings at 1 (1.2e-7). Mixed precision cannot resolve that perturbation.
  E_r then follows a_R T^4 of the gas, whose T comes from the FP32-stored rho and E
  (each rounded to half a spacing, relative), and the fourth power multiplies their
  relative rounding by four: E_r is held to 16 spacings at the background (max norm),
  and F, which follows the E_r gradient, to 4 spacings of c E_r. FP64 mode resolves
  both: it is held to 1e-7 of every field's perturbation.
- GPU at the full 128^3 (the bench's run) against the linear theory mode by mode: the
  Fourier coefficients of rho - 1 and E_r - 1 for every |n| <= 3 after 10 gas steps
  against exp(A(k) t) applied to the initial coefficients, A the 5x5 linear system
  derived from Eq. mixedframe:graysystem. The difference left is the scheme's
  truncation error and FP32 rounding: per Fourier coefficient (normalised by the cell
  count) the rounding is ~6e-8/sqrt(2e6) per store, ~1e-9 after 400 stores, against mode
  amplitudes of ~3e-6 (1e-4 RMS over ~2000 modes): ~3e-4. The truncation error is
  ~(k dx)^2 times the phase the mode turns through, k dx <= 0.15 and the phase <= 0.6
  rad here: ~1e-3 at |n| = 3. Bars: 2e-3 of a mode's initial amplitude for |n| <= 2,
  3e-3 for |n| = 3.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1306_0010_amd as P
import rhd_inputs as ri
from linear_rhd import c2_mode_prediction

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def perturbation_errors(gpu, ref, base):
    """{field: sum |gpu - ref| / sum |ref - base|} with base the background value (a
    number, or 0 for fields that vanish in the background)."""
    out = {}
    for k, b in base.items():
        g = np.asarray(gpu[k], dtype=np.float64)
        r = np.asarray(ref[k], dtype=np.float64)
        out[k] = float(np.abs(g - r).sum() / np.abs(r - b).sum())
    return out


FP32_SPACING_AT_1 = 2.0 ** -23


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_linear_box_32_perturbation_space_parity(precision):
    announce(f"linear box 32^3 perturbation space {precision}")
    pb = ri.c2_linear_box(32, precision=precision)
    spec, st0, chat = pb["spec"], pb["state"], pb["chat"]
    spec64 = dict(spec, precision="fp64")
    st, steps = st0, []
    for _ in range(10):
        dt, ns, _ = oracle.suggest_dt(spec64, st, chat)
        st, _ = oracle.step(spec64, st, dt, chat, ns)
        steps.append((dt, ns))
    ref = st
    with P.Solver(spec) as s:
        s.set_state(st0)
        for dt, ns in steps:
            s.step(dt, chat, ns)
        s.sync()
        gpu = s.get_state()
        diag = s.diagnostics()
    assert diag["nonfinite"] == 0
    E0 = float(st0["E"].flat[0])
    base = {"rho": 1.0, "Er": 1.0, "E": E0, "mx": 0.0, "my": 0.0, "mz": 0.0,
            "Fx": 0.0, "Fy": 0.0, "Fz": 0.0}
    err = perturbation_errors(gpu, ref, base)
    print("perturbation-space L1 errors:", {k: f"{v:.2e}" for k, v in err.items()})
    # the run moves the perturbations by far more than the bars: the check is not vacuous
    moved = float(np.abs(ref["rho"] - st0["rho"]).sum() / np.abs(st0["rho"] - 1.0).sum())
    assert moved > 0.1, moved
    if precision == "fp64":
        assert max(err.values()) < 1e-7, err
        return
    for k in ("rho", "E", "mx", "my", "mz"):
        assert err[k] < 2e-2, err
    dEr = float(np.abs(gpu["Er"] - ref["Er"]).max())
    cE = spec["c_light"] * float(np.abs(ref["Er"]).max())
    dF = max(float(np.abs(gpu[k] - ref[k]).max()) for k in ("Fx", "Fy", "Fz"))
    pert_Er = float(np.abs(ref["Er"] - 1.0).max())
    print(f"E_r: perturbation {pert_Er:.2e}, max error {dEr:.2e}; F: max error {dF / cE:.2e} of c E_r")
    assert pert_Er < 4 * FP32_SPACING_AT_1, pert_Er  # why mixed mode cannot resolve it
    assert dEr <= 16 * FP32_SPACING_AT_1, dEr
    assert dF <= 4 * FP32_SPACING_AT_1 * cE, dF


def test_linear_box_128_modes_follow_linear_theory():
    announce("linear box 128^3 modes vs linear theory")
    pb = ri.c2_linear_box(128, precision="mixed")
    spec, st0, chat = pb["spec"], pb["state"], pb["chat"]
    t = 0.0
    with P.Solver(spec) as s:
        s.set_state(st0)
        for _ in range(pb["steps"]):
            dt, ns = s.suggest_dt(chat)
            s.step(dt, chat, ns)
            t += dt
        s.sync()
        st = s.get_state()
    n = spec["nx"]
    R0, E0 = np.fft.fftn(st0["rho"] - 1.0), np.fft.fftn(st0["Er"] - 1.0)
    R1, E1 = np.fft.fftn(st["rho"] - 1.0), np.fft.fftn(st["Er"] - 1.0)
    worst, moved = {1: 0.0, 2: 0.0, 3: 0.0}, 0.0
    for kz in range(-3, 4):
        for ky in range(-3, 4):
            for kx in range(0, 4):
                kk = math.sqrt(kx * kx + ky * ky + kz * kz)
                if kk < 1 or kk > 3:
                    continue
                i = (kz % n, ky % n, kx % n)
                pr, pe = c2_mode_prediction(spec, chat, 10.0, t, R0[i], E0[i], (kx, ky, kz))
                amp = abs(R0[i]) + abs(E0[i])
                e = max(abs(R1[i] - pr), abs(E1[i] - pe)) / amp
                shell = 1 if kk < 1.5 else (2 if kk <= 2.0 + 1e-9 else 3)
                worst[shell] = max(worst[shell], e)
                moved = max(moved, max(abs(pr - R0[i]), abs(pe - E0[i])) / amp)
    print("largest mode errors by |n| shell:", {k: f"{v:.2e}" for k, v in worst.items()},
          f"largest change {moved:.2e}")
    assert worst[1] < 2e-3 and worst[2] < 2e-3 and worst[3] < 3e-3, worst
    assert moved > 10 * worst[1], (moved, worst)
