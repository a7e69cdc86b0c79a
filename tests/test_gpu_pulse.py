"""GPU parity on the advection of a radiation pulse (Sec. 4.3.2): the coupled 1D
problem (moving optically thick gas, implicit exchange, about 70 radiation subcycles
per gas step) with and without the O(beta tau) terms, against the FP64 oracle step by
step with the oracle's time steps: the whole run to t = 2w/v at 128 cells in FP64, and
the first 30 gas steps in mixed precision.

Tolerances as in test_gpu_parity.py: FP64 max-norm 1e-12, mixed precision L1 1e-5."""
import sys

import numpy as np
import pytest

import oracle
import paper_1306_0010_amd as P
import rhd_inputs as ri
from parity import assert_parity

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
NORM = {"fp64": "max", "mixed": "l1"}


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("beta_tau", [True, False])
def test_pulse_advection_matches_oracle(beta_tau, precision):
    announce(f"pulse advection beta_tau={beta_tau} {precision}")
    pb = ri.pulse_problem(128, advected=True, beta_tau=beta_tau, precision=precision)
    spec, chat = pb["spec"], pb["chat"]
    ref = pb["state"]
    max_steps = 10 ** 6 if precision == "fp64" else 30
    t, steps = 0.0, 0
    with P.Solver(spec) as s:
        s.set_state(ref)
        while t < pb["t_end"] * (1.0 - 1e-12) and steps < max_steps:
            dt, ns, _ = oracle.suggest_dt(spec, ref, chat)
            dt = min(dt, pb["t_end"] - t)
            s.step(dt, chat, ns)
            ref, _ = oracle.step(spec, ref, dt, chat, ns)
            t += dt
            steps += 1
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0 and diag["steps"] == steps
    assert diag["newton_iters"] > 0
    if precision == "fp64":
        assert t == pytest.approx(pb["t_end"], rel=1e-12) and steps > 200
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision],
                  label=f"pulse beta_tau={beta_tau} {precision}")
