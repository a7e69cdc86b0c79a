"""GPU checks on the expanding-shell test of Sec. 4.3.6 (octant, reflecting and outflow
faces, isothermal gas, central source, equilibrium M1 field): parity with the FP64
oracle over the first coupled gas steps at 32^3; at the paper's 128^3, the radiation-only
run holds the equilibrium field (as the paper reports), and the coupled run follows the
shell trajectory within the paper's errors (3.1 % in <r>, 7.0 % in <v_r> at
chat/a0 = 860; 5.3 % and 13 % at 430), with the error growing as chat falls.

Tolerances as in test_gpu_parity.py: FP64 max-norm 1e-12, mixed precision L1 1e-5."""
import sys
import time

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


# Near the source the flux is clamped to |F| = c E_r in 250-480 cell-stages per gas step;
# at that branch point of the closure FP64 results agree to ~sqrt(eps) times the
# dissipation share of the HLL flux (1.5e-11 seen), as for the dusty shell.
FP64_TOL_CLAMPED = 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shell_matches_oracle_at_32(precision):
    announce(f"shell 32^3 {precision}")
    pb = ri.shell_expansion_problem(32, precision=precision)
    spec, chat = pb["spec"], pb["chat"]
    ref = pb["state"]
    clamps = 0
    with P.Solver(spec) as s:
        s.set_state(ref)
        for _ in range(3):
            dt, ns, _ = oracle.suggest_dt(spec, ref, chat)
            s.step(dt, chat, ns)
            ref, cnt = oracle.step(spec, ref, dt, chat, ns)
            clamps += cnt["rad_fclamp"]
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0 and clamps > 0
    tol = FP64_TOL_CLAMPED if precision == "fp64" else TOL[precision]
    assert_parity(spec, gpu, ref, tol, NORM[precision], label=f"shell 32 {precision}")


def run_shell(n, chat_over_a0, every=0.005):
    """The coupled run to t = 0.124 with (t, <r>, <v_r>) every `every`."""
    pb = ri.shell_expansion_problem(n, chat_over_a0=chat_over_a0, precision="mixed")
    spec = pb["spec"]
    samples = [(0.0,) + ri.shell_moments(spec, pb["state"], pb["r"])]
    with P.Solver(spec) as s:
        s.set_state(pb["state"])
        t, nxt = 0.0, every
        while t < pb["t_end"] * (1 - 1e-12):
            dt, ns = s.suggest_dt(pb["chat"])
            dt = min(dt, nxt - t)
            s.step(dt, pb["chat"], ns)
            t += dt
            if t >= nxt * (1 - 1e-12):
                samples.append((t,) + ri.shell_moments(spec, s.get_state(), pb["r"]))
                nxt = min(nxt + every, pb["t_end"])
        diag = s.diagnostics()
    assert diag["nonfinite"] == 0
    return pb, samples


def test_shell_follows_the_trajectory_within_the_papers_errors():
    announce("shell 128^3 expansion")
    err = {}
    for chat in (860.0, 430.0):
        pb, samples = run_shell(128, chat)
        err[chat] = ri.shell_errors(pb["M0"], samples)
        assert samples[-1][1] == pytest.approx(2.0, rel=0.06)
    # the paper: 3.1 % and 7.0 % at 860, 5.3 % and 13 % at 430 (10 % slack)
    assert err[860.0][0] < 1.1 * 0.031 and err[860.0][1] < 1.1 * 0.070, err
    assert err[430.0][0] < 1.1 * 0.053 and err[430.0][1] < 1.1 * 0.13, err
    assert err[430.0][0] > err[860.0][0] and err[430.0][1] > err[860.0][1]


def test_radiation_only_run_holds_the_equilibrium_field():
    """Gas frozen, 1500 subcycles (about nine light-crossings of r0): the shell averages
    of E_r and F_r stay within 1.5 % and 3 % of the initial M1 equilibrium between
    r = 0.4 and 2 (inside 0.3 the initial field near the source is a reading, not a
    solution of the ODE)."""
    announce("shell 128^3 radiation only")
    pb = ri.shell_expansion_problem(128, precision="mixed", rad_only=True)
    spec, r, chat = pb["spec"], pb["r"], pb["chat"]
    dt = 0.4 * spec["dx"] / chat
    with P.Solver(spec) as s:
        s.set_state(pb["state"])
        s.run(np.full(1500, dt), np.ones(1500, dtype=np.int32), chat)
        s.sync()
        st, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    X, Y, Z = ri.cell_centres(spec)
    Fr = (st["Fx"] * X + st["Fy"] * Y + st["Fz"] * Z) / r
    bins = np.linspace(0.4, 2.0, 33)
    idx = np.digitize(r, bins)
    E0, F0 = pb["state"]["Er"], pb["profile"].F(r)
    for b in range(1, len(bins)):
        m = idx == b
        assert abs(st["Er"][m].mean() / E0[m].mean() - 1.0) < 0.015, bins[b]
        assert abs(Fr[m].mean() / F0[m].mean() - 1.0) < 0.03, bins[b]
