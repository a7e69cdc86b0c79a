"""GPU parity for the Eddington (P1) closure (Sec. 2.3; T = I/3, speeds -+chat/sqrt(3)):
every kernel path against the FP64 oracle with the same flag: the one-workgroup 1D path
on a large-amplitude pulse, the per-cell kernels on a 2D radiation-only state, the tiled
kernels on a 3D coupled state with moving gas, and a batch holding an M1 and a P1
member, each equal to its lone handle.

Tolerances as in test_gpu_parity.py: FP64 max-norm 1e-12, mixed precision L1 1e-5."""
import math
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
def test_p1_pulse_on_the_fused_1d_path(precision):
    """A pulse of amplitude 10 (f up to ~0.5) on 512 periodic cells with a scattering
    opacity, 300 steps in one rhd_run call (one-workgroup path)."""
    announce(f"p1 pulse 1d {precision}")
    n = 512
    spec = ri.default_spec(nx=n, dx=1.0 / n, c_light=1.0, exchange="none", rad_only=True,
                           theta_F=0.51, bc="periodic", closure="p1", precision=precision)
    st = ri.uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=0.0, kF=5.0)
    x = (np.arange(n) + 0.5) / n
    st["Er"][0, 0, :] = 1.0 + 10.0 * np.exp(-((x - 0.5) ** 2) / (2 * 0.05 ** 2))
    dt, steps = 0.4 / n, 300
    ref, _ = oracle.step(spec, st, dt, 1.0, 1, steps=steps)
    with P.Solver(spec) as s:
        s.set_state(st)
        s.run(np.full(steps, dt), np.ones(steps, dtype=np.int32), 1.0)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0 and diag["steps"] == steps
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"p1 1d {precision}")
    # the same run with the M1 closure ends far from it (0.84 at the pulse)
    ref_m1, _ = oracle.step(dict(spec, closure="m1"), st, dt, 1.0, 1, steps=steps)
    assert np.abs(ref_m1["Er"] - gpu["Er"]).max() > 0.1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_p1_per_cell_kernels_2d(precision):
    announce(f"p1 per-cell 2d {precision}")
    spec = ri.default_spec(nx=40, ny=27, dx=1 / 40, dy=1 / 27, c_light=20.0, rad_only=True,
                           exchange="full", theta_E=0.6, theta_F=0.51,
                           bc=("outflow", "reflect", "periodic", "periodic", "periodic",
                               "periodic"), closure="p1", precision=precision)
    st = ri.smooth_random_state(spec, seed=41, amp=0.2, f_amp=0.5, kappa=(3.0, 2.0), v_amp=0.0)
    dt = 0.35 / (spec["c_light"] * 40)
    ref, _ = oracle.step(spec, st, dt, spec["c_light"], 1, steps=4)
    with P.Solver(spec) as s:
        s.set_state(st)
        s.run(np.full(4, dt), np.ones(4, dtype=np.int32), spec["c_light"])
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"p1 2d {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_p1_tiled_kernels_3d_coupled(precision):
    """A 3D ideal-gas box with moving gas, full exchange and the O(beta tau) terms, two
    gas steps of CFL-limited subcycles on the tiled kernels."""
    announce(f"p1 tiled 3d {precision}")
    spec = ri.default_spec(nx=70, ny=19, nz=12, dx=1 / 70, dy=1 / 19, dz=1 / 12, c_light=40.0,
                           exchange="full", theta_E=0.7, theta_F=0.51, bc="periodic",
                           beta_tau=True, closure="p1", precision=precision)
    st = ri.smooth_random_state(spec, seed=43, amp=0.15, f_amp=0.4, kappa=(1.0, 1.0), v_amp=0.1)
    chat = 20.0
    ref = st
    with P.Solver(spec) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, 8 if precision == "fp64" else 16)
        s.set_state(st)
        for _ in range(2):
            dt, ns, _ = oracle.suggest_dt(spec, ref, chat)
            s.step(dt, chat, ns)
            ref, _ = oracle.step(spec, ref, dt, chat, ns)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"p1 3d {precision}")


def test_batch_of_m1_and_p1_members_equals_lone_handles():
    """Each member of a batch keeps its own closure: an M1 and a P1 member of the same
    input step together and each equals its lone handle to rounding (the batch runs
    other kernels of the same device code); the two results differ."""
    announce("p1 batch member")
    pbs = []
    for closure in ("m1", "p1"):
        spec = ri.default_spec(nx=40, ny=24, nz=20, dx=1 / 40, dy=1 / 24, dz=1 / 20,
                               c_light=100.0, exchange="full", theta_E=0.7, theta_F=0.51,
                               bc="periodic", closure=closure, precision="mixed")
        st = ri.smooth_random_state(spec, seed=17, amp=0.1, f_amp=0.4, kappa=(3.0, 2.0),
                                    v_amp=0.1)
        pbs.append(dict(spec=spec, state=st, chat=10.0))
    ref = []
    for pb in pbs:
        with P.Solver(pb["spec"]) as s:
            s.set_kernel_variant(P.RHD_KERNELS_TILED, 8, 16)
            s.set_state(pb["state"])
            for _ in range(3):
                dt, ns = s.suggest_dt(pb["chat"])
                s.step(dt, pb["chat"], ns)
            ref.append(s.get_state())
    b = P.rhd_batch_create(8, 8, 16)
    solvers = []
    try:
        for pb in pbs:
            s = P.Solver(pb["spec"])
            s.set_state(pb["state"])
            P.rhd_batch_add(b, s.h, pb["chat"])
            solvers.append(s)
        for _ in range(3):
            P.rhd_batch_step(b)
        outs = [s.get_state() for s in solvers]
        for s in solvers:
            P.rhd_batch_remove(b, s.h)
    finally:
        P.rhd_batch_destroy(b)
        for s in solvers:
            s.close()
    for pb, o, r in zip(pbs, outs, ref):
        assert_parity(pb["spec"], o, r, 1e-6, "max", label=f"batch {pb['spec']['closure']}")
    assert np.abs(outs[0]["Er"] - outs[1]["Er"]).max() > 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_p1_shadow_matches_oracle(precision):
    """The P1 closure with the opacity law and the fixed beam face (the coarse shadow
    test, 150 steps): the per-cell kernels against the oracle."""
    announce(f"p1 shadow {precision}")
    pb = ri.shadow_problem(56, 16, emission=False, precision=precision)
    spec = dict(pb["spec"], closure="p1")
    dt, chat, steps = pb["dt"], pb["chat"], 150
    ref, _ = oracle.step(spec, pb["state"], dt, chat, 1, steps=steps)
    with P.Solver(spec) as s:
        s.set_state(pb["state"])
        s.set_boundary(spec["bvals"])
        s.run(np.full(steps, dt), np.ones(steps, dtype=np.int32), chat)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"p1 shadow {precision}")
