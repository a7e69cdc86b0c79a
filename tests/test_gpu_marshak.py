"""GPU parity for fixed radiation faces and the c_v = alpha T^3 gas: the non-equilibrium
Marshak wave of Sec. 4.1.3, driven by the Su & Olson surface solution, against the FP64
oracle step by step with the same boundary states; fixed faces on 2D and 3D grids with
a seeded state, meeting reflecting and periodic faces at edges and corners.

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


def run_both(spec, st, steps, dt, chat, nsub, bvals_at):
    """The same driven run on the GPU and in the oracle; bvals_at(step) gives the fixed
    faces' states of each step."""
    ref = st
    spec_o = dict(spec)
    with P.Solver(spec) as s:
        s.set_state(st)
        for n in range(steps):
            bv = bvals_at(n)
            s.set_boundary(bv)
            s.step(dt, chat, nsub)
            spec_o["bvals"] = bv
            ref, _ = oracle.step(spec_o, ref, dt, chat, nsub)
        s.sync()
        return s.get_state(), ref, s.diagnostics()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_marshak_wave_matches_oracle(precision):
    announce(f"marshak {precision}")
    pb = ri.marshak_problem(96, precision=precision)
    spec, dt = pb["spec"], pb["dt"]
    gpu, ref, diag = run_both(spec, pb["state"], 80, dt, 1.0, 1,
                              lambda n: ri.marshak_boundary((n + 0.5) * dt))
    assert diag["nonfinite"] == 0 and diag["steps"] == 80
    assert gpu["Er"][0, 0, 0] > 0.3  # the wave has entered the medium
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"marshak {precision}")


def fixed_case(n, bc, seed, precision):
    spec = ri.default_spec(nx=n[0], ny=n[1], nz=n[2], dx=1.0 / n[0], dy=1.0 / n[1],
                           dz=1.0 / max(n[2], 1), c_light=20.0, rad_only=True,
                           exchange="full", theta_E=0.6, theta_F=0.51, bc=bc,
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=seed, amp=0.1, f_amp=0.3, kappa=(3.0, 2.0), v_amp=0.0)
    rng = np.random.default_rng(seed)
    table = [(float(rng.uniform(0.5, 2.0)), *(float(x) for x in rng.uniform(-3.0, 3.0, 3)))
             for _ in range(6)]
    return spec, st, tuple(table)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n,bc", [
    ((40, 18, 1), ("fixed", "fixed", "reflect", "fixed", "periodic", "periodic")),
    ((21, 13, 11), ("fixed", "outflow", "periodic", "periodic", "reflect", "fixed")),
    ((70, 9, 6), ("fixed", "fixed", "fixed", "fixed", "fixed", "fixed")),
])
def test_fixed_faces_match_oracle(n, bc, precision):
    """Seeded states with fixed faces beside every other boundary kind, including cells
    beyond two or three fixed faces at once; each step sets new face states. The 3D
    grids run the per-cell kernels (fixed faces never take the tiled path)."""
    announce(f"fixed faces {n} {bc} {precision}")
    spec, st, table = fixed_case(n, bc, seed=sum(n), precision=precision)
    dt = 0.3 / (spec["c_light"] * max(n))
    gpu, ref, diag = run_both(spec, st, 3, dt, spec["c_light"], 1,
                              lambda k: tuple((E * (1 + 0.1 * k), fx, fy, fz)
                                              for (E, fx, fy, fz) in table))
    assert diag["nonfinite"] == 0
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"fixed {n} {precision}")


def test_boundary_calls_are_checked():
    announce("fixed face errors")
    pb = ri.marshak_problem(16)
    with P.Solver(pb["spec"]) as s:
        for face, U, why in [(2, (1.0, 0, 0, 0), "inactive y face"),
                             (0, (0.0, 0, 0, 0), "E_r = 0"),
                             (1, (1.0, float("nan"), 0, 0), "not finite"),
                             (6, (1.0, 0, 0, 0), "no such face")]:
            with pytest.raises(P.RhdError) as e:
                P.rhd_set_boundary(s.h, face, U)
            assert e.value.code == P.RHD_EINVAL, why
    spec = ri.default_spec(nx=8, ny=8, nz=8, dx=0.125, dy=0.125, dz=0.125, bc="periodic")
    with P.Solver(spec) as s:
        with pytest.raises(P.RhdError):
            P.rhd_set_boundary(s.h, 0, (1.0, 0.0, 0.0, 0.0))


def stepped(spec, st, dts, nsubs, chat, bvals=None):
    """Reference: one rhd_set_boundary + rhd_step per step."""
    with P.Solver(spec) as s:
        s.set_state(st)
        for k, (dt, ns) in enumerate(zip(dts, nsubs)):
            if bvals is not None:
                s.set_boundary(bvals[k])
            s.step(dt, chat, ns)
        s.sync()
        return s.get_state(), s.diagnostics()


def run_once(spec, st, dts, nsubs, chat, bvals=None):
    with P.Solver(spec) as s:
        s.set_state(st)
        s.run(dts, nsubs, chat, bvals)
        s.sync()
        return s.get_state(), s.diagnostics()


def assert_same(a, b, da, db):
    for k in ri.FIELDS:
        assert np.array_equal(a[k], b[k]), k
    for k in ("steps", "subcycles", "exch_theta1", "exch_bisect", "newton_iters", "newton_max",
              "rad_fclamp", "rad_efloor", "nonfinite"):
        assert da[k] == db[k], k
    assert da["ledger"] == db["ledger"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_equals_stepping_on_the_marshak_wave(precision):
    announce(f"rhd_run marshak 1200 fp64")
    pb = ri.marshak_problem(1200)
    dts = np.full(40, pb["dt"])
    nsubs = np.ones(40, dtype=np.int32)
    bvals = np.array([ri.marshak_boundary((k + 0.5) * pb["dt"], nq=400) for k in range(40)])
    a, da = run_once(pb["spec"], pb["state"], dts, nsubs, 1.0, bvals)
    b, db = stepped(pb["spec"], pb["state"], dts, nsubs, 1.0, bvals)
    assert_same(a, b, da, db)
    """rhd_run on a small 1D radiation-only grid takes 1024 steps per launch of one
    workgroup; across three launches its result and counters equal step-by-step
    stepping bit for bit. The 1200-cell FP64 grid takes the step-by-step path inside
    rhd_run and must give the same."""
    announce(f"rhd_run marshak {precision}")
    pb = ri.marshak_problem(96, precision=precision)
    spec, dt = pb["spec"], pb["dt"]
    n = 2300
    dts = np.full(n, dt)
    nsubs = np.ones(n, dtype=np.int32)
    bvals = np.array([ri.marshak_boundary((k + 0.5) * dt, nq=400) for k in range(n)])
    a, da = run_once(spec, pb["state"], dts, nsubs, 1.0, bvals)
    b, db = stepped(spec, pb["state"], dts, nsubs, 1.0, bvals)
    assert_same(a, b, da, db)
    assert a["Er"][0, 0, 0] > 0.5


def test_run_equals_stepping_with_exchange_opacity_and_emission_fields():
    """A 1D periodic radiation-only grid of 1500 cells (more cells than threads, mixed
    precision, so still one workgroup) with the ideal-gas exchange (Newton iterations),
    per-cell opacities, emission and a subcycle count that changes from step to step."""
    announce("rhd_run 1d ideal gas")
    n = 1500
    spec = ri.default_spec(nx=n, dx=1.0 / n, c_light=20.0, rad_only=True, exchange="full",
                           theta_E=0.7, theta_F=0.51, bc="periodic", precision="mixed")
    st = ri.smooth_random_state(spec, seed=77, amp=0.2, f_amp=0.3, kappa=(3.0, 2.0), v_amp=0.0,
                                with_j=True)
    assert np.ndim(st["kP"]) > 0 and np.ptp(st["kP"]) > 0 and st.get("j") is not None
    nsubs = np.array([1, 2, 3, 4, 2, 1] * 20, dtype=np.int32)
    dts = 0.35 * spec["dx"] / spec["c_light"] * nsubs
    a, da = run_once(spec, st, dts, nsubs, spec["c_light"])
    b, db = stepped(spec, st, dts, nsubs, spec["c_light"])
    assert da["newton_iters"] > 0
    assert_same(a, b, da, db)


def test_run_on_other_grids_enqueues_the_steps():
    announce("rhd_run 3d")
    spec = ri.default_spec(nx=20, ny=12, nz=10, dx=0.05, dy=1 / 12, dz=0.1, c_light=30.0,
                           exchange="full", bc="periodic", precision="mixed")
    st = ri.smooth_random_state(spec, seed=5, amp=0.1, f_amp=0.3, kappa=(3.0, 2.0), v_amp=0.1)
    dt, ns, _ = oracle.suggest_dt(spec, st, 30.0)
    dts, nsubs = np.full(3, dt), np.full(3, ns, dtype=np.int32)
    a, da = run_once(spec, st, dts, nsubs, 30.0)
    b, db = stepped(spec, st, dts, nsubs, 30.0)
    assert_same(a, b, da, db)


def test_run_checks_every_step_before_enqueueing():
    announce("rhd_run errors")
    pb = ri.marshak_problem(32)
    spec, dt = pb["spec"], pb["dt"]
    with P.Solver(spec) as s:
        s.set_state(pb["state"])
        before = s.get_state()
        dts = np.full(8, dt)
        dts[5] = 10 * dt  # breaks the CFL condition in step 5
        with pytest.raises(P.RhdError) as e:
            s.run(dts, np.ones(8, dtype=np.int32), 1.0)
        assert e.value.code == P.RHD_ECFL
        bv = np.array([ri.marshak_boundary(0.1)] * 8)
        bv[3, 0, 0] = -1.0
        with pytest.raises(P.RhdError) as e:
            s.run(np.full(8, dt), np.ones(8, dtype=np.int32), 1.0, bv)
        assert e.value.code == P.RHD_EINVAL
        after = s.get_state()
        assert s.diagnostics()["steps"] == 0
        for k in ri.FIELDS:
            assert np.array_equal(before[k], after[k]), k
