"""GPU parity for the opacity law kappa(T_gas, rho) and the shadow test of Sec. 4.1.1:
the coarse shadow problem (fixed beam face, outflow and reflecting faces, per-cell
kernels) without and with emission, and a 3D box with the law on the tiled kernels,
each against the FP64 oracle on the same inputs.

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
# The beam enters at the realizability limit f = 1, where the M1 eigenvalues have a
# square-root branch point: a rounding difference delta in f (the two sides evaluate the
# closure in different but equivalent forms) moves the transverse wave speeds by
# chat sqrt(2 delta) ~ 1e-8 chat. Those speeds set the HLL dissipation across the edge of
# the shadow, so FP64 results agree to ~sqrt(eps) there (4.5e-9 seen); 2e-8 bounds it.
FP64_TOL_BEAM = 2e-8


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def run_shadow(emission, precision, steps=150, heat_capacity=1.0):
    pb = ri.shadow_problem(56, 16, emission=emission, precision=precision,
                           heat_capacity=heat_capacity)
    spec, st, dt, chat = pb["spec"], pb["state"], pb["dt"], pb["chat"]
    ref, _ = oracle.step(spec, st, dt, chat, 1, steps=steps)
    with P.Solver(spec) as s:
        s.set_state(st)
        s.set_boundary(spec["bvals"])
        s.run(np.full(steps, dt), np.ones(steps, dtype=np.int32), chat)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0 and diag["steps"] == steps
    return spec, gpu, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shadow_without_emission_matches_oracle(precision):
    announce(f"shadow absorption {precision}")
    spec, gpu, ref = run_shadow(False, precision)
    tol = FP64_TOL_BEAM if precision == "fp64" else TOL[precision]
    assert_parity(spec, gpu, ref, tol, NORM[precision], label=f"shadow absorption {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shadow_with_emission_well_conditioned_matches_oracle(precision):
    """The emission variant with a gas of 10^-6 the heat capacity (e ~ 3.6e4 erg/cm^3
    in the cloud, so the exchange's condition number e / E_r drops to ~1e8): the same
    kernels (opacity law refreshed per step, full exchange, fixed beam face) meet the
    usual bars on every field."""
    announce(f"shadow emission small heat capacity {precision}")
    spec, gpu, ref = run_shadow(True, precision, heat_capacity=1e-6)
    tol = FP64_TOL_BEAM if precision == "fp64" else TOL[precision]
    assert_parity(spec, gpu, ref, tol, NORM[precision], label=f"shadow emission cv/1e6 {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_shadow_with_emission_matches_oracle_to_the_exchange_conditioning(precision):
    """With emission the exchange sets E_r = (chat/c)(Ebar - e) (Eq. source:eradupdate).
    In this cgs problem the gas energy density e reaches 3.6e10 erg/cm^3 in the cloud
    while E_r is ~1e-4, so the update has the condition number K = e / ((c/chat) E_r)
    ~ 1e14 of Eq. source:kappacond: any FP64 solver leaves E_r with rounding of
    ~eps e. The gas fields meet the usual bars; E_r and F are held per cell to the
    usual bar plus 10 eps (chat/c) times the largest Ebar of the grid (transport carries
    the cloud's rounding to its neighbours; F: times c)."""
    announce(f"shadow emission {precision}")
    spec, gpu, ref = run_shadow(True, precision)
    gas = ("rho", "mx", "my", "mz", "E")
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], fields=gas,
                  label=f"shadow emission gas {precision}")
    eps = np.finfo(np.float64).eps
    c = spec["c_light"]
    ebar = ref["E"] + ref["Er"]  # chat = c
    base = (FP64_TOL_BEAM if precision == "fp64" else 3e-6) * float(np.max(ref["Er"]))
    bound = base + 10 * eps * float(np.max(ebar))
    dE = np.abs(gpu["Er"] - ref["Er"])
    assert np.all(dE <= bound), float(np.max(dE) / bound)
    for k in ("Fx", "Fy"):
        dF = np.abs(gpu[k] - ref[k])
        assert np.all(dF <= c * (base + 10 * eps * float(np.max(ebar)))), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_opacity_law_on_tiled_kernels_matches_oracle(precision):
    """A 3D ideal-gas box (full coupling, gas moving) whose opacities follow
    kappa = k0 (T/T0)^-1 (rho/rho0)^0.5, refreshed every gas step; the tiled kernels
    read the law's per-cell opacities."""
    announce(f"opacity law 3d {precision}")
    spec = ri.default_spec(nx=70, ny=9, nz=12, dx=1 / 70, dy=1 / 9, dz=1 / 12, c_light=40.0,
                           exchange="full", theta_E=0.7, theta_F=0.51, bc="periodic",
                           kappa_law=(3.0, 1.0, 1.0, -1.0, 0.5), precision=precision)
    st = ri.smooth_random_state(spec, seed=31, amp=0.15, f_amp=0.3, kappa=(1.0, 1.0), v_amp=0.1)
    chat = 20.0
    ref = st
    with P.Solver(spec) as s:
        s.set_state(st)
        for _ in range(3):
            dt, ns, _ = oracle.suggest_dt(spec, ref, chat)
            dt_g, ns_g = s.suggest_dt(chat)
            assert ns_g == ns and dt_g == pytest.approx(dt, rel=1e-5 if precision == "mixed" else 1e-12)
            s.step(dt, chat, ns)
            ref, _ = oracle.step(spec, ref, dt, chat, ns)
        s.sync()
        gpu = s.get_state()
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"law 3d {precision}")


# Transverse flux of a beam below the smallest normal number of each precision.
SUBNORMAL = {"fp64": 1e-315, "mixed": 1e-42}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["1d fused", "2d per-cell", "3d tiled"])
def test_beam_with_subnormal_transverse_flux_stays_finite(case, precision):
    """A beam at f = 1 whose flux across the faces of one direction is subnormal, with
    random signs; in the shadow test's lit region FP64 develops such values after ~1900
    steps at 280 x 80. The HLL bounds across those faces then differ by a subnormal
    amount, whose reciprocal overflows; the flux is the central one there, as when the
    bounds vanish (negligible against the oracle's, which divides). The 1D grid carries
    the beam along y (a passive component) and the subnormal part along x, the only
    active direction, on the one-workgroup path; 2D runs the per-cell kernels, 3D the
    tiled ones."""
    announce(f"subnormal transverse flux {case} {precision}")
    n = {"1d fused": (64, 1, 1), "2d per-cell": (40, 24, 1), "3d tiled": (48, 16, 12)}[case]
    spec = ri.default_spec(nx=n[0], ny=n[1], nz=n[2], dx=1.0 / n[0], dy=1.0 / n[1],
                           dz=1.0 / n[2], c_light=1.0, rad_only=True, exchange="none",
                           theta_F=1.0, bc="periodic", precision=precision)
    st = ri.uniform_state(spec, Er=1.0, kP=0.0, kF=0.0)  # transparent: f stays 1
    rng = np.random.default_rng(12)
    tiny = SUBNORMAL[precision] * rng.choice([-1.0, 1.0], size=st["Er"].shape)
    tiny *= rng.integers(1, 50, size=st["Er"].shape)
    if case == "1d fused":
        st["Fy"][:], st["Fx"][:] = 1.0, tiny
    else:
        st["Fx"][:], st["Fy"][:] = 1.0, tiny
    dt = 0.3 * min(spec["dx"], spec["dy"] if n[1] > 1 else 1.0, spec["dz"] if n[2] > 1 else 1.0)
    steps = 4
    ref, _ = oracle.step(spec, st, dt, 1.0, 1, steps=steps)
    with P.Solver(spec) as s:
        if case == "3d tiled":
            s.set_kernel_variant(P.RHD_KERNELS_TILED, 8 if precision == "fp64" else 16)
        s.set_state(st)
        s.run(np.full(steps, dt), np.ones(steps, dtype=np.int32), 1.0)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0 and diag["steps"] == steps
    for k in ri.FIELDS:
        if gpu.get(k) is not None:
            assert np.isfinite(gpu[k]).all(), k
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"subnormal {case}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["1d fused", "2d per-cell", "3d tiled"])
@pytest.mark.parametrize("Er", [1e-12, 1e-8])
def test_exchange_that_rounds_the_radiation_away_is_floored(Er, case, precision):
    """Gas at 1 K holding e ~ 1.2e8 erg/cm^3 beside a beam of E_r far below the spacing
    of e (condition number K ~ 1e20, Eq. source:kappacond): the exchange's E_r rounds to
    zero or below and is raised to the floor, as in the oracle; a zero E_r left in place
    made the closure of the beam 0 * inf. Every path (the one-workgroup 1D path, the
    per-cell and the tiled kernels) ends at E_r = er_floor in every cell."""
    announce(f"exchange floor {case} {precision} Er={Er}")
    n = {"1d fused": (64, 1, 1), "2d per-cell": (40, 24, 1), "3d tiled": (48, 16, 12)}[case]
    spec = ri.default_spec(nx=n[0], ny=n[1], nz=n[2], dx=0.1, dy=0.1, dz=0.1, c_light=ri.C_CGS,
                           a_rad=ri.A_RAD_CGS, r_gas=ri.R_GAS_CGS, gamma=5.0 / 3.0, rad_only=True,
                           exchange="full", theta_E=1.0, bc="periodic", er_floor=1e-30,
                           precision=precision)
    c = spec["c_light"]
    st = ri.uniform_state(spec, rho=1.0, P=ri.R_GAS_CGS, Er=Er, F=(c * Er, 0.0, 0.0),
                          kP=1.0, kF=1.0)
    floor = float(np.float32(spec["er_floor"])) if precision == "mixed" else spec["er_floor"]
    dt = 1e-12
    nsubs = np.array([0, 1, 1], dtype=np.int32)  # the exchange alone, then whole steps
    ref, _ = oracle.step(spec, st, dt, c, 0)
    ref, _ = oracle.step(spec, ref, dt, c, 1, steps=2)
    with P.Solver(spec) as s:
        if case == "3d tiled":
            s.set_kernel_variant(P.RHD_KERNELS_TILED, 8 if precision == "fp64" else 16)
        s.set_state(st)
        s.run(np.full(1, dt), nsubs[:1], c)
        s.sync()
        assert np.all(s.get_state()["Er"] == floor)
        s.run(np.full(2, dt), nsubs[1:], c)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    assert np.all(ref["Er"] == spec["er_floor"]) and np.all(gpu["Er"] == floor)
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label=f"exchange floor {case}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_opacity_law_follows_a_new_state(precision):
    """With the gas frozen and absorption only, the law's values are kept between steps;
    rhd_set_state with a hotter gas must bring new ones: a handle stepped on state A,
    then given state B and stepped again, ends where a fresh handle on B ends, bit for
    bit, and the oracle agrees."""
    announce(f"opacity law cache {precision}")
    pb = ri.shadow_problem(56, 16, emission=False, precision=precision)
    spec, dt, chat = pb["spec"], pb["dt"], pb["chat"]
    A = pb["state"]
    B = ri.copy_state(A)
    B["E"] = B["E"] * 1.7  # a hotter gas: a lower opacity under kappa ~ T^-3.5
    with P.Solver(spec) as s:
        s.set_state(A)
        s.set_boundary(spec["bvals"])
        s.run(np.full(3, dt), np.ones(3, dtype=np.int32), chat)
        s.set_state(B)
        s.run(np.full(3, dt), np.ones(3, dtype=np.int32), chat)
        s.sync()
        got = s.get_state()
    with P.Solver(spec) as s:
        s.set_state(B)
        s.set_boundary(spec["bvals"])
        s.run(np.full(3, dt), np.ones(3, dtype=np.int32), chat)
        s.sync()
        fresh = s.get_state()
    for k in ri.FIELDS:
        assert np.array_equal(got[k], fresh[k]), k
    ref, _ = oracle.step(spec, B, dt, chat, 1, steps=3)
    tol = FP64_TOL_BEAM if precision == "fp64" else TOL[precision]
    assert_parity(spec, got, ref, tol, NORM[precision], label=f"law cache {precision}")
