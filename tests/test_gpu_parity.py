"""GPU parity: the HIP library, called through its C interface, against the FP64 CPU
oracle on the same seeded inputs.

Tolerances (stated per field against its natural scale, see parity.py):
  FP64 mode  -- max-norm error <= 1e-12 (both sides are FP64; they differ by operation
                order, fused multiply-adds and the algebraically equivalent closure forms);
  mixed mode -- L1 error <= 1e-5 (FP32 storage and stencils, FP64 exchange and ledger).
Grids are chosen so that launches have several blocks and a ragged tail in x and y.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1306_0010_amd as P
import rhd_inputs as ri
from parity import assert_parity, field_errors, window
from bench import TILE_C3  # the 256^3 workloads' tile shape, as the benchmark times them

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
NORM = {"fp64": "max", "mixed": "l1"}
# Cases whose radiation flux reaches the realizability limit f = 1 in many cells (the
# dusty shell clamps F in ~2e3 cell-stages of its first step). At f = 1 the extreme M1
# eigenvalues have a square-root branch point: a rounding difference delta in f moves
# them by chat sqrt(2 delta), i.e. by ~1e-8 chat for delta of a few FP64 ulp. The speeds
# enter the HLL dissipation term, so FP64 results agree to ~sqrt(eps) times the share of
# that term instead of ~eps; 1e-10 bounds it with a margin of three over what is seen.
FP64_TOL_BRANCH_POINT = {"dusty_shell_32": 1e-10}
# The shadow problem's beam enters at f = 1 exactly, across the whole fixed face: the
# same branch point, reached by every lit cell, whose FP64 results agree to ~sqrt(eps).
FP64_TOL_BEAM = 2e-8


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def run_gpu(spec, st, steps, chat, dt=None, nsub=None, variant=None):
    """Run ``steps`` gas steps on the GPU with the given (dt, nsub). ``variant`` is
    (kernel variant, tile rows, z chunk) or None for the library's default."""
    with P.Solver(spec) as s:
        if variant is not None:
            s.set_kernel_variant(*variant)
        s.set_state(st)
        for _ in range(steps):
            s.step(dt, chat, nsub)
        s.sync()
        return s.get_state(), s.diagnostics()


def step_sizes(spec, st, chat):
    dt, ns, _ = oracle.suggest_dt(spec, st, chat)
    return dt, ns


CASES = {}


def case(fn):
    CASES[fn.__name__] = fn
    return fn


@case
def rhd3d_periodic(precision):
    spec = ri.default_spec(nx=37, ny=29, nz=21, dx=1 / 37, dy=1 / 29, dz=1 / 21, c_light=50.0,
                           exchange="full", theta_E=0.51, theta_F=0.51, bc="periodic",
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=1, amp=0.1, f_amp=0.3, kappa=(3.0, 2.0), v_amp=0.1)
    return spec, st, 10.0, 2


@case
def rhd3d_mixed_bc_beta_tau(precision):
    spec = ri.default_spec(nx=33, ny=17, nz=12, dx=1 / 33, dy=1 / 17, dz=1 / 12, c_light=30.0,
                           exchange="full", beta_tau=True, theta_E=1.0, theta_F=0.51,
                           bc=("outflow", "outflow", "reflect", "reflect", "periodic", "periodic"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=2, amp=0.1, f_amp=0.4, kappa=(2.0, 5.0), v_amp=0.2,
                                with_j=True)
    return spec, st, 8.0, 2


@case
def rhd3d_two_full_x_tiles(precision):
    """128 cells in x: two full 64-wide tiles, so the faces on a tile edge (inside the
    grid and at a reflecting wall) come from the extra work items of the tiled kernels."""
    spec = ri.default_spec(nx=128, ny=9, nz=6, dx=1 / 128, dy=1 / 9, dz=1 / 6, c_light=40.0,
                           exchange="full", beta_tau=True, theta_E=0.51, theta_F=0.51,
                           bc=("reflect", "reflect", "outflow", "outflow", "periodic", "periodic"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=8, amp=0.1, f_amp=0.4, kappa=(1.0, 4.0), v_amp=0.2,
                                with_j=True)
    return spec, st, 12.0, 2


@case
def dusty_shell_32(precision):
    """The dusty-shell workload at 32^3: isothermal gas, outflow faces, radiative
    equilibrium, lognormal shell and a central Gaussian source; chat is 20 v_max. One gas
    step: the source accelerates the central gas to several times the sound speed within
    it, so a second step at the same dt would exceed the CFL limit."""
    pb = ri.c4_dusty_shell(32, precision=precision)
    spec, st = pb["spec"], pb["state"]
    _, _, vmax = oracle.suggest_dt(spec, st, 1.0)
    return spec, st, pb["chat_over_vmax"] * vmax, 1


@case
def rad_only_absorb_2d_wave(precision):
    pb = ri.radiation_wave(2, 16)
    spec = dict(pb["spec"], precision=precision)
    return spec, pb["state"], pb["chat"], 4


@case
def rad_only_outflow_source_3d(precision):
    spec = ri.default_spec(nx=70, ny=9, nz=10, dx=1 / 70, dy=1 / 9, dz=1 / 10, c_light=1.0,
                           exchange="none", rad_only=True, theta_F=1.0, bc="outflow",
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=4, amp=0.2, f_amp=0.5, kappa=(0.0, 20.0), with_j=True)
    return spec, st, 1.0, 3


@case
def isothermal_3d(precision):
    spec = ri.default_spec(nx=24, ny=20, nz=18, dx=1 / 24, dy=1 / 20, dz=1 / 18, c_light=40.0,
                           isothermal=True, iso_cs=1.0, exchange="none", theta_F=1.0,
                           bc=("outflow", "outflow", "periodic", "periodic", "reflect", "reflect"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=5, amp=0.2, f_amp=0.2, kappa=(1.0, 3.0), v_amp=0.3)
    return spec, st, 6.0, 2


@case
def one_d_exchange(precision):
    spec = ri.default_spec(nx=300, dx=1 / 300, c_light=100.0, exchange="full", theta_E=0.51,
                           bc="periodic", precision=precision)
    st = ri.smooth_random_state(spec, seed=6, amp=0.2, f_amp=0.3, kappa=(20.0, 20.0), v_amp=0.1)
    return spec, st, 20.0, 5


@case
def two_d_reflect(precision):
    spec = ri.default_spec(nx=65, ny=7, dx=1 / 65, dy=1 / 7, c_light=20.0, exchange="full",
                           bc=("reflect", "reflect", "reflect", "reflect", "periodic", "periodic"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=7, amp=0.15, f_amp=0.3, kappa=(1.0, 1.0), v_amp=0.2)
    return spec, st, 5.0, 3


@case
def one_d_along_z(precision):
    """A column along z only (x and y inactive): the boundary mapping and the flux
    directions of the last dimension alone, with reflecting ends and moving gas."""
    spec = ri.default_spec(nz=160, dz=1 / 160, c_light=60.0, exchange="full", theta_E=0.51,
                           beta_tau=True, bc=("periodic",) * 4 + ("reflect", "reflect"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=9, amp=0.2, f_amp=0.3, kappa=(5.0, 5.0), v_amp=0.2)
    return spec, st, 15.0, 3


@case
def two_d_xz_plane(precision):
    """An x-z plane (y inactive) with outflow in x and periodic z."""
    spec = ri.default_spec(nx=40, nz=30, dx=1 / 40, dz=1 / 30, c_light=30.0, exchange="full",
                           bc=("outflow", "outflow", "periodic", "periodic", "periodic", "periodic"),
                           precision=precision)
    st = ri.smooth_random_state(spec, seed=10, amp=0.15, f_amp=0.4, kappa=(2.0, 3.0), v_amp=0.2)
    return spec, st, 8.0, 2


@case
def two_d_yz_plane(precision):
    """A y-z plane (x inactive) with reflecting y walls and outflow in z."""
    spec = ri.default_spec(ny=24, nz=36, dy=1 / 24, dz=1 / 36, c_light=30.0, exchange="full",
                           theta_E=0.7, bc=("periodic", "periodic", "reflect", "reflect", "outflow",
                                            "outflow"), precision=precision)
    st = ri.smooth_random_state(spec, seed=11, amp=0.15, f_amp=0.4, kappa=(2.0, 3.0), v_amp=0.2,
                                with_j=True)
    return spec, st, 8.0, 2


VARIANTS = {"per_cell": (P.RHD_KERNELS_PER_CELL, 8, 16), "tiled": (P.RHD_KERNELS_TILED, 8, 16),
            "face_split": (P.RHD_KERNELS_FACE_SPLIT, 8, 16)}


@pytest.mark.parametrize("variant", ["per_cell", "tiled", "face_split"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_step_matches_oracle(name, precision, variant):
    announce(f"{name} {precision} {variant}")
    spec, st, chat, steps = CASES[name](precision)
    dt, ns = step_sizes(spec, st, chat)
    ref, cnt = oracle.step(spec, st, dt, chat, ns, steps=steps)
    gpu, diag = run_gpu(spec, st, steps, chat, dt, ns, VARIANTS[variant])
    tol = TOL[precision]
    if precision == "fp64":
        tol = FP64_TOL_BRANCH_POINT.get(name, tol)
    assert_parity(spec, gpu, ref, tol, NORM[precision], label=f"{name} {precision}")
    assert diag["nonfinite"] == 0 and diag["steps"] == steps and diag["subcycles"] == steps * ns
    if precision == "fp64":
        # same branch decisions: exchange fallbacks, floors and clamps
        for k in ("exch_theta1", "exch_bisect", "gas_rhofloor", "gas_pfloor", "rad_efloor"):
            assert diag[k] == cnt[k], (k, diag[k], cnt[k])
        assert abs(diag["newton_iters"] - cnt["newton_iters"]) <= 1e-3 * max(1, cnt["newton_iters"])


@pytest.mark.parametrize("rows,zchunk,precision", [(4, 16, "fp64"), (8, 3, "fp64"), (4, 7, "mixed"),
                                                   (8, 16, "mixed"), (16, 16, "mixed"), (16, 1, "mixed")])
def test_tile_shapes_agree_with_per_cell_kernels(rows, zchunk, precision):
    """Every tile shape gives the per-cell kernels' result to rounding."""
    announce(f"tile shape {rows} {zchunk} {precision}")
    spec, st, chat, steps = rhd3d_mixed_bc_beta_tau(precision)
    dt, ns = step_sizes(spec, st, chat)
    a, _ = run_gpu(spec, st, 2, chat, dt, ns, (P.RHD_KERNELS_PER_CELL, 8, 16))
    b, _ = run_gpu(spec, st, 2, chat, dt, ns, (P.RHD_KERNELS_TILED, rows, zchunk))
    assert_parity(spec, b, a, 1e-13 if precision == "fp64" else 2e-6, "max", label="tile vs per-cell")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(CASES) + ["shadow_fixed_face", "beam_fixed_faces_3d"])
def test_face_split_kernels_equal_per_cell_kernels(name, precision):
    """The face-split kernels evaluate the per-cell kernels' face fluxes with the same
    code and sum them in the same order; the compiler may still contract multiply-adds
    differently in the two kernels, so the states agree to rounding (the bar against the
    oracle), on every grid dimension and boundary kind, fixed faces included (the coarse
    shadow problem, whose beam sits at the branch point f = 1, and a 3D box with two fixed
    faces)."""
    announce(f"face split vs per cell {name} {precision}")
    if name == "shadow_fixed_face":
        pb = ri.shadow_problem(56, 16, emission=True, precision=precision, heat_capacity=1e-6)
        spec, st, dt, chat, ns, steps = pb["spec"], pb["state"], pb["dt"], pb["chat"], 1, 6
    elif name == "beam_fixed_faces_3d":
        spec = ri.default_spec(nx=20, ny=12, nz=10, dx=1 / 20, dy=1 / 12, dz=1 / 10, c_light=10.0,
                               exchange="full", rad_only=True, bc=("fixed", "outflow", "reflect", "fixed",
                                                    "periodic", "periodic"), precision=precision)
        st = ri.smooth_random_state(spec, seed=5, amp=0.2, f_amp=0.3, kappa=(1.0, 4.0), v_amp=0.1,
                                    with_j=True)
        spec["bvals"] = [[4.0, 3.0, 0.5, -0.2], [0.0] * 4, [0.0] * 4, [2.0, 0.1, -1.5, 0.3],
                         [0.0] * 4, [0.0] * 4]
        chat = 10.0
        dt, ns = step_sizes(spec, st, chat)
        steps = 3
    else:
        spec, st, chat, steps = CASES[name](precision)
        dt, ns = step_sizes(spec, st, chat)
    runs = []
    for v in ("per_cell", "face_split"):
        with P.Solver(spec) as s:
            s.set_kernel_variant(*VARIANTS[v])
            s.set_state(st)
            if "bvals" in spec:
                s.set_boundary(spec["bvals"])
            for _ in range(steps):
                s.step(dt, chat, ns)
            s.sync()
            runs.append((s.get_state(), s.diagnostics()))
    (a, da), (b, db) = runs
    assert da["nonfinite"] == 0 and db["nonfinite"] == 0
    tol = TOL[precision]
    if precision == "fp64":
        tol = FP64_TOL_BRANCH_POINT.get(name, FP64_TOL_BEAM if name == "shadow_fixed_face" else tol)
    assert_parity(spec, b, a, tol, NORM[precision], label=f"face split vs per cell {name}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["one_d_exchange", "pulse_beta_tau", "pulse_fixed_face"])
def test_one_workgroup_subcycles_equal_per_cell_kernels(name, precision):
    """A small 1D grid along x runs the subcycles of a step in one workgroup by default,
    with the per-cell kernels' device code: the states and counters agree bit for bit
    with the per-cell kernels', on a coupled step with the exchange, the pulse with its
    O(beta tau) terms, and a rad-only grid with a fixed face."""
    announce(f"one-workgroup subcycles vs per cell {name} {precision}")
    if name == "one_d_exchange":
        spec, st, chat, steps = one_d_exchange(precision)
        dt, ns = step_sizes(spec, st, chat)
    elif name == "pulse_beta_tau":
        pb = ri.pulse_problem(256, advected=True, beta_tau=True, precision=precision)
        spec, st, chat, steps = pb["spec"], pb["state"], pb["chat"], 4
        dt, ns = step_sizes(spec, st, chat)
    else:
        spec = ri.default_spec(nx=400, dx=1 / 400, c_light=10.0, exchange="full", rad_only=True,
                               bc=("fixed", "outflow", "periodic", "periodic", "periodic",
                                   "periodic"), precision=precision)
        st = ri.smooth_random_state(spec, seed=8, amp=0.2, f_amp=0.3, kappa=(2.0, 5.0))
        spec["bvals"] = [[3.0, 2.5, 0.1, 0.0]] + [[0.0] * 4] * 5
        chat, steps = 10.0, 3
        dt, ns = step_sizes(spec, st, chat)
    runs = []
    for v in (VARIANTS["per_cell"], (P.RHD_KERNELS_TILED, 8, 8)):
        with P.Solver(spec) as s:
            s.set_kernel_variant(*v)
            s.set_state(st)
            if "bvals" in spec:
                s.set_boundary(spec["bvals"])
            for _ in range(steps):
                s.step(dt, chat, ns)
            s.sync()
            runs.append((s.get_state(), s.diagnostics()))
    (a, da), (b, db) = runs
    assert ns > 1 and da["subcycles"] == db["subcycles"] == steps * ns
    for k in ri.FIELDS:
        if a.get(k) is not None:
            assert np.array_equal(a[k], b[k]), k
    for k in ("rad_efloor", "rad_fclamp", "exch_theta1", "exch_bisect", "newton_iters",
              "nonfinite"):
        assert da[k] == db[k], k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c1_gaussian_diffusion_full_run(precision):
    announce(f"c1 {precision}")
    pb = ri.c1_diffusion()
    spec = dict(pb["spec"], precision=precision)
    ref, _ = oracle.run(pb)
    gpu, diag = run_gpu(spec, pb["state"], pb["steps"], pb["chat"], pb["dt"], pb["nsub"])
    assert_parity(spec, gpu, ref, TOL[precision], NORM[precision], label="c1")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sod_gas_only_steps(precision):
    announce(f"sod {precision}")
    pb = ri.sod_tube(130)
    spec = dict(pb["spec"], precision=precision)
    st = pb["state"]
    dt, _, _ = oracle.suggest_dt(spec, st, 1.0)
    ref, _ = oracle.step(spec, st, dt, 1.0, 0, steps=40)
    gpu, _ = run_gpu(spec, st, 40, 1.0, dt, 0)
    assert_parity(spec, gpu, ref, {"fp64": 1e-11, "mixed": 1e-5}[precision], NORM[precision],
                  label="sod")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ledger_and_suggest_dt(precision):
    announce(f"ledger {precision}")
    spec, st, chat, _ = rhd3d_periodic(precision)
    dt, ns = step_sizes(spec, st, chat)
    with P.Solver(spec) as s:
        s.set_state(st)
        gdt, gns = s.suggest_dt(chat)
        tol = 1e-13 if precision == "fp64" else 2e-6
        assert gdt == pytest.approx(dt, rel=tol)
        assert gns == ns
        L0 = s.ledger(chat)
        ref0 = oracle.ledger(spec, st, chat)
        assert np.allclose(L0, ref0, rtol=1e-12 if precision == "fp64" else 1e-6, atol=1e-12)
        s.step(dt, chat, ns)
        L1 = s.diagnostics()["ledger"]
        # periodic box without the O(beta tau) terms: E + (c/chat) E_r and mass are conserved
        assert L1[0] == pytest.approx(L0[0], rel=1e-13 if precision == "fp64" else 2e-6)
        assert L1[4] == pytest.approx(L0[4], rel=1e-14 if precision == "fp64" else 2e-6)


def test_forced_bisection_matches_oracle():
    announce("forced bisection")
    spec, st, chat, _ = rhd3d_periodic("fp64")
    spec = dict(spec, newton_maxit=0)
    dt, ns = step_sizes(spec, st, chat)
    ref, cnt = oracle.step(spec, st, dt, chat, ns)
    gpu, diag = run_gpu(spec, st, 1, chat, dt, ns)
    assert diag["exch_bisect"] == spec["nx"] * spec["ny"] * spec["nz"] == cnt["exch_bisect"]
    assert_parity(spec, gpu, ref, 1e-12, "max", label="bisection")


def test_errors_are_reported():
    announce("errors")
    spec, st, chat, _ = rhd3d_periodic("fp64")
    dt, ns = step_sizes(spec, st, chat)
    with P.Solver(spec) as s:
        with pytest.raises(P.RhdError) as e:
            s.step(dt, chat, ns)
        assert e.value.code == P.RHD_ESTATE
        s.set_state(st)
        for args, code in [((-dt, chat, ns), P.RHD_EINVAL), ((dt, 0.0, ns), P.RHD_EINVAL),
                           ((dt, chat, -1), P.RHD_EINVAL),
                           ((dt * 2.5, chat, ns), P.RHD_ECFL)]:
            with pytest.raises(P.RhdError) as e:
                s.step(*args)
            assert e.value.code == code, args
        s.step(dt, chat, ns)
        s.sync()


def test_nonfinite_state_is_detected():
    announce("nonfinite")
    spec, st, chat, _ = rhd3d_periodic("fp64")
    st = ri.copy_state(st)
    bad = (3, 5, 7)  # (k, j, i)
    st["Er"][bad] = np.nan
    dt, ns = step_sizes(spec, ri.smooth_random_state(spec, seed=1, amp=0.1, f_amp=0.3,
                                                     kappa=(3.0, 2.0), v_amp=0.1), chat)
    with P.Solver(spec) as s:
        s.set_state(st)
        s.step(dt, chat, ns)
        with pytest.raises(P.RhdError) as e:
            s.sync()
        assert e.value.code == P.RHD_ENONFINITE
        d = s.diagnostics()
        assert d["nonfinite"] > 0
        flat = bad[2] + spec["nx"] * (bad[1] + spec["ny"] * bad[0])
        assert 0 <= d["first_nonfinite_cell"] <= flat


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_restart_and_determinism(precision):
    announce(f"checkpoint {precision}")
    spec, st, chat, _ = rhd3d_mixed_bc_beta_tau(precision)
    dt, ns = step_sizes(spec, st, chat)
    a, _ = run_gpu(spec, st, 4, chat, dt, ns)
    b, _ = run_gpu(spec, st, 4, chat, dt, ns)
    half, _ = run_gpu(spec, st, 2, chat, dt, ns)
    st2 = dict(st)
    st2.update(half)
    c, _ = run_gpu(spec, st2, 2, chat, dt, ns)
    for k in ri.FIELDS:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["rhd3d_periodic", "two_d_reflect", "one_d_exchange"])
def test_autotune_keeps_state_and_result(name, precision):
    """The autotuner restores the state and counters exactly, picks a valid kernel
    choice, and the step after it still matches the oracle: on a 3D grid (tiled shapes
    among the candidates), a 2D grid and a 1D grid (per-cell, face-split or the default
    choice)."""
    announce(f"autotune {name} {precision}")
    spec, st, chat, _ = CASES[name](precision)
    dt, ns = step_sizes(spec, st, chat)
    ref, _ = oracle.step(spec, st, dt, chat, ns)
    with P.Solver(spec) as s:
        s.set_state(st)
        before = s.get_state()
        d0 = s.diagnostics()
        v, rows, zc = s.autotune(chat, dt / ns, reps=2)
        assert v in (P.RHD_KERNELS_PER_CELL, P.RHD_KERNELS_TILED, P.RHD_KERNELS_FACE_SPLIT)
        assert rows in (4, 8, 16) and zc >= 1
        after = s.get_state()
        for k in ri.FIELDS:
            assert np.array_equal(before[k], after[k]), k
        d1 = s.diagnostics()
        for k in ("rad_fclamp", "rad_efloor", "nonfinite"):
            assert d0[k] == d1[k]
        if name != "rhd3d_periodic":
            assert (rows, zc) == ((8, 16) if v != P.RHD_KERNELS_TILED else (8, 8))
        s.step(dt, chat, ns)
        s.sync()
        gpu = s.get_state()
    tol = FP64_TOL_BRANCH_POINT.get(name, TOL[precision]) if precision == "fp64" else TOL[precision]
    assert_parity(spec, gpu, ref, tol, NORM[precision], label="after autotune")


def test_torch_stream_and_device_pointers():
    announce("torch interop")
    import torch
    spec, st, chat, _ = rhd3d_periodic("fp64")
    dt, ns = step_sizes(spec, st, chat)
    ref, _ = oracle.step(spec, st, dt, chat, ns)
    dev = torch.device("cuda:0")
    N = spec["nx"] * spec["ny"] * spec["nz"]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to(dev)
    rho, E, Er = t(st["rho"]), t(st["E"]), t(st["Er"])
    mom = torch.cat([t(st["mx"]), t(st["my"]), t(st["mz"])])
    Fr = torch.cat([t(st["Fx"]), t(st["Fy"]), t(st["Fz"])])
    kP, kF = t(st["kP"]), t(st["kF"])
    stream = torch.cuda.current_stream(dev)
    h = P.rhd_create(P.params_from_spec(spec), stream.cuda_stream)
    try:
        P.rhd_set_state_device(h, rho.data_ptr(), mom.data_ptr(), E.data_ptr(), Er.data_ptr(),
                               Fr.data_ptr(), kP.data_ptr(), kF.data_ptr(), 0)
        P.rhd_step(h, dt, chat, ns)
        out = {k: torch.empty(n, dtype=torch.float64, device=dev)
               for k, n in (("rho", N), ("mom", 3 * N), ("E", N), ("Er", N), ("Fr", 3 * N))}
        P.rhd_get_state_device(h, out["rho"].data_ptr(), out["mom"].data_ptr(), out["E"].data_ptr(),
                               out["Er"].data_ptr(), out["Fr"].data_ptr())
        stream.synchronize()
    finally:
        P.rhd_destroy(h)
    sh = (spec["nz"], spec["ny"], spec["nx"])
    o = {k: v.cpu().numpy() for k, v in out.items()}
    gpu = {"rho": o["rho"].reshape(sh), "E": o["E"].reshape(sh), "Er": o["Er"].reshape(sh),
           "mx": o["mom"][:N].reshape(sh), "my": o["mom"][N:2 * N].reshape(sh),
           "mz": o["mom"][2 * N:].reshape(sh), "Fx": o["Fr"][:N].reshape(sh),
           "Fy": o["Fr"][N:2 * N].reshape(sh), "Fz": o["Fr"][2 * N:].reshape(sh)}
    assert_parity(spec, gpu, ref, 1e-12, "max", label="torch")


# ---------------------------------------------------------------------------
# full-size workloads, sampled: windows the oracle can compute one by one
# ---------------------------------------------------------------------------

def window_check(spec, st, gpu, chat, dt, nsub, centres, w, margin, bc_modes, tol, norm):
    """Oracle on sub-boxes of side w + 2 margin around each centre (boundary-mapped like
    the full grid), compared on the central w^3 cells, which lie outside the reach of the
    window's own boundary for one gas step."""
    size = (w + 2 * margin,) * 3
    for cz in centres:
        lo = tuple(c - w // 2 - margin for c in cz)
        sub = window(st, lo, size, bc_modes)
        sspec = dict(spec, nx=size[0], ny=size[1], nz=size[2], bc=("outflow",) * 6)
        ref, _ = oracle.step(sspec, sub, dt, chat, nsub)
        core = tuple(slice(margin, margin + w) for _ in range(3))
        rc = {k: ref[k][core] for k in ri.FIELDS}
        gsub = window({k: gpu[k] for k in ri.FIELDS}, lo, size, bc_modes)
        gc = {k: gsub[k][core] for k in ri.FIELDS}
        assert_parity(spec, gc, rc, tol, norm, label=f"window at {cz}")


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_full_size_box_one_step_windows(precision):
    """The 128^3 linear-perturbation box, one full gas step with one subcycle, at the
    launch configuration of the benchmark; windows include the periodic wrap."""
    announce(f"128^3 box windows {precision}")
    pb = ri.c2_linear_box(128, precision=precision)
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    dt, ns, _ = oracle.suggest_dt(spec, st, chat)
    dt1 = dt / ns  # one subcycle of the right size; the gas step shrinks with it
    gpu, diag = run_gpu(spec, st, 1, chat, dt1, 1)
    assert diag["nonfinite"] == 0
    centres = [(64, 64, 64), (3, 125, 60), (127, 0, 1)]
    window_check(spec, st, gpu, chat, dt1, 1, centres, 8, 8, ("wrap",) * 3, TOL[precision],
                 NORM[precision])


def test_full_size_point_source_subcycle_windows():
    """The 256^3 concentrated-source workload (mixed precision, outflow faces, emission)
    in the benchmark's launch configuration, one radiation subcycle, sampled around the
    source and at a domain corner."""
    announce("256^3 point source windows")
    pb = ri.c3_point_source(256)
    spec, st = pb["spec"], pb["state"]
    # let the source run for a while first so the windows see a radiation field
    with P.Solver(spec) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, *TILE_C3)
        s.set_state(st)
        for _ in range(20):
            s.step(pb["dt"], pb["chat"], 1)
        s.sync()
        mid = s.get_state()
        mid_full = dict(st)
        mid_full.update(mid)
        s.step(pb["dt"], pb["chat"], 1)
        s.sync()
        gpu = s.get_state()
    centres = [(128, 128, 128), (120, 131, 126), (4, 4, 251)]
    window_check(spec, mid_full, gpu, pb["chat"], pb["dt"], 1, centres, 8, 6, ("edge",) * 3,
                 1e-5, "l1")


def test_full_size_dusty_shell_step_windows():
    """The 256^3 dusty shell (isothermal gas, outflow faces, lognormal shell, central
    source, no exchange) in the benchmark's launch configuration: one full gas step
    (isothermal gas Van Leer, one radiation subcycle, source correction) at
    chat = 20 v_max(t=0), sampled at the source, on the shell where it crosses the x
    axis and the y axis, and at a corner."""
    announce("256^3 dusty shell windows")
    pb = ri.c4_dusty_shell(256)
    spec, st = pb["spec"], pb["state"]
    spec64 = dict(spec, precision="fp64")
    chat = pb["chat_over_vmax"] * oracle.suggest_dt(spec64, st, 1.0)[2]
    dt, ns, _ = oracle.suggest_dt(spec64, st, chat)
    dt1 = dt / ns  # one subcycle of the right size; the gas step shrinks with it
    gpu, diag = run_gpu(spec, st, 1, chat, dt1, 1, variant=(P.RHD_KERNELS_TILED, *TILE_C3))
    assert diag["nonfinite"] == 0
    n = spec["nx"]
    shell = int(round((0.3 + 0.5) * n - 0.5))  # cell index where r = 0.3 on an axis
    centres = [(128, 128, 128), (shell, 128, 128), (128, n - 1 - shell, 128), (4, 251, 4)]
    window_check(spec, st, gpu, chat, dt1, 1, centres, 8, 8, ("edge",) * 3, TOL["mixed"],
                 NORM["mixed"])


def test_full_size_box_bench_run_properties():
    """The benchmark workload exactly as timed (128^3, mixed, 10 gas steps with CFL
    subcycles): conservation of E + (c/chat) E_r and of mass to FP32 storage rounding,
    no floors, clamps or non-finite values, and agreement with the FP64 mode run to
    well below the perturbation amplitude."""
    announce("128^3 bench run properties")
    pb = ri.c2_linear_box(128, precision="mixed")
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    outs = {}
    for prec in ("mixed", "fp64"):
        sp = dict(spec, precision=prec)
        with P.Solver(sp) as s:
            s.set_state(st)
            L0 = s.ledger(chat)
            for _ in range(pb["steps"]):
                dt, ns = s.suggest_dt(chat)
                s.step(dt, chat, ns)
            s.sync()
            d = s.diagnostics()
            outs[prec] = s.get_state()
        assert d["nonfinite"] == 0
        assert d["rad_fclamp"] == 0 and d["rad_efloor"] == 0
        assert d["gas_rhofloor"] == 0 and d["gas_pfloor"] == 0
        assert d["ledger"][0] == pytest.approx(L0[0], rel=1e-12 if prec == "fp64" else 1e-6)
        assert d["ledger"][4] == pytest.approx(L0[4], rel=1e-13 if prec == "fp64" else 1e-6)
        assert d["subcycles"] == 10 * 20
    err = field_errors(spec, outs["mixed"], outs["fp64"])
    assert max(v[1] for v in err.values()) < 1e-5, err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dusty_shell_32_over_several_gas_steps(precision):
    """The 32^3 dusty shell over four gas steps, each with the step size and subcycle count
    the oracle's CFL rule gives for the oracle's own state at that step (the source speeds
    the central gas up, so a fixed dt would break the CFL limit after one step). The GPU
    takes the same (dt, nsub) schedule from the same initial state."""
    announce(f"dusty shell 32^3 four gas steps {precision}")
    pb = ri.c4_dusty_shell(32, precision=precision)
    spec, st = pb["spec"], pb["state"]
    chat = pb["chat_over_vmax"] * oracle.suggest_dt(spec, st, 1.0)[2]
    ref, schedule = st, []
    for _ in range(4):
        dt, ns, _ = oracle.suggest_dt(spec, ref, chat)
        schedule.append((dt, ns))
        ref, _ = oracle.step(spec, ref, dt, chat, ns)
    with P.Solver(spec) as s:
        s.set_state(st)
        for dt, ns in schedule:
            s.step(dt, chat, ns)
        s.sync()
        gpu, diag = s.get_state(), s.diagnostics()
    assert diag["nonfinite"] == 0
    print(f"  schedule (dt, nsub): {[(f'{dt:.3e}', ns) for dt, ns in schedule]}", flush=True)
    errs = field_errors(spec, gpu, ref)
    print("  errors (max, L1): " + ", ".join(f"{k}=({v[0]:.2e}, {v[1]:.2e})" for k, v in errs.items()),
          flush=True)
    # each gas step adds its own rounding differences (at the clamped cells, ~sqrt(eps) of
    # the HLL dissipation in FP64; FP32 rounding in mixed precision), so the bar is the
    # one-step bar times the number of steps (seen: FP64 E_r 1.6e-10 max, 4.4 times its
    # one-step difference; mixed E_r 1.3e-5 L1)
    one = TOL[precision] if precision == "mixed" else FP64_TOL_BRANCH_POINT["dusty_shell_32"]
    assert_parity(spec, gpu, ref, len(schedule) * one, NORM[precision],
                  label=f"dusty shell 32^3, 4 steps, {precision}")
