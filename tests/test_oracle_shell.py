"""Pins for the expanding-shell test of Sec. 4.3.6 (its initial state and reference
solution, which the GPU runs are measured against): the dimensional parameters give the
printed Mach number, optical depth and dynamical time; with a shell FWHM of 0.1 r0 the
critical point of the equilibrium ODE falls at the printed r_crit = 1.128 r0; the
tabulated f(r) solves Eq. radshell:odefluxm1; F*(r) has divergence j*(r); the energy
density inside the shell matches the plane-parallel Eddington model of Eq.
radshell:Ermodel; and the printed shell trajectory (Eqs. radshell:odepos and
radshell:odevel) solves Eq. radshell:odeaccelreduced and reaches 2 r0 near t = 0.12 t0."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import rhd_inputs as ri


@pytest.fixture(scope="module")
def prof():
    return ri.shell_profile()


def test_parameters_give_the_printed_scales():
    par = ri.shell_parameters()
    assert par["M0"] == pytest.approx(13.0, rel=0.01)
    assert par["tau0"] == pytest.approx(6.6, rel=0.01)
    assert 1.0 / par["M0"] == pytest.approx(0.076, abs=0.001)


def test_critical_point_is_the_printed_one(prof):
    """Eq. radshell:rcrit with H = 0.1 r0 (the shell FWHM, a reading) gives the paper's
    r_crit = 1.128 r0; the bracket of Eq. radshell:odefluxm1 vanishes there with
    f = 2 sqrt(3)/5, so the point is a regular singularity."""
    assert prof.r_crit == pytest.approx(1.128, abs=5e-4)
    assert abs(prof._bracket(prof.r_crit, prof.f_crit)) < 1e-8
    # other shell widths move it: the pin fixes H
    assert abs(ri.ShellProfile(prof.M0, prof.tau0, prof.c, H=0.15).r_crit - 1.128) > 5e-3


def test_reduced_flux_solves_the_equilibrium_ode(prof):
    r = np.linspace(0.35, 3.0, 400)
    r = r[np.abs(r - prof.r_crit) > 0.01]
    e = 1e-5
    lhs = (prof.f(r + e) - prof.f(r - e)) / (2 * e)
    rhs = np.array([prof.dfdr(x, float(prof.f(x))) for x in r])
    assert np.max(np.abs(lhs - rhs) / (np.abs(rhs) + 0.1)) < 2e-3
    f = prof.f(r)
    assert np.all((f > 0) & (f < 1))
    # far outside the shell the field streams (f -> 1); inside it the diffuse field of
    # the shell dominates (f small)
    assert float(prof.f(3.0)) > 0.98 and float(prof.f(0.9)) < 0.1


def test_source_flux_has_divergence_j(prof):
    """F*(r) of Eq. radshell:fluxprofile against the flux of the source Eq.
    radshell:sourceprofile: (1/r^2) d(r^2 F*)/dr = j*, and 4 pi r^2 F* -> L far out."""
    r = np.linspace(0.01, 0.4, 80)
    e = 1e-6
    div = ((r + e) ** 2 * prof.F(r + e) - (r - e) ** 2 * prof.F(r - e)) / (2 * e) / r ** 2
    assert np.allclose(div, prof.j(r), rtol=1e-5, atol=1e-9 * prof.j(0.0))
    assert 4 * math.pi * 2.0 ** 2 * float(prof.F(2.0)) == pytest.approx(prof.L, rel=1e-12)


def test_cavity_energy_matches_the_eddington_model(prof):
    """Eq. radshell:Ermodel: E_Edd = (3 F*/c)(tau_sh + 2/3) with the shell's optical
    depth tau0 at r0; the M1 equilibrium inside the shell (r = 0.6 .. 0.9) agrees to 5 %."""
    E_edd = 3.0 * float(prof.F(1.0)) / prof.c * (prof.tau0 + 2.0 / 3.0)
    for r in (0.6, 0.75, 0.9):
        assert float(prof.E(r)) == pytest.approx(E_edd, rel=0.05)


def test_shell_trajectory_solves_the_reduced_ode():
    """Eqs. radshell:odepos and radshell:odevel against a numerical solution of
    r'' = M0^2 / r^2 from r = 1 at rest; the shell reaches 2 r0 near t = 0.12 t0."""
    M0 = ri.shell_parameters()["M0"]
    t = np.linspace(0.0, 0.124, 32)
    sol = solve_ivp(lambda tt, y: [y[1], M0 ** 2 / y[0] ** 2], (0.0, 0.124), [1.0, 0.0],
                    t_eval=t, rtol=1e-11, atol=1e-12)
    r, v = ri.shell_trajectory(M0, t)
    assert np.allclose(r, sol.y[0], rtol=1e-8)
    assert np.allclose(v, sol.y[1], rtol=1e-7, atol=1e-8)
    r2, _ = ri.shell_trajectory(M0, [0.12, 0.125])
    assert r2[0] < 2.0 < r2[1]
