"""Oracle pins for the Eddington (P1) closure, the alternative to M1 of Sec. 2.3
(T = I/3 whatever F is) with the wave speeds -+chat/sqrt(3) of Sec. 2.4's diffusion
limit for every state, which is the fixed-eigenvalue comparison run of the radiative
shock test (Sec. 4.3.5). Its face flux equals the M1 flux wherever F = 0; without
opacity the P1 system is the wave equation, and the oracle converges at second order to
d'Alembert's solution at amplitudes where M1 stays far from it; with a scattering
opacity it follows the exact telegraph solution at any amplitude; and, as Sec. 2.3
says, it lets the beam of the shadow test flow round the cloud."""
import math

import numpy as np
import pytest

import oracle
import rhd_inputs as ri
from test_oracle_physics import telegraph_solution


def test_p1_flux_is_the_m1_flux_where_the_flux_vanishes():
    """M1's closure at f = 0 is T = I/3 with speeds -+chat/sqrt(3) (pinned to the
    paper's printed limits elsewhere), so with F = 0 on both sides the two fluxes agree;
    with F != 0 they differ; and the P1 flux of two equal states is the physical flux
    (chat F_d/c, chat c E_r/3 along d)."""
    rng = np.random.default_rng(3)
    c, chat = 3.0, 2.0
    for d in range(3):
        for _ in range(20):
            EL, ER = rng.uniform(0.1, 5.0, 2)
            UL, UR = np.array([EL, 0.0, 0.0, 0.0]), np.array([ER, 0.0, 0.0, 0.0])
            a = oracle.p1_hll_flux(UL, UR, d, c, chat)
            b = oracle.rad_hll_flux(UL, UR, d, c, chat)
            assert np.allclose(a, b, rtol=1e-14, atol=1e-14 * max(EL, ER) * c * chat)
        U = np.array([2.0, 1.5, -0.7, 0.4])
        phys = np.zeros(4)
        phys[0] = chat * U[1 + d] / c
        phys[1 + d] = chat * c * U[0] / 3.0
        assert np.allclose(oracle.p1_hll_flux(U, U, d, c, chat), phys, rtol=1e-15)
        assert not np.allclose(oracle.p1_hll_flux(U, U, d, c, chat),
                               oracle.rad_hll_flux(U, U, d, c, chat), rtol=1e-3)


def pulse_run(closure, N, t, rk=0.0, A=10.0, sig=0.05):
    """Periodic [0, 1), c = chat = 1, no exchange, E_r = 1 + A g(x) with a Gaussian g
    of width sig about x = 1/2, F = 0, CFL 0.4."""
    spec = ri.default_spec(nx=N, dx=1.0 / N, c_light=1.0, exchange="none", rad_only=True,
                           theta_F=0.51, bc="periodic", closure=closure)
    st = ri.uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=0.0, kF=rk)
    x = (np.arange(N) + 0.5) / N

    def g(y):
        return np.exp(-((((y - 0.5) + 0.5) % 1.0 - 0.5) ** 2) / (2 * sig ** 2))

    st["Er"][0, 0, :] = 1.0 + A * g(x)
    steps = int(math.ceil(t / (0.4 / N)))
    out, cnt = oracle.step(spec, st, t / steps, 1.0, 1, steps=steps)
    return x, st["Er"][0, 0].copy(), out, cnt, g


def test_p1_converges_to_dalembert_where_m1_does_not():
    """Without opacity, dE/dt = -chat dG/dx and dG/dt = -(chat/3) dE/dx (G = F/c): the
    pulse splits into halves moving at -+chat/sqrt(3), E = 1 + (A/2)(g(x - vt) +
    g(x + vt)) and F = c (A/2)(g(x - vt) - g(x + vt))/sqrt(3). With A = 10 the halves
    reach f ~ 0.5; the P1 error falls about fourfold per doubling of N, while M1 (a
    different, nonlinear system there) stays ~100x further away."""
    t, v, A = 0.25, 1.0 / math.sqrt(3.0), 10.0
    errs = {}
    for closure in ("p1", "m1"):
        errs[closure] = []
        for N in (64, 128, 256):
            x, _, out, cnt, g = pulse_run(closure, N, t, A=A)
            Eex = 1.0 + 0.5 * A * (g(x - v * t) + g(x + v * t))
            Fex = 0.5 * A * (g(x - v * t) - g(x + v * t)) / math.sqrt(3.0)
            errs[closure].append(np.abs(out["Er"][0, 0] - Eex).mean()
                                 + np.abs(out["Fx"][0, 0] - Fex).mean())
            assert cnt["rad_fclamp"] == 0
    p1 = errs["p1"]
    assert p1[0] / p1[1] > 3.5 and p1[1] / p1[2] > 3.5 and p1[2] < 5e-3
    assert min(errs["m1"]) > 100 * p1[2]


@pytest.mark.parametrize("rk", [5.0, 20.0])
def test_p1_follows_the_telegraph_solution_at_large_amplitude(rk):
    """With a scattering opacity rho kappa_F = rk the P1 system is linear at every
    amplitude: the exact Fourier solution holds for the pulse of amplitude 10, and the
    oracle converges to it at second order. M1 at the same amplitude differs by a fixed
    amount."""
    errs = {}
    for closure in ("p1", "m1"):
        errs[closure] = []
        for N in (128, 256):
            _, E0, out, _, _ = pulse_run(closure, N, 0.2, rk=rk)
            tel = telegraph_solution(E0, rk, 1.0, 0.2)
            errs[closure].append(np.abs(out["Er"][0, 0] - tel).sum() / np.abs(tel).sum())
    assert errs["p1"][1] < 3e-4 and errs["p1"][0] / errs["p1"][1] > 3.5
    assert errs["m1"][1] > 30 * errs["p1"][1]


def test_p1_lets_the_beam_flow_round_the_cloud():
    """Sec. 2.3: an isotropic closure lets directed radiation leak round an obstruction.
    In the coarse shadow test after three light-crossing times, M1 leaves the right
    boundary behind the cloud below 0.15 T1 while P1 leaves it as bright as above the
    cloud."""
    Tr = {}
    for closure in ("m1", "p1"):
        pb = ri.shadow_problem(56, 16, emission=False)
        spec = dict(pb["spec"], closure=closure)
        steps = int(math.ceil(3 * pb["crossing"] / pb["dt"]))
        st, _ = oracle.step(spec, pb["state"], pb["dt"], pb["chat"], 1, steps=steps)
        y = (np.arange(16) + 0.5) * spec["dy"]
        T = ri.radiation_temperature(st["Er"][0, :, -1]) / pb["T1"]
        Tr[closure] = (T[y < 0.045], T[y > 0.08])
        assert np.all(np.isfinite(st["Er"]))
    assert np.all(Tr["m1"][0] < 0.15) and np.all(Tr["m1"][1] > 0.95)
    assert np.all(Tr["p1"][0] > 0.9) and np.all(np.abs(Tr["p1"][0] - Tr["p1"][1].mean()) < 0.05)
