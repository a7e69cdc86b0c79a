"""Oracle pins for the opacity law kappa(T_gas, rho) and the shadow test of Sec. 4.1.1:
the law against the relaxation ODE it defines, the M1 shadow behind a dense cloud
(sharp without emission, softer with it, as the paper finds), the floor on
reconstructed face states that keeps cells next to the floor finite, and the floor on
E_r after an ill-conditioned exchange."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import rhd_inputs as ri


def relax_spec(law):
    return ri.default_spec(nx=4, dx=0.25, c_light=1.0, a_rad=1.0, r_gas=1.0, gamma=5.0 / 3.0,
                           rad_only=True, exchange="full", theta_E=1.0, bc="periodic",
                           kappa_law=law)


def relax_oracle(law, rho, e0, Er0, t_end, n):
    spec = relax_spec(law)
    st = ri.uniform_state(spec, rho=rho, P=1.0, Er=Er0, kP=1.0, kF=1.0)
    st["E"] = np.full_like(st["rho"], e0)
    st, _ = oracle.step(spec, st, t_end / n, 1.0, 0, steps=n)
    return float(st["E"][0, 0, 0]), float(st["Er"][0, 0, 0])


def relax_ode(law, rho, e0, Er0, t_end):
    """de/dt = -c rho kappa (a_R T^4 - E_r), dE_r/dt = +chat rho kappa (a_R T^4 - E_r)
    with T = (gamma - 1) e / (rho r_gas) and kappa = k0 (T/T0)^a (rho/rho0)^b."""
    k0, T0, rho0, a, b = law

    def rhs(_, y):
        e, Er = y
        T = (2.0 / 3.0) * e / rho
        kap = k0 * (T / T0) ** a * (rho / rho0) ** b
        s = rho * kap * (T ** 4 - Er)
        return [-s, s]

    sol = solve_ivp(rhs, (0.0, t_end), [e0, Er0], method="Radau", rtol=1e-11, atol=1e-14)
    return sol.y[0, -1], sol.y[1, -1]


@pytest.mark.parametrize("law", [(1.0, 1.0, 1.0, -3.5, 1.0), (0.5, 2.0, 0.5, 1.5, -0.5)])
def test_opacity_law_follows_the_relaxation_ode(law):
    """Gas and radiation relax with the opacity the law gives at the gas temperature of
    each step. With theta = 1 and the opacity held over a step the scheme is first
    order: its error against the ODE halves with the step. A wrong exponent, base or
    density factor changes the ODE and does not converge to it."""
    rho, e0, Er0, t_end = 2.0, 3.0, 3.0, 0.4
    ref = relax_ode(law, rho, e0, Er0, t_end)
    errs = []
    for n in (20, 40, 80):
        e, Er = relax_oracle(law, rho, e0, Er0, t_end, n)
        errs.append(abs(e - ref[0]) + abs(Er - ref[1]))
        assert e + Er == pytest.approx(e0 + Er0, rel=1e-13)
    assert errs[2] < 0.02 * abs(e0 - ref[0])
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


def shadow_run(emission, crossings=3.0, n=(56, 16), theta_F=None, steps=None):
    pb = ri.shadow_problem(*n, emission=emission)
    spec = dict(pb["spec"])
    if theta_F is not None:
        spec["theta_F"] = theta_F
    if steps is None:
        steps = int(math.ceil(crossings * pb["crossing"] / pb["dt"]))
    st, cnt = oracle.step(spec, pb["state"], pb["dt"], pb["chat"], 1, steps=steps)
    y = (np.arange(n[1]) + 0.5) * spec["dy"]
    return pb, st, y, cnt


@pytest.fixture(scope="module")
def shadows():
    return {em: shadow_run(em) for em in (False, True)}


def test_m1_casts_a_sharp_shadow_without_emission(shadows):
    """Sec. 4.1.1: the beam passes the thin ambient gas (tau = 0.1 across the box) and
    the cloud (tau ~ 10^2 per cell) stops it. At the right boundary after three
    light-crossing times the radiation temperature is T1 within the ambient absorption
    above the cloud and far below it in the cloud's shadow (|y| < 0.06), with the
    transition at the cloud's edge."""
    pb, st, y, _ = shadows[False]
    Tr = ri.radiation_temperature(st["Er"][0, :, -1]) / pb["T1"]
    assert np.all(Tr[y > 0.08] > 0.95)
    assert np.all(Tr[y < 0.045] < 0.15)
    assert np.all(np.isfinite(st["Er"])) and np.all(st["Er"] > 0)


def test_emission_softens_the_shadow(shadows):
    """With thermal emission the exchange, split from transport, gives back as
    isotropic radiation the beam energy the cloud's surface cells take up during a step
    (the paper puts the softer shadow down to this operator-split implicit solver), so
    the shadow is brighter and less sharp than without emission, yet still darker than
    the lit region."""
    pb0, st0, y, _ = shadows[False]
    pb1, st1, _, cnt = shadows[True]
    T0 = ri.radiation_temperature(st0["Er"][0, :, -1]) / pb0["T1"]
    T1 = ri.radiation_temperature(st1["Er"][0, :, -1]) / pb1["T1"]
    shade = y < 0.045
    assert np.all(T1[shade] > 2.0 * T0[shade])
    assert T1[-1] > 0.9 and np.all(T1[shade] < T1[-1] - 0.3)
    assert cnt["newton_iters"] > 0


def test_face_states_next_to_the_floor_stay_finite():
    """A theta near 1/2 lets the cloud's strong absorption drive E_r below zero, so cells
    sit at the floor next to lit cells; the reconstructed face state between them would
    round to E_r = 0, where the closure is 0/0. The floor on face states keeps every
    value finite."""
    pb, st, _, cnt = shadow_run(False, theta_F=0.51, steps=60)
    assert cnt["rad_efloor"] > 0
    for k in ("Er", "Fx", "Fy"):
        assert np.all(np.isfinite(st[k])), k


def cold_gas_spec(nx=8, ny=6):
    return ri.default_spec(nx=nx, ny=ny, dx=0.1, dy=0.1, c_light=ri.C_CGS, a_rad=ri.A_RAD_CGS,
                           r_gas=ri.R_GAS_CGS, gamma=5.0 / 3.0, rad_only=True, exchange="full",
                           theta_E=1.0, bc="periodic", er_floor=1e-30)


# gas at T = 1 K, rho = 1 in cgs: e = 1.24e8 erg/cm^3, whose spacing is 1.5e-8
COLD_E = ri.R_GAS_CGS * 1.0 / (2.0 / 3.0)


@pytest.mark.parametrize("Er", [1e-12, 1e-8])
def test_exchange_that_rounds_the_radiation_away_is_floored(Er):
    """Eq. source:kappacond: E_r from Eq. source:eradupdate carries a relative error of
    about K eps, with K = e / ((c/chat) E_r) ~ 1e20 here, so it rounds to one spacing of
    e below zero (E_r = 1e-12) or to exactly zero (1e-8). After the exchange E_r is
    raised to the floor (a step without radiation subcycles shows the exchange alone);
    the stage that follows keeps it there, with |F| <= c E_r, and every value stays
    finite; the combined energy e + (c/chat) E_r changes by less than one spacing of e."""
    spec = cold_gas_spec()
    c = spec["c_light"]
    st = ri.uniform_state(spec, rho=1.0, P=ri.R_GAS_CGS, Er=Er, F=(c * Er, 0.0, 0.0),
                          kP=1.0, kF=1.0)
    e0 = float(st["E"][0, 0, 0])
    assert e0 == pytest.approx(COLD_E, rel=1e-15)
    x, Er_raw, *_ = oracle.exchange_cell(spec, 1.0, e0, Er, 1.0, 1e-12, c)
    assert Er_raw <= 0.0
    ex, _ = oracle.step(spec, st, 1e-12, c, 0)
    assert np.all(ex["Er"] == spec["er_floor"])
    assert np.all(ex["E"] == x)
    out, cnt = oracle.step(spec, st, 1e-12, c, 1)
    for k in ("Er", "Fx", "Fy", "E"):
        assert np.all(np.isfinite(out[k])), k
    assert np.all(out["Er"] == spec["er_floor"])
    assert np.all(np.abs(out["Fx"]) <= c * out["Er"] * (1 + 1e-15))
    total = lambda s: s["E"] + s["Er"]  # chat = c
    assert np.all(np.abs(total(out) - total(st)) <= 2 * np.spacing(COLD_E))
