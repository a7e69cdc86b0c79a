"""Oracle pins for the advection of a radiation pulse (Sec. 4.3.2), the paper's check of
the O(beta tau) terms: a pulse of radiation in pressure and radiative equilibrium with
optically thick gas (tau0 = 200, beta tau0 = 0.02), carried 2w by a uniform flow, against
the same pulse left in place. At 128 cells (a quarter of the paper's resolution) the
advected density and gas temperature stay within the paper's bounds of the static run
(6.6 % with the terms, 7.7 % without), closer with the O(beta tau) terms than without,
and gas and radiation temperatures agree at the 1e-3 level, as the paper finds."""
import numpy as np
import pytest

import oracle
import rhd_inputs as ri


def run(n, advected, beta_tau):
    pb = ri.pulse_problem(n, advected=advected, beta_tau=beta_tau)
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    t = 0.0
    while t < pb["t_end"] * (1.0 - 1e-12):
        dt, ns, _ = oracle.suggest_dt(spec, st, chat)
        dt = min(dt, pb["t_end"] - t)
        st, _ = oracle.step(spec, st, dt, chat, ns)
        t += dt
    return pb, st


@pytest.fixture(scope="module")
def pulse_errors():
    out = {}
    for bt in (True, False):
        pa, sa = run(128, True, bt)
        ps, ss = run(128, False, bt)
        Ta = ri.gas_temperature(pa["spec"], sa)[0, 0]
        Ts = ri.gas_temperature(ps["spec"], ss)[0, 0]
        Trad = (sa["Er"][0, 0] / pa["spec"]["a_rad"]) ** 0.25
        out[bt] = dict(rho=float(np.max(np.abs(sa["rho"][0, 0] / ss["rho"][0, 0] - 1.0))),
                       T=float(np.max(np.abs(Ta / Ts - 1.0))),
                       trad=float(np.max(np.abs(Trad / Ta - 1.0))),
                       moved=float(np.max(np.abs(ss["rho"][0, 0] / ps["state"]["rho"][0, 0] - 1.0))))
    return out


def test_advected_pulse_matches_the_static_pulse(pulse_errors):
    for bt, bound in ((True, 0.066), (False, 0.077)):
        e = pulse_errors[bt]
        assert e["rho"] < bound and e["T"] < bound, (bt, e)
        # the pulse itself has evolved well beyond that difference (diffusion pulls gas
        # inward), so the comparison is not trivially met
        assert e["moved"] > 4 * e["rho"], (bt, e)


def test_beta_tau_terms_bring_the_advected_pulse_closer(pulse_errors):
    on, off = pulse_errors[True], pulse_errors[False]
    assert on["rho"] < 0.9 * off["rho"] and on["T"] < 0.9 * off["T"]


def test_gas_and_radiation_stay_in_equilibrium(pulse_errors):
    for bt in (True, False):
        assert pulse_errors[bt]["trad"] < 3e-3


def test_pulse_is_the_same_in_cgs_and_code_units():
    """The problem stated in cgs and in units of w, w/a0, rho0, T0 and rho0 a0^2 (where
    a_R = P0, r_gas = 1/gamma and kappa = tau0) is one problem: five coupled gas steps
    with their subcycles give the same dimensionless density and temperature to
    rounding, and the same time steps. A constant entering in the wrong units (a_R, c,
    r_gas, the opacity) breaks this."""
    res = {}
    for units in ("cgs", "code"):
        pb = ri.pulse_problem(128, units=units)
        spec, st, chat = pb["spec"], pb["state"], pb["chat"]
        dts = []
        for _ in range(5):
            dt, ns, _ = oracle.suggest_dt(spec, st, chat)
            st, _ = oracle.step(spec, st, dt, chat, ns)
            dts.append((dt / pb["t_end"], ns))
        res[units] = (ri.gas_temperature(spec, st)[0, 0] / pb["T0"], st["rho"][0, 0] / pb["rho0"],
                      st["Er"][0, 0] / (spec["a_rad"] * pb["T0"] ** 4), dts)
    a, b = res["cgs"], res["code"]
    for k in range(3):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=0.0), k
    for (ta, na), (tb, nb) in zip(a[3], b[3]):
        assert na == nb and ta == pytest.approx(tb, rel=1e-12)
