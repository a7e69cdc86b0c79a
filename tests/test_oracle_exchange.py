"""Pins of the oracle's implicit gas-radiation energy exchange (Sec. 3.4,
Eqs. source:energyexchange to source:kappacond).

The quartic the oracle solves is checked against the theta-scheme it was derived
from (Eq. source:energyupdate, written in (e, E_r) before any elimination), the
invariant Ebar of Eq. source:combinedenergy, the equilibrium it relaxes to (solved
independently with mpmath), and the relaxation ODE Eq. source:energyexchange
integrated by scipy, including the time-step order of theta = 1 and theta = 1/2.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import rhd_inputs as ri


def alpha_of(spec, rho):
    """a_R T^4 = alpha e^4 with T = (gamma-1) e / (rho r_gas) (Eq. momenteqns:perfectgas)."""
    return spec["a_rad"] * ((spec["gamma"] - 1.0) / (rho * spec["r_gas"])) ** 4


def random_cells(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        yield dict(rho=10 ** rng.uniform(-1, 1), e=10 ** rng.uniform(-1, 1),
                   Er=10 ** rng.uniform(-2, 1), kP=10 ** rng.uniform(-1, 2),
                   dt=10 ** rng.uniform(-4, -1), c=10 ** rng.uniform(0, 4),
                   chat_frac=10 ** rng.uniform(-3, 0))


@pytest.mark.parametrize("theta", [1.0, 0.51, 0.5])
def test_root_satisfies_theta_scheme_and_conserves_ebar(theta):
    n_checked = 0
    for cell in random_cells(300, 11):
        c = cell["c"]
        chat = c * cell["chat_frac"]
        spec = ri.default_spec(c_light=c, theta_E=theta, a_rad=0.7, r_gas=1.3, gamma=1.4)
        x, Er1, it, th1, bis = oracle.exchange_cell(spec, cell["rho"], cell["e"], cell["Er"],
                                                    cell["kP"], cell["dt"], chat)
        # Eq. source:combinedenergy: e + (c/chat) E_r does not change
        eb0 = cell["e"] + (c / chat) * cell["Er"]
        assert x + (c / chat) * Er1 == pytest.approx(eb0, rel=4e-16 * 8)
        th = 1.0 if th1 else theta
        # Eq. source:energyupdate in its original two-variable form
        a = alpha_of(spec, cell["rho"])
        k = chat * cell["rho"] * cell["kP"]
        lhs = (Er1 - cell["Er"]) / cell["dt"]
        rhs = k * (th * (a * x ** 4 - Er1) + (1 - th) * (a * cell["e"] ** 4 - cell["Er"]))
        # rounding of x (relative ~1e-16) reaches E_r^{n+1} = (chat/c)(Ebar - x) scaled by
        # Ebar, and the left side divides it by dt
        scale = (k * (a * x ** 4 + Er1 + a * cell["e"] ** 4 + cell["Er"])
                 + (abs(Er1) + cell["Er"] + (chat / c) * (x + eb0)) / cell["dt"])
        assert abs(lhs - rhs) <= 1e-12 * scale
        assert x > 0.0
        n_checked += 1
    assert n_checked == 300


def test_theta_fallback_when_unbracketed():
    """Sec. 3.4: for theta < 1 a stiff cell far from equilibrium may have c0 > 0 and
    no feasible root; the oracle redoes it with theta = 1."""
    # hot gas, cold radiation, chat << c, eta = c rho kappa dt = 1000: with theta = 0.51
    # the constant term c0 = 0.49 eta (alpha e^4 - E_r) - (e + (chat/c) eta 0.51 Ebar) > 0
    spec = ri.default_spec(c_light=1.0, theta_E=0.51)
    x, Er1, it, th1, bis = oracle.exchange_cell(spec, 1.0, 1.0, 1e-3, 100.0, 10.0, 0.01)
    assert th1
    spec1 = ri.default_spec(c_light=1.0, theta_E=1.0)
    x1, Er11, *_ = oracle.exchange_cell(spec1, 1.0, 1.0, 1e-3, 100.0, 10.0, 0.01)
    assert x == x1 and Er1 == Er11
    # a mildly stiff cell keeps theta = 0.51
    _, _, _, th1b, _ = oracle.exchange_cell(spec, 1.0, 1.0, 0.15, 1.0, 0.01, 0.01)
    assert not th1b


def test_equilibrium_is_fixed_point():
    spec = ri.default_spec(c_light=50.0, theta_E=0.51)
    rho, e = 2.0, 3.0
    Er = alpha_of(spec, rho) * e ** 4
    x, Er1, *_ = oracle.exchange_cell(spec, rho, e, Er, 5.0, 0.3, 5.0)
    assert x == pytest.approx(e, rel=1e-14)
    assert Er1 == pytest.approx(Er, rel=1e-13)


def test_stiff_limit_reaches_radiative_equilibrium():
    """With theta = 1 and eta -> infinity the update lands on the equilibrium
    alpha x^4 = E_r, x + (c/chat) E_r = Ebar, found here with mpmath at 40 digits."""
    spec = ri.default_spec(c_light=100.0, theta_E=1.0)
    rho, e, Er, chat = 1.5, 0.2, 5.0, 10.0
    x, Er1, *_ = oracle.exchange_cell(spec, rho, e, Er, 1e9, 1.0, chat)
    mpmath.mp.dps = 40
    a = mpmath.mpf(alpha_of(spec, rho))
    Eb = mpmath.mpf(e) + mpmath.mpf(100.0 / chat) * mpmath.mpf(Er)
    xe = mpmath.findroot(lambda y: y + mpmath.mpf(100.0 / chat) * a * y ** 4 - Eb, 1.0)
    assert x == pytest.approx(float(xe), rel=1e-7)
    assert Er1 == pytest.approx(float(a * xe ** 4), rel=1e-6)


def test_bisection_fallback_matches_newton():
    """Forcing the bisection branch (no Newton iterations allowed) ends on the same
    root after the polishing step."""
    cell = dict(rho=1.0, e=1.0, Er=0.5, kP=3.0, dt=0.2)
    spec = ri.default_spec(c_light=10.0, theta_E=1.0)
    x0, *_ = oracle.exchange_cell(spec, cell["rho"], cell["e"], cell["Er"], cell["kP"], cell["dt"], 2.0)
    spec_b = ri.default_spec(c_light=10.0, theta_E=1.0, newton_maxit=0)
    x1, Er1, it, th1, bis = oracle.exchange_cell(spec_b, cell["rho"], cell["e"], cell["Er"], cell["kP"],
                                                 cell["dt"], 2.0)
    assert bis
    assert x1 == pytest.approx(x0, rel=1e-15)


def relax_problem(theta):
    spec = ri.default_spec(c_light=20.0, theta_E=theta, exchange="full", rad_only=True,
                           gamma=5.0 / 3.0, a_rad=1.0, r_gas=1.0)
    st = ri.uniform_state(spec, rho=1.0, P=1.0, Er=0.05, kP=0.5, kF=0.5)
    return spec, st


def relax_ode(t_end, chat):
    """Reference: Eq. source:energyexchange integrated by scipy at tight tolerance."""
    spec, st = relax_problem(1.0)
    c = spec["c_light"]
    rho, kP = 1.0, 0.5
    a = alpha_of(spec, rho)

    def rhs(_t, y):
        e, Er = y
        s = rho * kP * (a * e ** 4 - Er)
        return [-c * s, chat * s]

    e0 = float(st["E"].flat[0])
    sol = solve_ivp(rhs, (0.0, t_end), [e0, float(st["Er"].flat[0])], method="Radau",
                    rtol=1e-12, atol=1e-14)
    return sol.y[0, -1], sol.y[1, -1]


@pytest.mark.parametrize("theta,order", [(1.0, 1.0), (0.5, 2.0)])
def test_relaxation_trajectory_and_order(theta, order):
    """A uniform cell relaxes along the ODE; the error of the theta-scheme falls
    like dt for theta = 1 and like dt^2 for theta = 1/2."""
    chat, t_end = 5.0, 0.4
    e_ref, Er_ref = relax_ode(t_end, chat)
    errs = []
    for nsteps in (16, 32, 64):
        spec, st = relax_problem(theta)
        st, _ = oracle.step(spec, st, t_end / nsteps, chat, 1, steps=nsteps)
        errs.append(abs(float(st["Er"].flat[0]) - Er_ref) / Er_ref)
        # gas internal energy follows Ebar = e + (c/chat) E_r
        assert float(st["E"].flat[0]) + spec["c_light"] / chat * float(st["Er"].flat[0]) == pytest.approx(
            1.5 + spec["c_light"] / chat * 0.05, rel=1e-14)
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < (0.02 if order == 1 else 5e-4)
    for s in slopes:
        assert s == pytest.approx(order, abs=0.25)


def test_absorption_only_damps_E_with_kappa_P_and_F_with_kappa_F():
    """Absorption-only mode (Sec. 3.4): E_r decays by absorption alone, dE/dt =
    -chat rho kappa_P E (Eq. source:stiff:radenergy:soln is its theta-scheme), while F
    decays with kappa_F (Eq. source:stiff:radmomentum:soln). In a uniform box transport
    vanishes, so the subcycled result must converge to the two exponentials, at second
    order for theta = 1/2. Distinct kappa_P and kappa_F make a swap of the two opacities
    converge to the wrong rate. The gas energy is left alone in this mode."""
    spec = ri.default_spec(nx=4, dx=0.25, c_light=1.0, exchange="absorb_only", rad_only=True,
                           theta_F=0.5, bc="periodic")
    kP, kF, F0, t = 3.0, 0.5, 0.01, 0.5
    st = ri.uniform_state(spec, rho=1.0, P=1.0, Er=1.0, F=(F0, 0.0, 0.0), kP=kP, kF=kF)
    errs = []
    for steps in (16, 32, 64):
        s2, cnt = oracle.step(spec, st, t / steps, 1.0, 1, steps=steps)
        assert cnt["rad_fclamp"] == 0 and cnt["rad_efloor"] == 0
        eE = abs(float(s2["Er"].mean()) / math.exp(-kP * t) - 1.0)
        eF = abs(float(s2["Fx"].mean()) / (F0 * math.exp(-kF * t)) - 1.0)
        errs.append((eE, eF))
        assert np.array_equal(s2["E"], st["E"])
    assert errs[-1][0] < 1e-3 and errs[-1][1] < 1e-5, errs
    for a, b in zip(errs, errs[1:]):
        assert a[0] / b[0] > 3.5 and a[1] / b[1] > 3.5, errs
