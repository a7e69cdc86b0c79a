"""Pins of the oracle's single-state pieces: M1 closure (Sec. 2.3), M1 eigenvalues
(Sec. 3.3), HLL (Eq. hyperbolic:hllflux2), MC slopes and the gas Riemann solver.

Each check compares against something the paper or the mathematics fixes: printed
limits, Levermore's realizability conditions, the eigenvalues of the flux Jacobian
computed numerically, consistency and upwinding of the Riemann fluxes.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import rhd_inputs as ri

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def random_states(n, seed, fmin=0.0, fmax=1.0, c=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        E = 10.0 ** rng.uniform(-3, 3)
        f = rng.uniform(fmin, fmax)
        nh = rng.standard_normal(3)
        nh /= np.linalg.norm(nh)
        out.append((E, f * c * E * nh, f, nh))
    return out


def test_eddington_factor_printed_limits():
    g0, g1 = GOLDEN["eddington_factor_diffusion"], GOLDEN["eddington_factor_streaming"]
    assert oracle.eddington_factor(g0["f"]) == pytest.approx(g0["chi"], abs=1e-16)
    assert oracle.eddington_factor(g1["f"]) == pytest.approx(g1["chi"], abs=1e-16)


def test_eddington_factor_monotone_in_range():
    rng = GOLDEN["eddington_factor_range"]
    f = np.linspace(0.0, 1.0, 2001)
    chi = np.array([oracle.eddington_factor(x) for x in f])
    assert np.all(np.diff(chi) > 0)
    assert chi.min() >= rng["chi_min"] - 1e-16 and chi.max() <= rng["chi_max"] + 1e-16


@pytest.mark.parametrize("c", [1.0, 3.0e4])
def test_levermore_sufficient_conditions(c):
    """Eq. m1:suffconds: tr T = 1 and x.(T - f f).x >= 0 for all x; T has F along an
    eigenvector with eigenvalue chi(f) and (1 - chi)/2 across it (Eq. m1:m1tns)."""
    for E, F, f, nh in random_states(200, 1, c=c):
        P = oracle.m1_pressure(E, F, c)
        T = P / E
        assert np.trace(T) == pytest.approx(1.0, abs=1e-14)
        fv = F / (c * E)
        w = np.linalg.eigvalsh(0.5 * (T + T.T) - np.outer(fv, fv))
        assert w.min() >= -1e-13
        chi = oracle.eddington_factor(f)
        assert T @ nh == pytest.approx(chi * nh, abs=1e-13)
        perp = np.cross(nh, [1.0, 0.0, 0.0] if abs(nh[0]) < 0.9 else [0.0, 1.0, 0.0])
        perp /= np.linalg.norm(perp)
        assert T @ perp == pytest.approx(0.5 * (1 - chi) * perp, abs=1e-13)


def test_pressure_tensor_limits():
    """Sec. 2.3: diffusion limit T = I/3, streaming limit T = n n."""
    E = 2.5
    assert oracle.m1_pressure(E, [0.0, 0.0, 0.0], 1.0) == pytest.approx(E / 3 * np.eye(3), abs=1e-15)
    nh = np.array([1.0, 2.0, -2.0]) / 3.0
    P = oracle.m1_pressure(E, E * nh, 1.0)
    assert P == pytest.approx(E * np.outer(nh, nh), abs=1e-14)


def test_eigen_printed_limits():
    g = GOLDEN["eigen_diffusion_limit"]
    chat = 7.0
    for d in range(3):
        l1, l3 = oracle.m1_eigen(1.3, [0.0, 0.0, 0.0], 1.0, chat, d)
        assert l1 == pytest.approx(g["lambda1_over_chat"] * chat, rel=1e-15)
        assert l3 == pytest.approx(g["lambda3_over_chat"] * chat, rel=1e-15)
    # At f = 1 the radicand of Eq. hyperbolic:evals13 has a square-root branch point:
    # f = 1 - delta gives a radicand ~ 2 delta (1 - mu^2), so a rounding-level delta
    # (a few ulp of f) moves lambda by up to chat sqrt(2 delta) ~ 1e-7 chat.
    branch_tol = chat * math.sqrt(2.0 * 8 * np.finfo(float).eps)
    rng = np.random.default_rng(5)
    for _ in range(50):
        nh = rng.standard_normal(3)
        nh /= np.linalg.norm(nh)
        for d in range(3):
            l1, l3 = oracle.m1_eigen(2.0, 2.0 * nh, 1.0, chat, d)
            assert l1 == pytest.approx(chat * nh[d], abs=branch_tol)
            assert l3 == pytest.approx(chat * nh[d], abs=branch_tol)
    # exactly on the branch point (F along an axis, f computes to exactly 1)
    for d in range(3):
        F = [0.0, 0.0, 0.0]
        F[d] = 2.0
        assert oracle.m1_eigen(2.0, F, 1.0, chat, d) == (chat, chat)
        F[d] = -2.0
        assert oracle.m1_eigen(2.0, F, 1.0, chat, d) == (-chat, -chat)


def test_eigen_ordering_and_bound():
    """lambda_1 <= lambda_2 <= lambda_3 with lambda_2 from Eq. hyperbolic:evals2, and
    |lambda| <= chat."""
    chat = 3.0
    for E, F, f, nh in random_states(300, 2, fmin=1e-3, fmax=0.999):
        for d in range(3):
            l1, l3 = oracle.m1_eigen(E, F, 1.0, chat, d)
            mu = nh[d]
            l2 = chat * (mu / f) * (2.0 - math.sqrt(4.0 - 3.0 * f * f))
            assert l1 <= l2 + 1e-12 * chat and l2 <= l3 + 1e-12 * chat
            assert -chat * (1 + 1e-14) <= l1 and l3 <= chat * (1 + 1e-14)


def physical_flux(U, d, c, chat):
    """(chat F_d / c, chat c P_d.) from the oracle's pressure tensor."""
    P = oracle.m1_pressure(U[0], U[1:], c)
    return np.array([chat * U[1 + d] / c, chat * c * P[d, 0], chat * c * P[d, 1], chat * c * P[d, 2]])


def test_eigen_equal_extreme_eigenvalues_of_flux_jacobian():
    """Eq. hyperbolic:evals13 are the extreme eigenvalues of A = dF/dU (Eq.
    hyperbolic:linear). A is built by central differences of the flux."""
    c, chat = 2.0, 5.0
    for E, F, f, nh in random_states(60, 3, fmin=0.02, fmax=0.97, c=c):
        U = np.array([E, *F])
        for d in range(3):
            A = np.zeros((4, 4))
            for q in range(4):
                h = 1e-6 * (abs(U[q]) + 1e-3 * c * E)
                Up, Um = U.copy(), U.copy()
                Up[q] += h
                Um[q] -= h
                A[:, q] = (physical_flux(Up, d, c, chat) - physical_flux(Um, d, c, chat)) / (2 * h)
            ev = np.linalg.eigvals(A)
            assert np.abs(ev.imag).max() < 1e-5 * chat
            l1, l3 = oracle.m1_eigen(E, F, c, chat, d)
            assert ev.real.min() == pytest.approx(l1, abs=2e-6 * chat)
            assert ev.real.max() == pytest.approx(l3, abs=2e-6 * chat)


def test_hll_consistency_and_upwinding():
    c, chat = 1.5, 4.0
    for E, F, f, nh in random_states(100, 4, c=c):
        U = np.array([E, *F])
        for d in range(3):
            assert oracle.rad_hll_flux(U, U, d, c, chat) == pytest.approx(
                physical_flux(U, d, c, chat), rel=1e-13, abs=1e-13 * chat * c * E)
    # free-streaming beam along +x: S_L >= 0, so the flux is the left state's
    UL = np.array([1.0, c * 1.0, 0.0, 0.0])
    UR = np.array([0.2, c * 0.2, 0.0, 0.0])
    assert oracle.rad_hll_flux(UL, UR, 0, c, chat) == pytest.approx(physical_flux(UL, 0, c, chat),
                                                                     rel=1e-15)
    assert oracle.rad_hll_flux(UR[[0, 1, 2, 3]] * [1, -1, 1, 1], UL * [1, -1, 1, 1], 0, c,
                               chat) == pytest.approx(physical_flux(UL * [1, -1, 1, 1], 0, c, chat),
                                                      rel=1e-15)


def test_hll_diffusion_limit_closed_form():
    """Two states with F = 0: speeds are -/+ chat/sqrt 3, so Eq. hyperbolic:hllflux2
    reduces to the average flux minus (chat / (2 sqrt 3)) (U_R - U_L)."""
    c, chat = 2.0, 3.0
    UL = np.array([1.0, 0.0, 0.0, 0.0])
    UR = np.array([0.4, 0.0, 0.0, 0.0])
    s = chat / math.sqrt(3.0)
    expect = 0.5 * (physical_flux(UL, 0, c, chat) + physical_flux(UR, 0, c, chat)) - 0.5 * s * (UR - UL)
    assert oracle.rad_hll_flux(UL, UR, 0, c, chat) == pytest.approx(expect, rel=1e-14)


def test_hll_mirror_symmetry():
    c, chat = 1.0, 2.0
    rng = np.random.default_rng(6)
    for E, F, f, nh in random_states(50, 7, c=c):
        UL = np.array([E, *F])
        E2 = E * rng.uniform(0.5, 2.0)
        UR = np.array([E2, *(F * 0.7)])
        for d in range(3):
            m = np.ones(4)
            m[1 + d] = -1.0
            a = oracle.rad_hll_flux(UL, UR, d, c, chat)
            b = oracle.rad_hll_flux(UR * m, UL * m, d, c, chat)
            assert b == pytest.approx(-(a * m), rel=1e-12, abs=1e-12 * c * chat * E)


def test_mc_slope():
    assert oracle.mc_slope(1.0, -1.0) == 0.0
    assert oracle.mc_slope(0.0, 3.0) == 0.0
    assert oracle.mc_slope(1.0, 1.0) == 1.0
    assert oracle.mc_slope(1.0, 10.0) == 2.0          # limited by 2 * backward
    assert oracle.mc_slope(-10.0, -1.0) == -2.0       # limited by 2 * forward
    assert oracle.mc_slope(1.0, 2.0) == 1.5           # central difference
    rng = np.random.default_rng(8)
    for _ in range(200):
        a, b = rng.standard_normal(2)
        s = oracle.mc_slope(a, b)
        if a * b > 0:
            assert abs(s) <= 2 * min(abs(a), abs(b)) + 1e-15
            assert np.sign(s) == np.sign(a)


def test_gas_riemann_consistency_contact_and_symmetry():
    spec = ri.default_spec(gamma=1.4)
    rng = np.random.default_rng(9)
    for _ in range(50):
        W = np.array([rng.uniform(0.1, 2), *rng.uniform(-1, 1, 3), rng.uniform(0.1, 2)])
        for d in range(3):
            assert oracle.gas_riemann(spec, W, W, d) == pytest.approx(oracle.gas_flux(spec, W, d),
                                                                      rel=1e-13, abs=1e-13)
    # a stationary contact is a fixed point of HLLC: no mass or energy crosses it
    WL = np.array([1.0, 0.0, 0.3, -0.2, 1.0])
    WR = np.array([0.1, 0.0, -0.5, 0.4, 1.0])
    fl = oracle.gas_riemann(spec, WL, WR, 0)
    assert fl[0] == pytest.approx(0.0, abs=1e-15)
    assert fl[4] == pytest.approx(0.0, abs=1e-15)
    assert fl[1] == pytest.approx(1.0, rel=1e-15)
    # mirror symmetry
    WL = np.array([1.0, 0.3, 0.1, 0.2, 1.0])
    WR = np.array([0.5, -0.2, 0.0, 0.1, 0.4])
    m = np.array([1, -1, 1, 1, 1.0])
    a = oracle.gas_riemann(spec, WL, WR, 0)
    b = oracle.gas_riemann(spec, WR * m, WL * m, 0)
    assert b == pytest.approx(-(a * m), rel=1e-13, abs=1e-15)


def test_isothermal_gas_flux_is_hlle():
    spec = ri.default_spec(isothermal=True, iso_cs=0.7)
    W = np.array([1.2, 0.1, 0.0, 0.0, 0.0])
    assert oracle.gas_riemann(spec, W, W, 0)[:4] == pytest.approx(oracle.gas_flux(spec, W, 0)[:4])
    assert oracle.gas_flux(spec, W, 0)[1] == pytest.approx(1.2 * 0.01 + 1.2 * 0.49)
