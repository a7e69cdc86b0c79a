"""The linear system of gray radiation hydrodynamics about a static equilibrium
(Sec. 4.3.4), derived by the tests from Eq. mixedframe:graysystem; shared by the oracle
pins and the GPU checks of the linear-perturbation box."""
import math

import numpy as np
from scipy.linalg import expm


def linear_rhd_matrix(k, g, P0, C, Ch, tau, b):
    """d/dt of (d rho, d v, d p, d E_r, G = dF/c) for a perturbation exp(i k x) about
    a static equilibrium (rho0 = a0 = 1, a_R T0^4 = P0), linearised from
    Eq. mixedframe:graysystem with the closure at f = 0 (P = E_r / 3) and the
    simplified O(beta tau) term of Eq. m1:simplifiedsource switched by b."""
    ik = 1j * k
    bt = b * (4.0 / 3.0) * tau * P0 / C
    A = np.zeros((5, 5), complex)
    A[0, 1] = -ik
    A[1, 1] = -bt
    A[1, 2] = -ik
    A[1, 4] = tau
    A[2, 0] = (g - 1) * C * tau * 4 * P0
    A[2, 1] = -ik
    A[2, 2] = -(g - 1) * C * tau * 4 * P0 * g
    A[2, 3] = (g - 1) * C * tau
    A[3, 0] = -Ch * tau * 4 * P0
    A[3, 2] = Ch * tau * 4 * P0 * g
    A[3, 3] = -Ch * tau
    A[3, 4] = -Ch * ik
    A[4, 1] = Ch * bt
    A[4, 3] = -Ch * ik / 3.0
    A[4, 4] = -Ch * tau
    return A


def c2_mode_prediction(spec, chat, kappa, t, R0, E0, n_vec):
    """Linear-theory prediction of the Fourier coefficients of (rho - 1, E_r - 1) at
    time t for the wavevector n_vec (integer, in units of 2 pi / box side) of a box at
    rho = 1, P = 1, E_r = a_R T^4 = 1 with initial coefficients R0, E0 and v = F = P' = 0.
    Units: rho0, a0 = sqrt(gamma P / rho), box side 1, so P0 = 1/gamma, C = c/a0,
    Chat = chat/a0, tau = kappa rho L; pressures and E_r in units of rho0 a0^2."""
    g = spec["gamma"]
    a0 = math.sqrt(g)
    k = 2 * math.pi * math.sqrt(sum(q * q for q in n_vec))
    A = linear_rhd_matrix(k, g, 1.0 / g, spec["c_light"] / a0, chat / a0, kappa, 0)
    u1 = expm(A * t * a0) @ np.array([R0, 0.0, 0.0, E0 / g, 0.0], dtype=complex)
    return u1[0], u1[3] * g
