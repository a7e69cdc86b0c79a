"""Seeded synthetic inputs for the gray M1 radiation-hydrodynamics step.

This module only builds problem descriptions and initial arrays: it holds none of
the method's arithmetic (no closure, no fluxes, no time-step rule). Both the
oracle and the GPU library are fed from here.

A problem is a dict:

  spec   -- grid, constants, switches (see ``default_spec``);
  state  -- float64 arrays of shape (nz, ny, nx), C order, so that the flat cell
            index is i + nx*(j + ny*k): rho, mx, my, mz, E, Er, Fx, Fy, Fz,
            kP, kF (specific opacities) and optionally j (emissivity);
  chat   -- reduced speed of light used by the steps;
  dt, nsub, steps -- time stepping when the recipe fixes it (dt None means
            "take the CFL step of the current state").

Nondimensional code units throughout; r_gas = k_B/mu and a_R are part of spec.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("rho", "mx", "my", "mz", "E", "Er", "Fx", "Fy", "Fz")
BASE_SEED = 20130601


def default_spec(**over):
    spec = dict(
        nx=1, ny=1, nz=1,
        dx=1.0, dy=1.0, dz=1.0,
        gamma=5.0 / 3.0,
        c_light=1.0, a_rad=1.0, r_gas=1.0,
        iso_cs=1.0,
        cfl=0.4,
        theta_E=1.0, theta_F=0.51,
        newton_rtol=1e-10, newton_maxit=50,
        rho_floor=1e-10, p_floor=1e-14, er_floor=1e-30,
        bc=("periodic",) * 6,
        isothermal=False,
        exchange="full",          # "full" | "absorb_only" | "none"
        beta_tau=False,
        rad_only=False,
        precision="fp64",         # "fp64" | "mixed"
        cv_t3=False,              # gas heat capacity c_v = cv_alpha T^3 (Marshak problem)
        cv_alpha=0.0,
        bvals=((0.0,) * 4,) * 6,  # (E_r, F_x, F_y, F_z) of each "fixed" face
        kappa_law=None,           # (k0, T0, rho0, a, b): kappa = k0 (T/T0)^a (rho/rho0)^b
        closure="m1",             # "m1" | "p1" (Eddington: T = I/3, speeds -+chat/sqrt(3))
    )
    for k, v in over.items():
        if k not in spec:
            raise KeyError(f"unknown spec key {k!r}")
        spec[k] = v
    if isinstance(spec["bc"], str):
        spec["bc"] = (spec["bc"],) * 6
    return spec


def _zeros(spec):
    return np.zeros((spec["nz"], spec["ny"], spec["nx"]), dtype=np.float64)


def cell_centres(spec, origin=(0.0, 0.0, 0.0)):
    """Cell-centre coordinates (x, y, z) broadcast to shape (nz, ny, nx)."""
    x = origin[0] + (np.arange(spec["nx"]) + 0.5) * spec["dx"]
    y = origin[1] + (np.arange(spec["ny"]) + 0.5) * spec["dy"]
    z = origin[2] + (np.arange(spec["nz"]) + 0.5) * spec["dz"]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def uniform_state(spec, rho=1.0, P=1.0, v=(0.0, 0.0, 0.0), Er=1.0, F=(0.0, 0.0, 0.0),
                  kP=1.0, kF=1.0):
    """Uniform gas and radiation; E is the ideal-gas total energy for pressure P."""
    s = {k: _zeros(spec) for k in FIELDS}
    s["rho"][:] = rho
    s["mx"][:] = rho * v[0]
    s["my"][:] = rho * v[1]
    s["mz"][:] = rho * v[2]
    ke = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    s["E"][:] = (P / (spec["gamma"] - 1.0) if not spec["isothermal"] else 0.0) + ke
    s["Er"][:] = Er
    s["Fx"][:] = F[0]
    s["Fy"][:] = F[1]
    s["Fz"][:] = F[2]
    s["kP"] = np.full_like(s["rho"], kP)
    s["kF"] = np.full_like(s["rho"], kF)
    return s


def copy_state(state):
    return {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v)
            for k, v in state.items()}


def random_phase_field(shape, kmin, kmax, rms, rng):
    """Real periodic field: unit-amplitude Fourier modes with integer wavevectors
    kmin <= |k| <= kmax and uniform random phases, scaled to the given RMS."""
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz, 1.0 / nz)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kk = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    mask = (kk >= kmin) & (kk <= kmax)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=kk.shape)
    coef = np.where(mask, np.exp(1j * phase), 0.0)
    field = np.fft.irfftn(coef, s=shape, axes=(0, 1, 2))
    cur = float(np.sqrt(np.mean(field ** 2)))
    return field * (rms / cur) if cur > 0 else field


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def c1_diffusion(n=256):
    """1D radiation-only M1 diffusion in a periodic unit box: scattering-dominated
    static gas (rho kappa_F = 100, no absorption), chat = c = 1, Gaussian pulse
    E_r = 1e-6 + exp(-(x-1/2)^2 / (2 0.05^2)), F = 0, CFL 0.4, to t = 0.05."""
    spec = default_spec(nx=n, dx=1.0 / n, c_light=1.0, exchange="none", rad_only=True,
                        theta_F=0.51, bc="periodic")
    st = uniform_state(spec, rho=1.0, P=1.0, Er=0.0, kP=0.0, kF=100.0)
    X, _, _ = cell_centres(spec)
    st["Er"][:] = 1e-6 + np.exp(-((X - 0.5) ** 2) / (2 * 0.05 ** 2))
    dt = 0.4 * spec["dx"] / 1.0
    steps = int(round(0.05 / dt))
    return dict(name="c1_diffusion_1d", spec=spec, state=st, chat=1.0, dt=dt, nsub=1,
                steps=steps, t_end=0.05, sigma0=0.05, D=1.0 / 300.0)


def c2_linear_box(n=128, seed=BASE_SEED + 1, precision="mixed", beta_tau=False):
    """3D RHD linear-perturbation box: periodic n^3 on [0,1)^3, rho = 1, P = 1,
    gamma = 5/3, E_r = a_R T^4 = 1, kappa_P = kappa_F = 10, a0 = sqrt(5/3),
    chat = 20 a0, c = 1e4 a0; random-phase perturbations of RMS 1e-4 in rho and E_r
    over integer wavenumbers 1..8; 10 gas steps with chat-limited subcycles."""
    a0 = math.sqrt(5.0 / 3.0)
    spec = default_spec(nx=n, ny=n, nz=n, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n,
                        gamma=5.0 / 3.0, c_light=1e4 * a0, a_rad=1.0, r_gas=1.0,
                        exchange="full", beta_tau=beta_tau, precision=precision,
                        theta_E=1.0, theta_F=0.51, bc="periodic")
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=10.0, kF=10.0)
    rng = np.random.default_rng(seed)
    shape = st["rho"].shape
    drho = random_phase_field(shape, 1, 8, 1e-4, rng)
    dEr = random_phase_field(shape, 1, 8, 1e-4, rng)
    st["rho"] += drho
    st["Er"] += dEr
    return dict(name=f"c2_rhd_linear_box_{n}cubed", spec=spec, state=st, chat=20.0 * a0,
                dt=None, nsub=None, steps=10)


def c3_point_source(n=256, precision="mixed"):
    """3D concentrated source: n^3 on [0,1)^3 with outflow faces, static gas,
    rho = 1 + 1e3 exp(-r^2/(2 sigma^2)) with sigma = 8 cells about the centre,
    emissivity j = 1 in the central 4^3 cells, kappa_P = 0 (no exchange),
    kappa_F = 1.2766 (core column ~ 50), c = chat = 1, E_r = 1e-10, F = 0,
    theta_F = 1, 200 radiation subcycles of CFL 0.4."""
    h = 1.0 / n
    spec = default_spec(nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, c_light=1.0,
                        exchange="none", rad_only=True, theta_F=1.0, bc="outflow",
                        precision=precision)
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1e-10, kP=0.0, kF=1.2766)
    X, Y, Z = cell_centres(spec)
    sig = 8.0 * h
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2
    st["rho"][:] = 1.0 + 1e3 * np.exp(-r2 / (2 * sig ** 2))
    st["mx"][:] = 0.0
    jj = np.zeros_like(st["rho"])
    c0 = n // 2 - 2
    jj[c0:c0 + 4, c0:c0 + 4, c0:c0 + 4] = 1.0
    st["j"] = jj
    return dict(name=f"c3_point_source_{n}cubed", spec=spec, state=st, chat=1.0,
                dt=0.4 * h, nsub=1, steps=200)


def c4_dusty_shell(n=256, seed=BASE_SEED + 4, precision="mixed"):
    """3D dusty shell: n^3 on [-1/2,1/2)^3 with outflow faces, isothermal gas
    (c_s = 1), radiative equilibrium (no exchange). Gaussian shell of radius 0.3
    and FWHM 0.05 with seeded lognormal density (sigma_ln rho = 1) so that the shell
    column gives tau ~ 20 at kappa = 1; central Gaussian source j of width 2 cells
    and luminosity set so that L kappa / (4 pi 0.3^2 c) = 20; c = 1e4; chat is 20x
    the initial signal speed and stays fixed. The log-density is a Gaussian random
    field of unit RMS made of random-phase modes with integer wavenumbers 2 .. n/8
    (at least 4), so it varies over eight cells or more."""
    h = 1.0 / n
    spec = default_spec(nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, c_light=1e4, iso_cs=1.0,
                        isothermal=True, exchange="none", theta_F=1.0, bc="outflow",
                        precision=precision)
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1e-10, kP=1.0, kF=1.0)
    X, Y, Z = cell_centres(spec, origin=(-0.5, -0.5, -0.5))
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    sig_sh = 0.05 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    smooth = 1.0 + 375.8 * np.exp(-((r - 0.3) ** 2) / (2 * sig_sh ** 2))
    rng = np.random.default_rng(seed)
    g = random_phase_field(smooth.shape, 2, max(4, n // 8), 1.0, rng)
    lognorm = np.exp(1.0 * g - 0.5)
    rho = np.where(smooth > 2.0, smooth * lognorm, smooth)
    st["rho"][:] = rho
    st["E"][:] = 0.0
    sig_s = 2.0 * h
    L = 20.0 * 4.0 * math.pi * 0.3 ** 2 * spec["c_light"] / 1.0
    st["j"] = L * np.exp(-(r ** 2) / (2 * sig_s ** 2)) / ((2 * math.pi) ** 1.5 * sig_s ** 3)
    return dict(name=f"c4_dusty_shell_{n}cubed", spec=spec, state=st, chat=None,
                dt=None, nsub=None, steps=100, chat_over_vmax=20.0)


def c5_requests(count=512, seed=BASE_SEED + 5, sizes=tuple(range(32, 193, 16)),
                load=1.2):
    """Served batch: a Poisson stream of independent periodic linear-perturbation
    boxes (as in the 3D box above) with nx, ny, nz iid uniform over 32..192 step 16,
    kappa_P = kappa_F log-uniform in [1, 1e3], chat/a0 uniform in [5, 50] and 20 gas
    steps each. Returns per-request recipes; arrival times are in units of the
    caller's measured single-stream service time times 1/load."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(count):
        nx, ny, nz = (int(rng.choice(sizes)) for _ in range(3))
        kappa = float(10.0 ** rng.uniform(0.0, 3.0))
        chat_over_a0 = float(rng.uniform(5.0, 50.0))
        t += float(rng.exponential(1.0 / load))
        reqs.append(dict(id=r, nx=nx, ny=ny, nz=nz, kappa=kappa,
                         chat_over_a0=chat_over_a0, steps=20, arrival=t,
                         seed=int(rng.integers(0, 2 ** 31 - 1))))
    return reqs


def c5_perturbations(req):
    """The seeded density and E_r perturbations of one served request (random-phase
    modes over integer wavenumbers 1..8, RMS 1e-4 each), shape (nz, ny, nx)."""
    shape = (req["nz"], req["ny"], req["nx"])
    rng = np.random.default_rng(req["seed"])
    drho = random_phase_field(shape, 1, 8, 1e-4, rng)
    dEr = random_phase_field(shape, 1, 8, 1e-4, rng)
    return drho, dEr


def c5_spec(req, precision="mixed"):
    a0 = math.sqrt(5.0 / 3.0)
    nx, ny, nz = req["nx"], req["ny"], req["nz"]
    return default_spec(nx=nx, ny=ny, nz=nz, dx=1.0 / nx, dy=1.0 / ny, dz=1.0 / nz,
                        gamma=5.0 / 3.0, c_light=1e4 * a0, exchange="full",
                        precision=precision, bc="periodic")


def c5_problem(req, precision="mixed", perturbations=None, compact=False):
    """The initial state of one served request (see ``c5_requests``). With compact, the
    uniform fields are scalars (broadcast by the consumers) instead of full arrays."""
    a0 = math.sqrt(5.0 / 3.0)
    spec = c5_spec(req, precision)
    drho, dEr = c5_perturbations(req) if perturbations is None else perturbations
    if compact:
        st = {"rho": 1.0 + drho, "mx": 0.0, "my": 0.0, "mz": 0.0,
              "E": 1.0 / (spec["gamma"] - 1.0), "Er": 1.0 + dEr, "Fx": 0.0, "Fy": 0.0,
              "Fz": 0.0, "kP": np.array([req["kappa"]]), "kF": np.array([req["kappa"]])}
    else:
        st = uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=req["kappa"], kF=req["kappa"])
        st["rho"] += drho
        st["Er"] += dEr
    return dict(name=f"c5_request_{req['id']}", spec=spec, state=st,
                chat=req["chat_over_a0"] * a0, dt=None, nsub=None, steps=req["steps"])


# --------------------------------------------------------------------------
# small problems for the checks
# --------------------------------------------------------------------------

def smooth_random_state(spec, seed, amp=0.1, Er0=1.0, f_amp=0.3, kappa=(1.0, 1.0),
                        v_amp=0.0, with_j=False):
    """A smooth, positive, sub-luminal random state for parity checks: each field is
    a background plus a few random-phase low modes."""
    rng = np.random.default_rng(seed)
    shape = (spec["nz"], spec["ny"], spec["nx"])
    kmax = max(2, min(shape) // 4) if min(shape) > 1 else 2

    def pert(a):
        if max(shape) == 1:
            return np.zeros(shape)
        return random_phase_field(shape, 1, kmax, a, rng)

    st = {}
    st["rho"] = 1.0 + pert(amp)
    v = [v_amp * pert(1.0) for _ in range(3)]
    P = 1.0 + pert(amp)
    st["mx"], st["my"], st["mz"] = (st["rho"] * vv for vv in v)
    ke = 0.5 * st["rho"] * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    st["E"] = (P / (spec["gamma"] - 1.0) if not spec["isothermal"] else 0.0) + ke
    st["Er"] = Er0 * (1.0 + pert(amp))
    c = spec["c_light"]
    for q in ("Fx", "Fy", "Fz"):
        st[q] = f_amp * c * st["Er"] * pert(1.0) / math.sqrt(3.0)
    st["kP"] = kappa[0] * (1.0 + pert(0.5 * amp))
    st["kF"] = kappa[1] * (1.0 + pert(0.5 * amp))
    if with_j:
        st["j"] = np.abs(pert(1.0))
    for k in st:
        st[k] = np.ascontiguousarray(st[k], dtype=np.float64)
    return st


def radiation_wave(dim, N, eps=1e-6, tau_lambda=0.1, theta_F=0.5):
    """Free-streaming damped radiation plane wave (streaming limit, f = 1) in a
    purely absorbing medium: 1D along x on [0, lambda); 2D on 2L x L with the wave
    vector at atan(2) in the xy-plane; 3D on 2L x L x L at atan(2) in-plane and
    atan(2/sqrt5) out of plane. lambda = 1, c = chat = 1, rho = 1,
    kappa = tau_lambda. Background E = 1 with F = c E n, perturbation eps (1, c n)."""
    lam = 1.0
    if dim == 1:
        alpha, beta, L = 0.0, 0.0, lam
        n3 = (N, 1, 1)
        ext = (L, 1.0, 1.0)
    elif dim == 2:
        alpha, beta, L = 0.0, math.atan(2.0), math.sqrt(5.0) / 2.0 * lam
        n3 = (2 * N, N, 1)
        ext = (2 * L, L, 1.0)
    else:
        alpha, beta, L = math.atan(2.0 / math.sqrt(5.0)), math.atan(2.0), 1.5 * lam
        n3 = (2 * N, N, N)
        ext = (2 * L, L, L)
    spec = default_spec(nx=n3[0], ny=n3[1], nz=n3[2], dx=ext[0] / n3[0],
                        dy=ext[1] / n3[1], dz=ext[2] / n3[2], c_light=1.0,
                        exchange="absorb_only", rad_only=True, theta_F=theta_F,
                        bc="periodic")
    nhat = np.array([math.cos(alpha) * math.cos(beta), math.cos(alpha) * math.sin(beta),
                     math.sin(alpha)])
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=tau_lambda / lam,
                       kF=tau_lambda / lam)
    X, Y, Z = cell_centres(spec)
    xp = X * nhat[0] + Y * nhat[1] + Z * nhat[2]
    E = 1.0 + eps * np.sin(2 * math.pi * xp / lam)
    st["Er"] = E
    st["Fx"] = E * nhat[0]
    st["Fy"] = E * nhat[1]
    st["Fz"] = E * nhat[2]
    widths = [spec["dx"], spec["dy"], spec["dz"]][:dim]
    return dict(name=f"radiation_wave_{dim}d_{N}", spec=spec, state=st, chat=1.0,
                nhat=nhat, lam=lam, eps=eps, tau_lambda=tau_lambda,
                t_end=lam / 1.0, dt=0.4 * min(widths))


def sod_tube(N=200, gamma=1.4):
    """Sod shock tube on [0,1) with outflow ends, radiation decoupled (kappa = 0,
    no exchange, negligible E_r): left rho = 1, P = 1; right rho = 0.125, P = 0.1."""
    spec = default_spec(nx=N, dx=1.0 / N, gamma=gamma, c_light=1.0, exchange="none",
                        bc="outflow", theta_F=1.0)
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1e-20, kP=0.0, kF=0.0)
    X, _, _ = cell_centres(spec)
    left = X < 0.5
    st["rho"] = np.where(left, 1.0, 0.125)
    P = np.where(left, 1.0, 0.1)
    st["E"] = P / (gamma - 1.0)
    return dict(name=f"sod_{N}", spec=spec, state=st, chat=1.0, t_end=0.2)


# --------------------------------------------------------------------------
# non-equilibrium Marshak wave (Sec. 4.1.3): the paper's own timing problem
# --------------------------------------------------------------------------

def _su_olson_integrands(chi, tau, eps):
    """The two integrands of the semi-analytic Su & Olson solution quoted in
    Sec. 4.1.3 (Eq. marshak:suolson), as functions of eta in (0, 1)."""
    def gam_theta(g):
        return g, np.arccos(np.sqrt(3.0 / (3.0 + 4.0 * g * g)))

    def first(eta):
        g, th = gam_theta(eta * np.sqrt(eps + 1.0 / (1.0 - eta * eta)))
        return np.exp(-tau * eta * eta) * np.sin(chi * g + th) / (eta * np.sqrt(3.0 + 4.0 * g * g))

    def second(eta):
        g, th = gam_theta(np.sqrt((1.0 - eta) * (eps + 1.0 / eta)))
        return (np.exp(-tau / (eps * eta)) * np.sin(chi * g + th)
                / (eta * (1.0 + eps * eta) * np.sqrt(3.0 + 4.0 * g * g)))

    return first, second


def su_olson_u(chi, tau, eps=1.0, nq=None):
    """u = c E_r / (4 F_inc) of the diffusion-approximation Marshak wave at optical
    depth chi = sqrt(3) rho kappa x and time tau = eps c rho kappa t (Eq.
    marshak:suolson). nq points of midpoint quadrature, as the paper evaluates it for
    the boundary value; nq = None integrates adaptively (scipy.integrate.quad)."""
    first, second = _su_olson_integrands(float(chi), float(tau), float(eps))
    if nq is None:
        import warnings
        from scipy.integrate import IntegrationWarning, quad
        with warnings.catch_warnings():
            # the integrands oscillate near the ends of (0, 1) at chi > 0
            warnings.simplefilter("ignore", IntegrationWarning)
            i1 = quad(first, 0.0, 1.0, limit=2000)[0]
            i2 = quad(second, 0.0, 1.0, limit=2000)[0]
    else:
        eta = (np.arange(nq) + 0.5) / nq
        i1 = float(np.sum(first(eta))) / nq
        i2 = float(np.sum(second(eta))) / nq
    return (1.0 - 2.0 * math.sqrt(3.0) / math.pi * i1
            - math.sqrt(3.0) / math.pi * math.exp(-float(tau)) * i2)


MARSHAK_EBG = 1e-10  # background E_r standing for the cold medium (the closure needs E_r > 0)


def marshak_problem(n=128, chi_max=100.0, eps=1.0, precision="fp64"):
    """The non-equilibrium Marshak wave of Sec. 4.1.3 in units a_R = c = 1, F_inc = 1/4,
    rho = kappa_0 = 1, chat = c: a 1D slab chi in [0, chi_max] (x = chi / sqrt(3)),
    static gas (radiation only) with c_v = alpha T^3, alpha = 4 a_R / eps, a fixed
    radiation state on both faces (set each step by marshak_boundary) and a cold start.
    Then u = E_r and v = a_R T^4 = eps e. The cold medium starts at E_r = 1e-10,
    F = 0, e = 1e-10 / eps (in equilibrium), since the M1 closure needs E_r > 0."""
    L = chi_max / math.sqrt(3.0)
    spec = default_spec(nx=n, dx=L / n, c_light=1.0, a_rad=1.0, cfl=0.4,
                        theta_E=1.0, theta_F=0.51, er_floor=1e-30, rad_only=True,
                        exchange="full", cv_t3=True, cv_alpha=4.0 / eps,
                        bc=("fixed", "fixed", "periodic", "periodic", "periodic", "periodic"),
                        precision=precision)
    st = uniform_state(spec, rho=1.0, P=1.0, Er=MARSHAK_EBG, kP=1.0, kF=1.0)
    st["E"] = np.full_like(st["rho"], MARSHAK_EBG / eps)
    return dict(name=f"marshak_{n}", spec=spec, state=st, chat=1.0, eps=eps,
                dt=spec["cfl"] * spec["dx"], nsub=1)


def marshak_boundary(t, eps=1.0, nq=4000):
    """Radiation states of the two faces at time t: on the left E_r = u(0, tau) from the
    midpoint quadrature of Eq. marshak:suolson and F from the Marshak condition
    c E_r + 2 F = 4 F_inc (Eq. marshak:bc_ix1); on the right the cold medium."""
    u0 = su_olson_u(0.0, eps * t, eps, nq=nq) if t > 0.0 else 0.0
    E0 = max(u0, MARSHAK_EBG)
    left = (E0, 0.5 * (1.0 - E0), 0.0, 0.0)
    right = (MARSHAK_EBG, 0.0, 0.0, 0.0)
    zero = (0.0, 0.0, 0.0, 0.0)
    return (left, right, zero, zero, zero, zero)


# --------------------------------------------------------------------------
# shadowing by a dense cloud (Sec. 4.1.1), cgs units
# --------------------------------------------------------------------------

C_CGS = 2.99792458e10          # cm / s
A_RAD_CGS = 7.5657e-15         # erg cm^-3 K^-4
R_GAS_CGS = 1.380649e-16 / 1.6735575e-24  # k_B / m_H (mean molecular weight 1)


def shadow_problem(nx=280, ny=80, emission=False, precision="fp64", heat_capacity=1.0):
    """The shadow test of Sec. 4.1.1: a 1 cm x 0.12 cm box of gas at rho0 = 1e-3 g/cm^3
    holding an ellipsoidal cloud of rho1 = 1 (Eqs. radshadow:rho, radshadow:delta;
    centre (0.5, 0), semi-axes 0.10 and 0.06), static, in radiative equilibrium at
    T0 = 290 K; from t = 0 the left face holds a beam of temperature T1 = 6 T0 moving
    right (E_r = a_R T1^4, F = c E_r x-hat); outflow on the right and top, reflection on
    the bottom; opacity kappa = 100 (T_gas/T0)^-3.5 (rho/rho0) cm^2/g for absorption
    and flux alike; chat = c. Without emission the source step is absorption only;
    with it, the full exchange. Gas: gamma = 5/3, mean molecular weight 1 (heat
    capacity scaled by heat_capacity: r_gas = heat_capacity k_B / m_H). theta = 1
    (the paper's default): the cloud's absorption per step is ~10^2-10^5, where a
    theta near 1/2 makes the damping factor negative."""
    Lx, Ly = 1.0, 0.12
    rho0, rho1, T0 = 1e-3, 1.0, 290.0
    T1 = 6.0 * T0
    spec = default_spec(nx=nx, ny=ny, dx=Lx / nx, dy=Ly / ny, gamma=5.0 / 3.0,
                        c_light=C_CGS, a_rad=A_RAD_CGS, r_gas=R_GAS_CGS * heat_capacity, cfl=0.4,
                        theta_E=1.0, theta_F=1.0, rad_only=True,
                        exchange="full" if emission else "absorb_only",
                        bc=("fixed", "outflow", "reflect", "outflow", "periodic", "periodic"),
                        kappa_law=(100.0, T0, rho0, -3.5, 1.0), precision=precision,
                        er_floor=1e-30, rho_floor=1e-12, p_floor=1e-30)
    X, Y, _ = cell_centres(spec)
    delta = 10.0 * (((X - 0.5) / 0.10) ** 2 + (Y / 0.06) ** 2 - 1.0)
    rho = rho0 + (rho1 - rho0) / (1.0 + np.exp(np.minimum(delta, 700.0)))
    Er0 = A_RAD_CGS * T0 ** 4
    st = uniform_state(spec, rho=1.0, P=1.0, Er=Er0, kP=1.0, kF=1.0)
    st["rho"] = rho
    st["E"] = rho * spec["r_gas"] * T0 / (spec["gamma"] - 1.0)
    E1 = A_RAD_CGS * T1 ** 4
    beam = (E1, C_CGS * E1, 0.0, 0.0)
    zero = (0.0, 0.0, 0.0, 0.0)
    spec["bvals"] = (beam, zero, zero, zero, zero, zero)
    dt = spec["cfl"] * min(spec["dx"], spec["dy"]) / C_CGS
    return dict(name=f"shadow_{nx}x{ny}_{'emission' if emission else 'absorption'}",
                spec=spec, state=st, chat=C_CGS, dt=dt, nsub=1, T0=T0, T1=T1,
                crossing=Lx / C_CGS)


def radiation_temperature(Er):
    """T_rad = (E_r / a_R)^(1/4) in cgs."""
    return (np.asarray(Er) / A_RAD_CGS) ** 0.25


def pulse_problem(n=512, advected=True, beta_tau=True, precision="fp64", units="code"):
    """Advection of a radiation pulse (Sec. 4.3.2): a periodic slab x/w in
    [-21.25, 21.25] with w = 20 cm, rho0 = 25 g/cm^3, T0 = 1.1e7 K, mean particle mass
    1.67e-24 g, kappa_P = kappa_F = 0.4 cm^2/g, gamma = 5/3, chat = 100 a0 with
    a0 = sqrt(gamma k_B T0 / mu). The gas temperature is T0 (1 + exp(-x^2/(2 w^2))) and
    the density follows from pressure equilibrium with E_r = a_R T^4 (Eq. radpulse:rho,
    with P0 = a_R T0^4 / (rho0 a0^2)); F = 0. The advected run moves the gas at
    v = 3e6 cm/s and starts the pulse 2w to the left, so that after t = 2w/v both runs
    centre it at x = 0; the unadvected run is the reference. theta = 0.51 (the paper's
    default for its tests).

    units="cgs" gives the problem as stated; units="code" (the default) the same problem
    in units of w, w/a0, rho0, T0 and rho0 a0^2 (so a_R = P0, r_gas = 1/gamma,
    kappa = rho0 kappa0 w = tau0, c = c/a0), whose values fit FP32: in cgs the fluxes
    chat c E_r reach 1e34 and their products with the wave speeds overflow FP32."""
    w, rho0, T0, mu, kappa0, v0 = 20.0, 25.0, 1.1e7, 1.67e-24, 0.4, 3e6
    gamma = 5.0 / 3.0
    r_cgs = 1.380649e-16 / mu
    a0 = math.sqrt(gamma * r_cgs * T0)
    P0 = A_RAD_CGS * T0 ** 4 / (rho0 * a0 ** 2)
    if units == "cgs":
        Lu, Du, Tu, Vu = 1.0, 1.0, 1.0, 1.0  # length, density, temperature, velocity units
    elif units == "code":
        Lu, Du, Tu, Vu = w, rho0, T0, a0
    else:
        raise ValueError(f"unknown units {units!r}")
    Eu = Du * Vu ** 2  # energy density unit
    a_rad = A_RAD_CGS * Tu ** 4 / Eu
    r_gas = r_cgs * Tu / Vu ** 2
    kappa = kappa0 * Du * Lu
    L = 42.5 * w / Lu
    spec = default_spec(nx=n, dx=L / n, gamma=gamma, c_light=C_CGS / Vu, a_rad=a_rad,
                        r_gas=r_gas, cfl=0.4, theta_E=0.51, theta_F=0.51, exchange="full",
                        beta_tau=beta_tau, bc="periodic", precision=precision,
                        er_floor=1e-30 / Eu, rho_floor=1e-12 / Du, p_floor=1e-30 / Eu)
    x = -0.5 * L + (np.arange(n) + 0.5) * spec["dx"]
    v = (v0 if advected else 0.0) / Vu
    t_end = 2.0 * w / v0 * Vu / Lu
    xc = -v * t_end  # start 2w to the left when advected
    d = (x - xc + 0.5 * L) % L - 0.5 * L  # periodic distance to the pulse centre
    T = (T0 / Tu) * (1.0 + np.exp(-d ** 2 / (2.0 * (w / Lu) ** 2)))
    Tr = T * Tu / T0
    rho = (rho0 / Du) * (1.0 / Tr + gamma * P0 / 3.0 * (1.0 / Tr - Tr ** 3))
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=kappa, kF=kappa)
    st["rho"][0, 0, :] = rho
    st["mx"][0, 0, :] = rho * v
    st["E"][0, 0, :] = rho * r_gas * T / (gamma - 1.0) + 0.5 * rho * v * v
    st["Er"][0, 0, :] = a_rad * T ** 4
    kind = ("advected" if advected else "static") + ("_betatau" if beta_tau else "")
    return dict(name=f"pulse_{n}_{kind}", spec=spec, state=st, chat=100.0 * a0 / Vu,
                t_end=t_end, x=x, w=w / Lu, T0=T0 / Tu, rho0=rho0 / Du, v=v, a0=a0 / Vu,
                P0=P0, tau0=rho0 * kappa0 * w, units=units)


def gas_temperature(spec, st):
    """T = (gamma - 1)(E - rho v^2/2) / (rho r_gas)."""
    rho = np.asarray(st["rho"])
    ke = 0.5 * (np.asarray(st["mx"]) ** 2 + np.asarray(st["my"]) ** 2
                + np.asarray(st["mz"]) ** 2) / rho
    return (spec["gamma"] - 1.0) * (np.asarray(st["E"]) - ke) / (rho * spec["r_gas"])


# --------------------------------------------------------------------------
# radiation-driven expanding shell (Sec. 4.3.6, the second shell test)
# --------------------------------------------------------------------------

MSUN_G = 1.989e33
PC_CM = 3.0857e18


def shell_parameters(Psi=2000.0, M_gmc=1e6 * MSUN_G, eps=0.5, kappa0=20.0, r0=5 * PC_CM,
                     a0=2e5):
    """The shell test's dimensional parameters and what follows from them: the cluster
    luminosity L = Psi eps M_GMC, the shell mass (1 - eps) M_GMC, the Mach number
    M0 = (L kappa0 / (4 pi r0 c a0^2))^(1/2) of Eq. radshell:mach0 and the optical depth
    tau0 = M_sh kappa0 / (4 pi r0^2) of Eq. radshell:tau0."""
    L = Psi * eps * M_gmc
    M_sh = (1.0 - eps) * M_gmc
    M0 = math.sqrt(L * kappa0 / (4.0 * math.pi * r0 * C_CGS * a0 ** 2))
    tau0 = M_sh * kappa0 / (4.0 * math.pi * r0 ** 2)
    return dict(L=L, M_sh=M_sh, M0=M0, tau0=tau0, c_over_a0=C_CGS / a0, r0=r0, a0=a0)


class ShellProfile:
    """Radial profiles of the shell test in code units (r0 = 1, rho0 = M_sh/(4/3 pi r0^3)
    = 1, a0 = 1, so M_sh = 4 pi/3 and kappa = 3 tau0): the Gaussian shell of Eq.
    radshell:rhoprofile with FWHM H, the source of Eq. radshell:sourceprofile with width
    sigma_star, its flux F*(r) of Eq. radshell:fluxprofile, and the reduced flux f(r) of
    the equilibrium ODE Eq. radshell:odefluxm1, integrated by fourth-order Runge-Kutta
    outward and inward from the critical point (r_crit, 2 sqrt(3)/5) where Eq.
    radshell:rcrit holds. Inward the regular solution meets the closure's singular value
    f = 2 sqrt(3)/5 again near the source, where the streaming field of the source takes
    over; inside that radius f is held at that value."""

    def __init__(self, M0, tau0, c, H=0.1, sigma_star=0.05, h=5e-5, r_min=1e-3, r_max=4.0):
        self.M0, self.tau0, self.c = M0, tau0, c
        self.kappa = 3.0 * tau0
        self.M_sh = 4.0 * math.pi / 3.0
        self.L = M0 ** 2 * 4.0 * math.pi * c / self.kappa
        self.H, self.sig_sh, self.sig_s = H, H / (2.0 * math.sqrt(2.0 * math.log(2.0))), sigma_star
        self.f_crit = 2.0 * math.sqrt(3.0) / 5.0
        self.r_crit = self._solve_rcrit()
        self._integrate(h, r_min, r_max)

    def rho(self, r):
        r = np.asarray(r, dtype=np.float64)
        return (self.M_sh / (4.0 * math.pi * r ** 2 * math.sqrt(2.0 * math.pi) * self.sig_sh)
                * np.exp(-(r - 1.0) ** 2 / (2.0 * self.sig_sh ** 2)))

    def j(self, r):
        r = np.asarray(r, dtype=np.float64)
        s = self.sig_s
        return self.L / (2.0 * math.pi * s * s) ** 1.5 * np.exp(-r ** 2 / (2.0 * s * s))

    def _bracket_F(self, r):
        from scipy.special import erf
        s = self.sig_s
        return (erf(r / (math.sqrt(2.0) * s))
                - 2.0 * r / math.sqrt(2.0 * math.pi * s * s) * np.exp(-r ** 2 / (2.0 * s * s)))

    def F(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.L / (4.0 * math.pi * r ** 2) * self._bracket_F(r)

    def dlnF(self, r):
        # d/dr of the bracket is 4 pi r^2 j / L (the bracket is the enclosed luminosity)
        s = self.sig_s
        dB = 2.0 * r ** 2 / (math.sqrt(2.0 * math.pi) * s ** 3) * np.exp(-r ** 2 / (2.0 * s * s))
        return -2.0 / r + dB / self._bracket_F(r)

    def _bracket(self, r, f):
        q = math.sqrt(max(4.0 - 3.0 * f * f, 0.0))
        return (self.dlnF(r) / 3.0 * (5.0 - 2.0 * q) + 2.0 / r * (2.0 - q)
                + float(self.rho(r)) * self.kappa * f)

    def dfdr(self, r, f):
        q = math.sqrt(max(4.0 - 3.0 * f * f, 0.0))
        return 3.0 * f * q / (5.0 * q - 8.0) * self._bracket(r, f)

    def _solve_rcrit(self):
        from scipy.optimize import brentq
        g = lambda r: 3.0 * self.dlnF(r) + 4.0 / r + 2.0 * math.sqrt(3.0) * float(self.rho(r)) * self.kappa
        return brentq(g, 1.0 + 0.1 * self.sig_sh, 1.0 + 10.0 * self.sig_sh)

    def _crit_slope(self):
        """f' at the critical point: with the bracket B(r, f) and q(f) = sqrt(4 - 3 f^2),
        l'Hopital's rule on f' = 3 f q B / (5 q - 8) gives 5 q_f f'^2 = 3 f q (B_r + B_f f');
        the regular solution is the root on which f grows outward."""
        rc, fc, e = self.r_crit, self.f_crit, 1e-6
        q = math.sqrt(4.0 - 3.0 * fc * fc)
        qf = -3.0 * fc / q
        Br = (self._bracket(rc + e, fc) - self._bracket(rc - e, fc)) / (2.0 * e)
        Bf = (self._bracket(rc, fc + e) - self._bracket(rc, fc - e)) / (2.0 * e)
        roots = np.roots([5.0 * qf, -3.0 * fc * q * Bf, -3.0 * fc * q * Br])
        return float(max(roots.real))

    def _rk4(self, r0, f0, r1, h):
        n = max(1, int(math.ceil(abs(r1 - r0) / abs(h))))
        hh = (r1 - r0) / n
        rs, fs = [r0], [f0]
        r, f = r0, f0
        for _ in range(n):
            k1 = self.dfdr(r, f)
            k2 = self.dfdr(r + hh / 2, f + hh / 2 * k1)
            k3 = self.dfdr(r + hh / 2, f + hh / 2 * k2)
            k4 = self.dfdr(r + hh, f + hh * k3)
            fn = f + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            if not (0.0 < fn < self.f_crit if hh < 0 else 0.0 < fn < 1.0):
                break
            r, f = r + hh, fn
            rs.append(r)
            fs.append(f)
        return np.array(rs), np.array(fs)

    def _integrate(self, h, r_min, r_max):
        p, d = self._crit_slope(), 5e-4
        ro, fo = self._rk4(self.r_crit + d, self.f_crit + p * d, r_max, h)
        ri, fi = self._rk4(self.r_crit - d, self.f_crit - p * d, r_min, -h)
        self.r_inner = float(ri[-1])  # where the inward solution meets f_crit again
        self.slope = p
        self._r = np.concatenate([ri[::-1], ro])
        self._f = np.concatenate([fi[::-1], fo])
        self.r_outer = float(ro[-1])

    def f(self, r):
        r = np.asarray(r, dtype=np.float64)
        out = np.interp(r, self._r, self._f)
        out = np.where(r < self.r_inner, self.f_crit, out)
        return np.where(r > self.r_outer, self._f[-1], out)

    def E(self, r):
        return self.F(r) / (self.c * self.f(r))


_SHELL_PROFILES = {}


def shell_profile(H=0.1, sigma_star=0.05):
    """The ShellProfile of the paper's parameters (computed once per H, sigma_star)."""
    key = (float(H), float(sigma_star))
    if key not in _SHELL_PROFILES:
        par = shell_parameters()
        _SHELL_PROFILES[key] = ShellProfile(par["M0"], par["tau0"], par["c_over_a0"], H=H,
                                            sigma_star=sigma_star)
    return _SHELL_PROFILES[key]


def shell_trajectory(M0, t):
    """The shell radius and velocity of Eqs. radshell:odepos and radshell:odevel (from
    r = r0 at rest, code units) at times t: r from inverting t(r)."""
    from scipy.optimize import brentq
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    tr = lambda r: (math.sqrt(r) * math.sqrt(r - 1.0)
                    + math.log(math.sqrt(r) + math.sqrt(r - 1.0))) / (M0 * math.sqrt(2.0))
    r = np.array([1.0 if tt <= 0 else brentq(lambda x: tr(x) - tt, 1.0, 1e3) for tt in t])
    v = M0 * math.sqrt(2.0) * np.sqrt(np.maximum(1.0 - 1.0 / r, 0.0))
    return r, v


def shell_expansion_problem(n=128, chat_over_a0=860.0, precision="mixed", H=0.1, sigma_star=0.05,
                            rad_only=False):
    """The expanding-shell test of Sec. 4.3.6 in code units (r0, rho0 = M_sh/(4/3 pi r0^3),
    a0): the octant [0, 2]^3 with n^3 cells, reflecting faces at 0 and outflow faces at 2,
    isothermal gas (c_s = 1) at rest in radiative equilibrium (no exchange), the Gaussian
    shell of FWHM H at r = 1 with the density floor 1e-8, kappa = 3 tau0 for the flux,
    the central source j*(r), the flux F*(r) r_hat and E_r = F*/(c f(r)) from the
    equilibrium ODE; c = c/a0 = 1.5e5, chat = chat_over_a0 (860 in the paper, also 430
    and 215); theta_F = 0.51 (the paper's default). The shell should reach r = 2 near
    t = 0.12."""
    par = shell_parameters()
    c = par["c_over_a0"]
    prof = shell_profile(H, sigma_star)
    h = 2.0 / n
    spec = default_spec(nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, c_light=c, iso_cs=1.0,
                        isothermal=True, exchange="none", theta_F=0.51, cfl=0.4, rad_only=rad_only,
                        bc=("reflect", "outflow", "reflect", "outflow", "reflect", "outflow"),
                        rho_floor=1e-8, er_floor=1e-30, precision=precision)
    X, Y, Z = cell_centres(spec)
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    st = uniform_state(spec, rho=1.0, P=1.0, Er=1.0, kP=0.0, kF=prof.kappa)
    st["rho"][:] = np.maximum(prof.rho(r), 1e-8)
    st["E"][:] = 0.0
    Fr = prof.F(r)
    st["Er"][:] = prof.E(r)
    st["Fx"][:] = Fr * X / r
    st["Fy"][:] = Fr * Y / r
    st["Fz"][:] = Fr * Z / r
    st["j"] = prof.j(r)
    return dict(name=f"shell_{n}cubed_chat{int(chat_over_a0)}", spec=spec, state=st,
                chat=float(chat_over_a0), M0=par["M0"], tau0=par["tau0"], profile=prof,
                t_end=0.124, r=r)


def shell_moments(spec, st, r=None):
    """Density-weighted mean radius and radial velocity over the grid, Eqs.
    radshell:ravgdef and radshell:vravgdef (uniform cells)."""
    if r is None:
        X, Y, Z = cell_centres(spec)
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    else:
        X, Y, Z = cell_centres(spec)
    rho = np.asarray(st["rho"])
    m = rho.sum()
    vr = (np.asarray(st["mx"]) * X + np.asarray(st["my"]) * Y + np.asarray(st["mz"]) * Z) / r
    return float((rho * r).sum() / m), float(vr.sum() / m)


def shell_errors(M0, samples):
    """Largest relative differences of the sampled (t, <r>, <v_r>) from the trajectory of
    Eqs. radshell:odepos and radshell:odevel; the velocity from the first sample after
    t = 0 (it starts at rest, where a relative error has no meaning)."""
    t = np.array([s[0] for s in samples])
    r = np.array([s[1] for s in samples])
    v = np.array([s[2] for s in samples])
    rex, vex = shell_trajectory(M0, t)
    moving = t > 0
    return (float(np.max(np.abs(r / rex - 1.0))),
            float(np.max(np.abs(v[moving] / vex[moving] - 1.0))))
