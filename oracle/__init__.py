"""Python access to the plain FP64 CPU oracle (``rhd_oracle.c``).

TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline leg of
the benchmark are the only code allowed to import this package. The GPU library
and its binding never import it, and it never imports them.

The oracle follows Skinner & Ostriker (2013), Sec. 3: the implicit gas-radiation
energy exchange (Sec. 3.4), the gas Van Leer step (Sec. 3.4, last part), the
radiation Van Leer subcycles with the M1 closure (Sec. 2.3), HLL fluxes bounded by
the M1 eigenvalues (Sec. 3.3) and the source terms of Sec. 3.4, and the
second-order gas source correction. See the header of rhd_oracle.c for the
readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rhd_oracle.c")
LIB = os.path.join(HERE, "librhd_oracle.so")

BC = {"periodic": 0, "outflow": 1, "reflect": 2, "fixed": 3}
ISOTHERMAL = 1 << 0
EXCH = {"full": 0 << 1, "absorb_only": 1 << 1, "none": 2 << 1}
BETA_TAU = 1 << 3
RAD_ONLY = 1 << 4
PRECISION_MIXED = 1 << 5
GAS_CV_T3 = 1 << 6
OPACITY_LAW = 1 << 7
CLOSURE_P1 = 1 << 8

STATE_FIELDS = ("rho", "mx", "my", "mz", "E", "Er", "Fx", "Fy", "Fz")


def build(force=True):
    """Compile the oracle with gcc (plain C99, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                           "-Wall", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("c_light", ctypes.c_double), ("a_rad", ctypes.c_double), ("r_gas", ctypes.c_double),
        ("iso_cs", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("theta_E", ctypes.c_double), ("theta_F", ctypes.c_double),
        ("newton_rtol", ctypes.c_double),
        ("newton_maxit", ctypes.c_int),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
        ("er_floor", ctypes.c_double),
        ("bc", ctypes.c_int * 6),
        ("flags", ctypes.c_uint),
        ("cv_alpha", ctypes.c_double),
        ("bval", (ctypes.c_double * 4) * 6),
        ("kappa_law", ctypes.c_double * 5),
    ]


class Fields(ctypes.Structure):
    _fields_ = [(name, ctypes.POINTER(ctypes.c_double)) for name in
                ("rho", "mx", "my", "mz", "E", "Er", "Fx", "Fy", "Fz", "kP", "kF", "j")]


class Counts(ctypes.Structure):
    _fields_ = [(name, ctypes.c_long) for name in
                ("exch_theta1", "exch_bisect", "newton_iters", "newton_max", "rad_fclamp",
                 "rad_efloor", "gas_rhofloor", "gas_pfloor")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_m1_eddington_factor.argtypes = [ctypes.c_double, dp]
        L.orc_m1_pressure.argtypes = [ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_m1_eigen.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, dp, dp]
        L.orc_rad_hll_flux.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       dp]
        L.orc_p1_hll_flux.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      dp]
        L.orc_gas_flux.argtypes = [dp, ctypes.c_int, ctypes.POINTER(Params), dp]
        L.orc_gas_riemann.argtypes = [dp, dp, ctypes.c_int, ctypes.POINTER(Params), dp]
        L.orc_exchange_cell.argtypes = [ctypes.c_double] * 6 + [
            ctypes.POINTER(Params), dp, ctypes.POINTER(ctypes.c_int),
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.orc_exchange_cell.restype = ctypes.c_double
        L.orc_mc_slope.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_mc_slope.restype = ctypes.c_double
        L.orc_step.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Fields), ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.POINTER(Counts)]
        L.orc_step.restype = ctypes.c_int
        L.orc_suggest_dt.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Fields),
                                     ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int), dp]
        L.orc_suggest_dt.restype = ctypes.c_int
        L.orc_ledger.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Fields),
                                 ctypes.c_double, dp]
        _lib = L
    return _lib


def make_params(spec):
    p = Params()
    for name in ("nx", "ny", "nz"):
        setattr(p, name, int(spec[name]))
    for name in ("dx", "dy", "dz", "gamma", "c_light", "a_rad", "r_gas", "iso_cs", "cfl",
                 "theta_E", "theta_F", "newton_rtol", "rho_floor", "p_floor", "er_floor"):
        setattr(p, name, float(spec[name]))
    p.newton_maxit = int(spec["newton_maxit"])
    for q in range(6):
        p.bc[q] = BC[spec["bc"][q]]
    flags = EXCH[spec["exchange"]]
    if spec["isothermal"]:
        flags |= ISOTHERMAL
    if spec["beta_tau"]:
        flags |= BETA_TAU
    if spec["rad_only"]:
        flags |= RAD_ONLY
    if spec["precision"] == "mixed":
        flags |= PRECISION_MIXED
    if spec["cv_t3"]:
        flags |= GAS_CV_T3
    if spec["kappa_law"] is not None:
        flags |= OPACITY_LAW
        for q in range(5):
            p.kappa_law[q] = float(spec["kappa_law"][q])
    if spec["closure"] == "p1":
        flags |= CLOSURE_P1
    elif spec["closure"] != "m1":
        raise ValueError(f"unknown closure {spec['closure']!r}")
    p.flags = flags
    p.cv_alpha = float(spec["cv_alpha"])
    for f in range(6):
        for q in range(4):
            p.bval[f][q] = float(spec["bvals"][f][q])
    return p


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fields(spec, state):
    """Flat contiguous float64 copies of the state plus a Fields struct over them."""
    n = int(spec["nx"]) * int(spec["ny"]) * int(spec["nz"])
    arrs = {}
    for k in STATE_FIELDS + ("kP", "kF"):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(state[k], dtype=np.float64),
                                                 (spec["nz"], spec["ny"], spec["nx"])))
        arrs[k] = np.array(a.reshape(n), dtype=np.float64, copy=True)
    if state.get("j") is not None:
        arrs["j"] = np.array(np.asarray(state["j"], dtype=np.float64).reshape(n), copy=True)
    f = Fields()
    for k in STATE_FIELDS + ("kP", "kF"):
        setattr(f, k, _dptr(arrs[k]))
    f.j = _dptr(arrs["j"]) if "j" in arrs else ctypes.POINTER(ctypes.c_double)()
    return f, arrs


def _unflatten(spec, arrs, state):
    shape = (spec["nz"], spec["ny"], spec["nx"])
    out = dict(state)
    for k in STATE_FIELDS:
        out[k] = arrs[k].reshape(shape).copy()
    return out


def step(spec, state, dt_gas, chat, nsub, steps=1):
    """Advance ``steps`` gas steps; returns (new_state, counters)."""
    p = make_params(spec)
    f, arrs = _fields(spec, state)
    cnt = Counts()
    for _ in range(steps):
        rc = lib().orc_step(ctypes.byref(p), ctypes.byref(f), float(dt_gas), float(chat),
                            int(nsub), ctypes.byref(cnt))
        if rc != 0:
            raise ValueError(f"orc_step returned {rc}")
    return _unflatten(spec, arrs, state), cnt.as_dict()


def suggest_dt(spec, state, chat):
    """(dt_gas, nsub, v_max) from the radiation-modified CFL condition."""
    p = make_params(spec)
    f, _ = _fields(spec, state)
    dt = ctypes.c_double()
    ns = ctypes.c_int()
    vm = ctypes.c_double()
    rc = lib().orc_suggest_dt(ctypes.byref(p), ctypes.byref(f), float(chat), ctypes.byref(dt),
                              ctypes.byref(ns), ctypes.byref(vm))
    if rc != 0:
        raise ValueError("orc_suggest_dt failed")
    return dt.value, ns.value, vm.value


def ledger(spec, state, chat):
    """[sum(E + (c/chat) E_r), sum(m + F/(c chat)) x3, sum(rho)] times dV."""
    p = make_params(spec)
    f, _ = _fields(spec, state)
    out = (ctypes.c_double * 5)()
    lib().orc_ledger(ctypes.byref(p), ctypes.byref(f), float(chat), out)
    return np.array(list(out))


def run(problem, steps=None, dt=None, nsub=None, chat=None, state=None):
    """Run a problem dict from ``rhd_inputs`` for a number of gas steps. When the
    recipe leaves dt or nsub open, each step takes the CFL step of its state."""
    spec = problem["spec"]
    st = problem["state"] if state is None else state
    chat = problem["chat"] if chat is None else chat
    steps = problem.get("steps", 1) if steps is None else steps
    total = {}
    for _ in range(steps):
        d, n = dt if dt is not None else problem.get("dt"), nsub if nsub is not None else problem.get("nsub")
        if d is None or n is None:
            d2, n2, _ = suggest_dt(spec, st, chat)
            d = d2 if d is None else d
            n = n2 if n is None else n
        st, cnt = step(spec, st, d, chat, n)
        for k, v in cnt.items():
            total[k] = max(total.get(k, 0), v) if k == "newton_max" else total.get(k, 0) + v
    return st, total


# ---- single-state pieces --------------------------------------------------

def eddington_factor(f):
    out = ctypes.c_double()
    lib().orc_m1_eddington_factor(float(f), ctypes.byref(out))
    return out.value


def m1_pressure(E, F, c):
    Fa = (ctypes.c_double * 3)(*[float(x) for x in F])
    P = (ctypes.c_double * 9)()
    lib().orc_m1_pressure(float(E), Fa, float(c), P)
    return np.array(list(P)).reshape(3, 3)


def m1_eigen(E, F, c, chat, d):
    Fa = (ctypes.c_double * 3)(*[float(x) for x in F])
    l1 = ctypes.c_double()
    l3 = ctypes.c_double()
    lib().orc_m1_eigen(float(E), Fa, float(c), float(chat), int(d), ctypes.byref(l1),
                       ctypes.byref(l3))
    return l1.value, l3.value


def rad_hll_flux(UL, UR, d, c, chat):
    a = (ctypes.c_double * 4)(*[float(x) for x in UL])
    b = (ctypes.c_double * 4)(*[float(x) for x in UR])
    out = (ctypes.c_double * 4)()
    lib().orc_rad_hll_flux(a, b, int(d), float(c), float(chat), out)
    return np.array(list(out))


def p1_hll_flux(UL, UR, d, c, chat):
    a = (ctypes.c_double * 4)(*[float(x) for x in UL])
    b = (ctypes.c_double * 4)(*[float(x) for x in UR])
    out = (ctypes.c_double * 4)()
    lib().orc_p1_hll_flux(a, b, int(d), float(c), float(chat), out)
    return np.array(list(out))


def gas_flux(spec, W, d):
    p = make_params(spec)
    a = (ctypes.c_double * 5)(*[float(x) for x in W])
    out = (ctypes.c_double * 5)()
    lib().orc_gas_flux(a, int(d), ctypes.byref(p), out)
    return np.array(list(out))


def gas_riemann(spec, WL, WR, d):
    p = make_params(spec)
    a = (ctypes.c_double * 5)(*[float(x) for x in WL])
    b = (ctypes.c_double * 5)(*[float(x) for x in WR])
    out = (ctypes.c_double * 5)()
    lib().orc_gas_riemann(a, b, int(d), ctypes.byref(p), out)
    return np.array(list(out))


def exchange_cell(spec, rho, e, Er, kP, dt, chat):
    """(e_new, Er_new, iterations, used_theta1, used_bisection) for one cell."""
    p = make_params(spec)
    er = ctypes.c_double()
    it = ctypes.c_int()
    t1 = ctypes.c_int()
    bi = ctypes.c_int()
    x = lib().orc_exchange_cell(float(rho), float(e), float(Er), float(kP), float(dt),
                                float(chat), ctypes.byref(p), ctypes.byref(er),
                                ctypes.byref(it), ctypes.byref(t1), ctypes.byref(bi))
    return x, er.value, it.value, bool(t1.value), bool(bi.value)


def mc_slope(dm, dp):
    return lib().orc_mc_slope(float(dm), float(dp))
