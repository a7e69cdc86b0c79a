"""Python binding of the gfx950 library for the gray two-moment (M1)
radiation-hydrodynamics step of Skinner & Ostriker (2013).

Argument marshalling only: every step of the method runs in the HIP kernels of
``librhd.so`` behind the C interface declared in ``include/rhd.h``. The functions
here carry the same names as that interface. If the library has not been built,
every call raises ``RhdError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhd.so")

RHD_OK = 0
RHD_EINVAL = -1
RHD_ECFL = -2
RHD_ENONFINITE = -3
RHD_ENOMEM = -4
RHD_EDEVICE = -5
RHD_ESTATE = -6
RHD_ETIMEOUT = -7
ERROR_NAMES = {RHD_EINVAL: "RHD_EINVAL", RHD_ECFL: "RHD_ECFL", RHD_ENONFINITE: "RHD_ENONFINITE",
               RHD_ENOMEM: "RHD_ENOMEM", RHD_EDEVICE: "RHD_EDEVICE", RHD_ESTATE: "RHD_ESTATE",
               RHD_ETIMEOUT: "RHD_ETIMEOUT"}
RHD_REQ_QUEUED, RHD_REQ_RUNNING, RHD_REQ_DONE, RHD_REQ_FAILED, RHD_REQ_CANCELLED = range(5)
REQ_STATUS_NAMES = ("queued", "running", "done", "failed", "cancelled")

RHD_BC_PERIODIC, RHD_BC_OUTFLOW, RHD_BC_REFLECT, RHD_BC_FIXED = 0, 1, 2, 3
RHD_ISOTHERMAL = 1 << 0
RHD_EXCHANGE_MASK = 3 << 1
RHD_EXCHANGE_FULL = 0 << 1
RHD_EXCHANGE_ABSORB_ONLY = 1 << 1
RHD_EXCHANGE_NONE = 2 << 1
RHD_BETA_TAU = 1 << 3
RHD_RAD_ONLY = 1 << 4
RHD_PRECISION_MIXED = 1 << 5
RHD_GAS_CV_T3 = 1 << 6
RHD_OPACITY_LAW = 1 << 7
RHD_CLOSURE_P1 = 1 << 8
RHD_KERNELS_PER_CELL = 0
RHD_KERNELS_TILED = 1
RHD_KERNELS_FACE_SPLIT = 2

EXPORTED = ("rhd_default_params", "rhd_create", "rhd_set_state", "rhd_set_state_device",
            "rhd_set_emission", "rhd_set_boundary", "rhd_step", "rhd_run", "rhd_suggest_dt", "rhd_ledger", "rhd_get_state",
            "rhd_get_state_device", "rhd_get_diagnostics", "rhd_reset_diagnostics", "rhd_sync",
            "rhd_device_bytes", "rhd_footprint_bytes", "rhd_destroy", "rhd_last_error",
            "rhd_set_timing", "rhd_get_timing", "rhd_set_kernel_variant", "rhd_autotune",
            "rhd_batch_create", "rhd_batch_add", "rhd_batch_remove", "rhd_batch_step",
            "rhd_batch_size", "rhd_batch_sync", "rhd_batch_destroy", "rhd_batch_last_error",
            "rhd_server_create", "rhd_server_submit", "rhd_server_poll", "rhd_server_wait",
            "rhd_server_fetch", "rhd_server_cancel", "rhd_server_get_stats", "rhd_server_destroy",
            "rhd_server_last_error", "rhd_subcycles_noalloc", "rhd_subcycles_noalloc_bytes",
            "rhd_batch_set_persistent", "rhd_server_set_persistent", "rhd_set_graph",
            "rhd_get_graph_stats")
RHD_NOALLOC_SCRATCH_BYTES = 64 << 20


class RhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class rhd_params(ctypes.Structure):
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
        ("kappa_law", ctypes.c_double * 5),
    ]


class rhd_diag(ctypes.Structure):
    _fields_ = [("ledger", ctypes.c_double * 5), ("vmax", ctypes.c_double)] + [
        (name, ctypes.c_longlong) for name in
        ("exch_theta1", "exch_bisect", "newton_iters", "newton_max", "rad_fclamp", "rad_efloor",
         "gas_rhofloor", "gas_pfloor", "nonfinite", "first_nonfinite_cell", "steps", "subcycles")]

    def as_dict(self):
        out = {"ledger": list(self.ledger), "vmax": self.vmax}
        for name, _ in self._fields_[2:]:
            out[name] = int(getattr(self, name))
        return out


class rhd_timing(ctypes.Structure):
    _fields_ = [("nkernels", ctypes.c_int), ("name", (ctypes.c_char * 24) * 12),
                ("calls", ctypes.c_longlong * 12), ("total_ms", ctypes.c_double * 12),
                ("cells", ctypes.c_longlong * 12)]

    def as_dict(self):
        return {self.name[k].value.decode(): {"calls": int(self.calls[k]),
                                              "total_ms": float(self.total_ms[k]),
                                              "cells": int(self.cells[k])}
                for k in range(self.nkernels)}


class rhd_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("error", ctypes.c_int), ("steps_done", ctypes.c_int),
                ("zone_updates", ctypes.c_longlong), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {"status": REQ_STATUS_NAMES[self.status], "error": int(self.error),
                "steps_done": int(self.steps_done), "zone_updates": int(self.zone_updates),
                "t_submit": self.t_submit, "t_start": self.t_start, "t_done": self.t_done}


class rhd_server_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_longlong) for name in
                ("submitted", "completed", "failed", "cancelled", "rejected", "zone_updates",
                 "rounds", "bytes_in_use", "peak_bytes")] + [
        (name, ctypes.c_int) for name in ("running", "queued", "peak_running")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib = None


def _share_torch_runtime():
    """Import torch (if installed) before the library is loaded. torch ships its own HIP
    runtime with the same soname as the system one; loaded first, it is the one the
    dynamic linker then hands to librhd.so too, so that torch streams and device
    pointers are valid in this library. Loaded the other way round, the process would
    hold two HIP runtimes and torch would see no GPU."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """The loaded library; raises RhdError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    _share_torch_runtime()
    if not os.path.exists(LIB_PATH):
        raise RhdError(RHD_EDEVICE, f"{LIB_PATH} is missing: build it with "
                                    "`python paper_1306_0010_amd/build.py` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    P = ctypes.POINTER(rhd_params)
    L.rhd_default_params.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.rhd_default_params.restype = None
    L.rhd_create.argtypes = [P, vp, ctypes.POINTER(vp)]
    L.rhd_set_state.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
    L.rhd_set_state_device.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
    L.rhd_set_emission.argtypes = [vp, dp]
    L.rhd_set_boundary.argtypes = [vp, ctypes.c_int, dp]
    L.rhd_run.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int), ctypes.c_double, dp]
    L.rhd_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    L.rhd_suggest_dt.argtypes = [vp, ctypes.c_double, dp, ctypes.POINTER(ctypes.c_int)]
    L.rhd_ledger.argtypes = [vp, ctypes.c_double]
    L.rhd_get_state.argtypes = [vp, dp, dp, dp, dp, dp]
    L.rhd_get_state_device.argtypes = [vp, vp, vp, vp, vp, vp]
    L.rhd_get_diagnostics.argtypes = [vp, ctypes.POINTER(rhd_diag)]
    L.rhd_reset_diagnostics.argtypes = [vp]
    L.rhd_sync.argtypes = [vp]
    L.rhd_device_bytes.argtypes = [vp]
    L.rhd_device_bytes.restype = ctypes.c_longlong
    L.rhd_footprint_bytes.argtypes = [P]
    L.rhd_footprint_bytes.restype = ctypes.c_longlong
    L.rhd_destroy.argtypes = [vp]
    L.rhd_destroy.restype = None
    L.rhd_set_timing.argtypes = [vp, ctypes.c_int]
    L.rhd_set_kernel_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    ip = ctypes.POINTER(ctypes.c_int)
    L.rhd_autotune.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ip, ip, ip]
    L.rhd_get_timing.argtypes = [vp, ctypes.POINTER(rhd_timing)]
    L.rhd_last_error.argtypes = [vp]
    L.rhd_last_error.restype = ctypes.c_char_p
    L.rhd_batch_create.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.rhd_batch_add.argtypes = [vp, vp, ctypes.c_double]
    L.rhd_batch_remove.argtypes = [vp, vp]
    L.rhd_batch_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    L.rhd_batch_size.argtypes = [vp]
    L.rhd_set_graph.argtypes = [vp, ctypes.c_int]
    L.rhd_set_graph.restype = ctypes.c_int
    L.rhd_get_graph_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong)]
    L.rhd_get_graph_stats.restype = ctypes.c_int
    L.rhd_batch_set_persistent.argtypes = [vp, ctypes.c_int]
    L.rhd_batch_set_persistent.restype = ctypes.c_int
    L.rhd_server_set_persistent.argtypes = [vp, ctypes.c_int]
    L.rhd_server_set_persistent.restype = ctypes.c_int
    L.rhd_batch_sync.argtypes = [vp]
    L.rhd_batch_destroy.argtypes = [vp]
    L.rhd_batch_destroy.restype = None
    L.rhd_batch_last_error.argtypes = [vp]
    L.rhd_batch_last_error.restype = ctypes.c_char_p
    L.rhd_server_create.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(vp)]
    L.rhd_server_submit.argtypes = [vp, P, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int, dp,
                                    ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_longlong)]
    L.rhd_server_poll.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(rhd_request_info)]
    L.rhd_server_wait.argtypes = [vp, ctypes.c_longlong, ctypes.c_double,
                                  ctypes.POINTER(rhd_request_info)]
    L.rhd_server_fetch.argtypes = [vp, ctypes.c_longlong, dp, dp, dp, dp, dp,
                                   ctypes.POINTER(rhd_diag)]
    L.rhd_server_cancel.argtypes = [vp, ctypes.c_longlong]
    L.rhd_server_get_stats.argtypes = [vp, ctypes.POINTER(rhd_server_stats)]
    L.rhd_server_destroy.argtypes = [vp]
    L.rhd_server_destroy.restype = None
    L.rhd_server_last_error.argtypes = [vp]
    L.rhd_server_last_error.restype = ctypes.c_char_p
    L.rhd_subcycles_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                        ctypes.c_double, vp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int]
    L.rhd_subcycles_noalloc.restype = ctypes.c_int
    L.rhd_subcycles_noalloc_bytes.argtypes = [P]
    L.rhd_subcycles_noalloc_bytes.restype = ctypes.c_longlong
    for name in ("rhd_server_create", "rhd_server_submit", "rhd_server_poll", "rhd_server_wait",
                 "rhd_server_fetch", "rhd_server_cancel", "rhd_server_get_stats"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("rhd_create", "rhd_set_state", "rhd_set_state_device", "rhd_set_emission",
                 "rhd_set_boundary", "rhd_run",
                 "rhd_step", "rhd_suggest_dt", "rhd_ledger", "rhd_get_state",
                 "rhd_get_state_device", "rhd_get_diagnostics", "rhd_reset_diagnostics",
                 "rhd_sync", "rhd_set_timing", "rhd_get_timing", "rhd_set_kernel_variant",
                 "rhd_autotune", "rhd_batch_create", "rhd_batch_add", "rhd_batch_remove",
                 "rhd_batch_step", "rhd_batch_size", "rhd_batch_sync"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, handle=None):
    if rc != RHD_OK:
        msg = lib().rhd_last_error(handle).decode(errors="replace")
        raise RhdError(rc, msg)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# cells of every live handle, recorded at rhd_create: the C functions read and write
# that many values (three per cell for momentum and flux) through the pointers passed
_CELLS = {}


def _check_len(name, a, n):
    if a is not None and a.size != n:
        raise ValueError(f"{name} holds {a.size} values, the grid needs {n}")


def _cells(h):
    if h not in _CELLS:
        raise ValueError("unknown or destroyed handle")
    return _CELLS[h]


# ---------------------------------------------------------------------------
# the C functions, same names
# ---------------------------------------------------------------------------

def rhd_default_params(nx, ny, nz):
    p = rhd_params()
    lib().rhd_default_params(ctypes.byref(p), int(nx), int(ny), int(nz))
    return p


def rhd_create(params, stream=None):
    """Returns an opaque handle (int). ``stream`` is a hipStream_t as an int (for
    example ``torch.cuda.current_stream().cuda_stream``) or None for an owned stream."""
    h = ctypes.c_void_p()
    _check(lib().rhd_create(ctypes.byref(params), ctypes.c_void_p(stream) if stream else None,
                            ctypes.byref(h)))
    _CELLS[h.value] = int(params.nx) * int(params.ny) * int(params.nz)
    return h.value


def rhd_set_state(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (rho, mom, E, Er, Fr, kappaP, kappaF)]
    n = _cells(h)
    nk = 1 if kappa_scalar else n
    for name, a, m in zip(("rho", "mom", "E", "Er", "Fr", "kappaP", "kappaF"), arrs,
                          (n, 3 * n, n, n, 3 * n, nk, nk)):
        _check_len(name, a, m)
    ptrs = [_dptr(a) if a is not None else None for a in arrs]
    _check(lib().rhd_set_state(h, *ptrs, int(kappa_scalar)), h)


def rhd_set_state_device(h, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar):
    """Device pointers (ints), e.g. ``tensor.data_ptr()`` of float64 CUDA tensors."""
    _check(lib().rhd_set_state_device(h, rho, mom, E, Er, Fr, kappaP, kappaF, int(kappa_scalar)), h)


def rhd_set_emission(h, j):
    if j is None:
        _check(lib().rhd_set_emission(h, None), h)
        return
    a = np.ascontiguousarray(j, dtype=np.float64)
    _check_len("j", a, _cells(h))
    _check(lib().rhd_set_emission(h, _dptr(a)), h)


def rhd_set_boundary(h, face, U):
    a = np.ascontiguousarray(U, dtype=np.float64)
    if a.shape != (4,):
        raise ValueError("U must hold (E_r, F_x, F_y, F_z)")
    _check(lib().rhd_set_boundary(h, int(face), _dptr(a)), h)


def rhd_step(h, dt_gas, chat, nsub):
    _check(lib().rhd_step(h, float(dt_gas), float(chat), int(nsub)), h)


def rhd_run(h, dt_gas, nsub, chat, bvals=None):
    """Many gas steps in one call: dt_gas and nsub per step; bvals None or an array of
    shape (steps, 6, 4) of fixed-face states per step."""
    dts = np.ascontiguousarray(dt_gas, dtype=np.float64).reshape(-1)
    ns = np.ascontiguousarray(nsub, dtype=np.int32).reshape(-1)
    if ns.shape != dts.shape:
        raise ValueError("dt_gas and nsub need one entry per step")
    bv = None
    if bvals is not None:
        bv = np.ascontiguousarray(bvals, dtype=np.float64)
        if bv.shape != (dts.size, 6, 4):
            raise ValueError("bvals must have shape (steps, 6, 4)")
    _check(lib().rhd_run(h, int(dts.size), _dptr(dts),
                         ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(chat),
                         _dptr(bv) if bv is not None else None), h)


def rhd_suggest_dt(h, chat):
    dt = ctypes.c_double()
    ns = ctypes.c_int()
    _check(lib().rhd_suggest_dt(h, float(chat), ctypes.byref(dt), ctypes.byref(ns)), h)
    return dt.value, ns.value


def rhd_ledger(h, chat):
    _check(lib().rhd_ledger(h, float(chat)), h)


def rhd_get_state(h, N):
    if N != _cells(h):
        raise ValueError(f"the handle's grid has {_cells(h)} cells, not {N}")
    out = {"rho": np.empty(N), "mom": np.empty(3 * N), "E": np.empty(N), "Er": np.empty(N),
           "Fr": np.empty(3 * N)}
    _check(lib().rhd_get_state(h, _dptr(out["rho"]), _dptr(out["mom"]), _dptr(out["E"]),
                               _dptr(out["Er"]), _dptr(out["Fr"])), h)
    return out


def rhd_get_state_device(h, rho, mom, E, Er, Fr):
    _check(lib().rhd_get_state_device(h, rho, mom, E, Er, Fr), h)


def rhd_get_diagnostics(h):
    d = rhd_diag()
    _check(lib().rhd_get_diagnostics(h, ctypes.byref(d)), h)
    return d.as_dict()


def rhd_reset_diagnostics(h):
    _check(lib().rhd_reset_diagnostics(h), h)


def rhd_sync(h):
    _check(lib().rhd_sync(h), h)


def rhd_set_timing(h, enable):
    _check(lib().rhd_set_timing(h, int(bool(enable))), h)


def rhd_get_timing(h):
    t = rhd_timing()
    _check(lib().rhd_get_timing(h, ctypes.byref(t)), h)
    return t.as_dict()


def rhd_set_kernel_variant(h, variant, tile_rows=8, zchunk=8):
    _check(lib().rhd_set_kernel_variant(h, int(variant), int(tile_rows), int(zchunk)), h)


def rhd_set_graph(h, enable):
    _check(lib().rhd_set_graph(h, int(bool(enable))), h)


def rhd_get_graph_stats(h):
    c, r = ctypes.c_longlong(), ctypes.c_longlong()
    _check(lib().rhd_get_graph_stats(h, ctypes.byref(c), ctypes.byref(r)), h)
    return c.value, r.value


def rhd_autotune(h, chat, dt_rad, reps=3):
    """Returns (variant, tile_rows, zchunk) chosen for the handle."""
    v, r, z = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().rhd_autotune(h, float(chat), float(dt_rad), int(reps), ctypes.byref(v),
                              ctypes.byref(r), ctypes.byref(z)), h)
    return v.value, r.value, z.value


def _bcheck(rc, b=None):
    if rc != RHD_OK:
        raise RhdError(rc, lib().rhd_batch_last_error(b).decode(errors="replace"))


def rhd_batch_create(max_solves, tile_rows=8, zchunk=8, stream=None):
    b = ctypes.c_void_p()
    _bcheck(lib().rhd_batch_create(ctypes.c_void_p(stream) if stream else None, int(max_solves),
                                   int(tile_rows), int(zchunk), ctypes.byref(b)))
    return b.value


def rhd_batch_add(b, h, chat):
    _bcheck(lib().rhd_batch_add(b, h, float(chat)), b)


def rhd_batch_remove(b, h):
    _bcheck(lib().rhd_batch_remove(b, h), b)


def rhd_batch_step(b):
    """One gas step of every member; returns (nsub list, dt list) in member order."""
    n = lib().rhd_batch_size(b)
    ns = (ctypes.c_int * max(n, 1))()
    dt = (ctypes.c_double * max(n, 1))()
    _bcheck(lib().rhd_batch_step(b, ns, dt), b)
    return list(ns)[:n], list(dt)[:n]


def rhd_batch_set_persistent(b, on):
    _bcheck(lib().rhd_batch_set_persistent(b, int(bool(on))), b)


def rhd_batch_size(b):
    return int(lib().rhd_batch_size(b))


def rhd_batch_sync(b):
    _bcheck(lib().rhd_batch_sync(b), b)


def rhd_batch_destroy(b):
    if b:
        lib().rhd_batch_destroy(b)


def rhd_batch_last_error(b=None):
    return lib().rhd_batch_last_error(b).decode(errors="replace")


def _scheck(rc, s=None):
    if rc != RHD_OK:
        raise RhdError(rc, lib().rhd_server_last_error(s).decode(errors="replace"))


def rhd_server_create(budget_bytes, max_slots, tile_rows=8, zchunk=8):
    s = ctypes.c_void_p()
    _scheck(lib().rhd_server_create(int(budget_bytes), int(max_slots), int(tile_rows), int(zchunk),
                                    ctypes.byref(s)))
    return s.value


def rhd_server_submit(s, params, rho, mom, E, Er, Fr, kappaP, kappaF, kappa_scalar, j, steps, chat):
    """Queue a request; returns its id. The arrays are copied before the call returns."""
    arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (rho, mom, E, Er, Fr, kappaP, kappaF, j)]
    n = int(params.nx) * int(params.ny) * int(params.nz)
    nk = 1 if kappa_scalar else n
    for name, a, m in zip(("rho", "mom", "E", "Er", "Fr", "kappaP", "kappaF", "j"), arrs,
                          (n, 3 * n, n, n, 3 * n, nk, nk, n)):
        _check_len(name, a, m)
    ptrs = [_dptr(a) if a is not None else None for a in arrs]
    rid = ctypes.c_longlong()
    _scheck(lib().rhd_server_submit(s, ctypes.byref(params), *ptrs[:7], int(kappa_scalar), ptrs[7],
                                    int(steps), float(chat), ctypes.byref(rid)), s)
    return rid.value


def rhd_server_set_persistent(s, on):
    _scheck(lib().rhd_server_set_persistent(s, int(bool(on))), s)


def rhd_server_poll(s, rid):
    info = rhd_request_info()
    _scheck(lib().rhd_server_poll(s, int(rid), ctypes.byref(info)), s)
    return info.as_dict()


def rhd_server_wait(s, rid, timeout_s=-1.0):
    """Blocks (without holding the GIL) until the request has finished; RhdError with
    code RHD_ETIMEOUT when timeout_s runs out first."""
    info = rhd_request_info()
    _scheck(lib().rhd_server_wait(s, int(rid), float(timeout_s), ctypes.byref(info)), s)
    return info.as_dict()


def rhd_server_fetch(s, rid, N):
    """(state dict, diagnostics dict, code) of a finished request, which is then forgotten.
    code is RHD_OK for a done request and the request's error for a failed one; RhdError
    for a request without a result."""
    out = {"rho": np.empty(N), "mom": np.empty(3 * N), "E": np.empty(N), "Er": np.empty(N),
           "Fr": np.empty(3 * N)}
    d = rhd_diag()
    rc = lib().rhd_server_fetch(s, int(rid), _dptr(out["rho"]), _dptr(out["mom"]), _dptr(out["E"]),
                                _dptr(out["Er"]), _dptr(out["Fr"]), ctypes.byref(d))
    if rc in (RHD_EINVAL, RHD_ESTATE):
        _scheck(rc, s)
    return out, d.as_dict(), rc


def rhd_server_cancel(s, rid):
    _scheck(lib().rhd_server_cancel(s, int(rid)), s)


def rhd_server_get_stats(s):
    st = rhd_server_stats()
    _scheck(lib().rhd_server_get_stats(s, ctypes.byref(st)), s)
    return st.as_dict()


def rhd_server_destroy(s):
    if s:
        lib().rhd_server_destroy(s)


def rhd_server_last_error(s=None):
    return lib().rhd_server_last_error(s).decode(errors="replace")


def rhd_subcycles_noalloc(params, stream, Er, Fr, rho, mom, kappaP, kappaF, kappaP_s, kappaF_s,
                          j, dt_gas, chat, nsub):
    """Radiation subcycles on caller-owned device arrays, allocating nothing. Every array
    argument is a device address (an int, e.g. a torch tensor's data_ptr()) or None."""
    _check(lib().rhd_subcycles_noalloc(ctypes.byref(params), stream, Er, Fr, rho, mom, kappaP,
                                       kappaF, float(kappaP_s), float(kappaF_s), j,
                                       float(dt_gas), float(chat), int(nsub)))


def rhd_subcycles_noalloc_bytes(params):
    return int(lib().rhd_subcycles_noalloc_bytes(ctypes.byref(params)))


def rhd_device_bytes(h):
    return int(lib().rhd_device_bytes(h))


def rhd_footprint_bytes(params):
    return int(lib().rhd_footprint_bytes(ctypes.byref(params)))


def rhd_destroy(h):
    if h:
        lib().rhd_destroy(h)
        _CELLS.pop(h, None)


def rhd_last_error(h=None):
    return lib().rhd_last_error(h).decode(errors="replace")


# ---------------------------------------------------------------------------
# problem description -> parameters, and a handle wrapper
# ---------------------------------------------------------------------------

_BC = {"periodic": RHD_BC_PERIODIC, "outflow": RHD_BC_OUTFLOW, "reflect": RHD_BC_REFLECT,
       "fixed": RHD_BC_FIXED}
_EXCH = {"full": RHD_EXCHANGE_FULL, "absorb_only": RHD_EXCHANGE_ABSORB_ONLY,
         "none": RHD_EXCHANGE_NONE}


def params_from_spec(spec):
    """rhd_params from a problem description dict (grid, constants, switches)."""
    p = rhd_default_params(spec["nx"], spec["ny"], spec["nz"])
    for name in ("dx", "dy", "dz", "gamma", "c_light", "a_rad", "r_gas", "iso_cs", "cfl",
                 "theta_E", "theta_F", "newton_rtol", "rho_floor", "p_floor", "er_floor"):
        setattr(p, name, float(spec[name]))
    p.newton_maxit = int(spec.get("newton_maxit", 50))
    for q in range(6):
        p.bc[q] = _BC[spec["bc"][q]]
    flags = _EXCH[spec["exchange"]]
    if spec["isothermal"]:
        flags |= RHD_ISOTHERMAL
    if spec["beta_tau"]:
        flags |= RHD_BETA_TAU
    if spec["rad_only"]:
        flags |= RHD_RAD_ONLY
    if spec["precision"] == "mixed":
        flags |= RHD_PRECISION_MIXED
    if spec.get("cv_t3"):
        flags |= RHD_GAS_CV_T3
    if spec.get("kappa_law") is not None:
        flags |= RHD_OPACITY_LAW
        for q in range(5):
            p.kappa_law[q] = float(spec["kappa_law"][q])
    if spec.get("closure", "m1") == "p1":
        flags |= RHD_CLOSURE_P1
    elif spec.get("closure", "m1") != "m1":
        raise ValueError(f"unknown closure {spec['closure']!r}")
    p.flags = flags
    p.cv_alpha = float(spec.get("cv_alpha", 0.0))
    return p


def _flat_state(st, shape):
    """The flat host arrays of a state dict, as rhd_set_state takes them. A field may be a
    full (nz, ny, nx) array or a uniform value (a scalar or a one-element array)."""
    n = int(np.prod(shape))

    def uniform(v):
        return v.size == 1

    def fill(out, k):
        v = np.asarray(st[k], dtype=np.float64)
        if uniform(v):
            out.fill(float(v.reshape(-1)[0]))
        else:
            out[:] = np.broadcast_to(v, shape).reshape(-1)

    def flat(k):
        out = np.empty(n)
        fill(out, k)
        return out

    def flat3(keys):
        out = np.empty(3 * n)
        for i, k in enumerate(keys):
            fill(out[i * n:(i + 1) * n], k)
        return out

    kP = np.asarray(st["kP"], dtype=np.float64)
    kF = np.asarray(st["kF"], dtype=np.float64)
    scalar = ((uniform(kP) or bool(np.all(kP == kP.flat[0]))) and
              (uniform(kF) or bool(np.all(kF == kF.flat[0]))))
    if scalar:
        kPa, kFa = np.array([kP.flat[0]]), np.array([kF.flat[0]])
    else:
        kPa, kFa = flat("kP"), flat("kF")
    return {"rho": flat("rho"), "mom": flat3(("mx", "my", "mz")), "E": flat("E"),
            "Er": flat("Er"), "Fr": flat3(("Fx", "Fy", "Fz")), "kP": kPa, "kF": kFa,
            "scalar": int(scalar), "j": flat("j") if st.get("j") is not None else None}


def _shaped_state(raw, shape):
    """A state dict of (nz, ny, nx) arrays from the flat arrays rhd_get_state fills."""
    N = int(np.prod(shape))
    return {"rho": raw["rho"].reshape(shape), "mx": raw["mom"][:N].reshape(shape),
            "my": raw["mom"][N:2 * N].reshape(shape), "mz": raw["mom"][2 * N:].reshape(shape),
            "E": raw["E"].reshape(shape), "Er": raw["Er"].reshape(shape),
            "Fx": raw["Fr"][:N].reshape(shape), "Fy": raw["Fr"][N:2 * N].reshape(shape),
            "Fz": raw["Fr"][2 * N:].reshape(shape)}


class Solver:
    """One handle: state in, steps, state out. ``state`` dicts hold float64 arrays of
    shape (nz, ny, nx) named rho, mx, my, mz, E, Er, Fx, Fy, Fz, kP, kF and optionally j."""

    def __init__(self, spec, stream=None):
        self.spec = dict(spec)
        self.shape = (spec["nz"], spec["ny"], spec["nx"])
        self.N = int(np.prod(self.shape))
        self.params = params_from_spec(spec)
        self.h = rhd_create(self.params, stream)

    def close(self):
        if self.h:
            rhd_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, st):
        a = _flat_state(st, self.shape)
        rhd_set_state(self.h, a["rho"], a["mom"], a["E"], a["Er"], a["Fr"], a["kP"], a["kF"],
                      a["scalar"])
        rhd_set_emission(self.h, a["j"])

    def step(self, dt_gas, chat, nsub):
        rhd_step(self.h, dt_gas, chat, nsub)

    def run(self, dt_gas, nsub, chat, bvals=None):
        rhd_run(self.h, dt_gas, nsub, chat, bvals)

    def set_boundary(self, bvals):
        """Set every fixed face's radiation state from a 6 x 4 table (x-, x+, y-, y+, z-,
        z+ by (E_r, F_x, F_y, F_z)); rows of other faces are ignored."""
        for f in range(6):
            if self.spec["bc"][f] == "fixed" and self.shape[2 - f // 2] > 1:
                rhd_set_boundary(self.h, f, bvals[f])

    def set_kernel_variant(self, variant, tile_rows=8, zchunk=8):
        rhd_set_kernel_variant(self.h, variant, tile_rows, zchunk)

    def autotune(self, chat, dt_rad, reps=3):
        return rhd_autotune(self.h, chat, dt_rad, reps)

    def set_graph(self, enable):
        rhd_set_graph(self.h, enable)

    def graph_stats(self):
        return rhd_get_graph_stats(self.h)

    def suggest_dt(self, chat):
        return rhd_suggest_dt(self.h, chat)

    def get_state(self):
        return _shaped_state(rhd_get_state(self.h, self.N), self.shape)

    def diagnostics(self):
        return rhd_get_diagnostics(self.h)

    def reset_diagnostics(self):
        rhd_reset_diagnostics(self.h)

    def ledger(self, chat):
        rhd_ledger(self.h, chat)
        return self.diagnostics()["ledger"]

    def sync(self):
        rhd_sync(self.h)


class Server:
    """The native server (rhd_server_*): submit independent 3D solves from any thread,
    wait for them and fetch their final states. Its worker thread admits requests in
    submission order within the memory budget and slot count and advances the running
    ones one gas step per round."""

    def __init__(self, budget_bytes, max_slots, tile_rows=8, zchunk=8):
        self.s = rhd_server_create(budget_bytes, max_slots, tile_rows, zchunk)
        self._shapes = {}

    def submit(self, spec, state, chat, steps):
        shape = (spec["nz"], spec["ny"], spec["nx"])
        a = _flat_state(state, shape)
        rid = rhd_server_submit(self.s, params_from_spec(spec), a["rho"], a["mom"], a["E"],
                                a["Er"], a["Fr"], a["kP"], a["kF"], a["scalar"], a["j"], steps,
                                chat)
        self._shapes[rid] = shape
        return rid

    def poll(self, rid):
        return rhd_server_poll(self.s, rid)

    def wait(self, rid, timeout_s=-1.0):
        return rhd_server_wait(self.s, rid, timeout_s)

    def fetch(self, rid):
        """(state dict, diagnostics, code) of a finished request; see rhd_server_fetch."""
        shape = self._shapes[rid]
        raw, diag, rc = rhd_server_fetch(self.s, rid, int(np.prod(shape)))
        del self._shapes[rid]
        return _shaped_state(raw, shape), diag, rc

    def cancel(self, rid):
        rhd_server_cancel(self.s, rid)

    def stats(self):
        return rhd_server_get_stats(self.s)

    def close(self):
        if self.s:
            rhd_server_destroy(self.s)
            self.s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
