"""Comparison helpers shared by the GPU parity tests (test code, no method arithmetic).

Errors are measured per field against a natural scale of that field, so fields that
vanish in the background (momentum, radiation flux) are not divided by zero:
rho, E, E_r are their own scale, momentum is compared to sqrt(rho E) and the radiation
flux to c E_r.
"""
import numpy as np

import rhd_inputs as ri

FIELDS = ri.FIELDS


def scales(spec, st):
    c = spec["c_light"]
    mom = np.sqrt(np.abs(st["rho"] * np.where(spec["isothermal"], st["rho"] * spec["iso_cs"] ** 2,
                                             np.abs(st["E"]))))
    return {"rho": np.abs(st["rho"]), "E": np.abs(st["E"]), "Er": np.abs(st["Er"]),
            "mx": mom, "my": mom, "mz": mom,
            "Fx": c * np.abs(st["Er"]), "Fy": c * np.abs(st["Er"]), "Fz": c * np.abs(st["Er"])}


def field_errors(spec, gpu, ref, fields=FIELDS):
    """{field: (max abs error / max scale, L1 error / L1 scale)}."""
    sc = scales(spec, ref)
    out = {}
    for k in fields:
        if spec["isothermal"] and k == "E":
            continue
        d = np.abs(np.asarray(gpu[k], dtype=np.float64) - np.asarray(ref[k], dtype=np.float64))
        s = sc[k]
        smax = float(s.max())
        if smax == 0.0:
            out[k] = (float(d.max()), float(d.sum()))
        else:
            out[k] = (float(d.max()) / smax, float(d.sum()) / float(s.sum()))
    return out


def assert_parity(spec, gpu, ref, tol, norm="max", fields=FIELDS, label=""):
    errs = field_errors(spec, gpu, ref, fields)
    idx = 0 if norm == "max" else 1
    worst = max(errs.items(), key=lambda kv: kv[1][idx])
    assert worst[1][idx] <= tol, f"{label}: worst field {worst[0]} {norm} error {worst[1][idx]:.3e} > {tol:.1e}; all: " + \
        ", ".join(f"{k}={v[idx]:.2e}" for k, v in errs.items())
    return errs


def window(state, lo, size, bc_modes):
    """Sub-box [lo, lo+size) of every array in ``state`` (shape (nz, ny, nx)), reading
    past the grid edge with numpy pad modes per axis ('wrap' for periodic, 'edge' for
    outflow). lo and size are (x, y, z)."""
    out = {}
    for k, v in state.items():
        if not isinstance(v, np.ndarray):
            out[k] = v
            continue
        a = v
        sl = []
        for ax_arr, ax_xyz in ((0, 2), (1, 1), (2, 0)):
            n = a.shape[ax_arr]
            l, s = lo[ax_xyz], size[ax_xyz]
            idx = np.arange(l, l + s)
            if bc_modes[ax_xyz] == "wrap":
                idx = np.mod(idx, n)
            else:
                idx = np.clip(idx, 0, n - 1)
            sl.append(idx)
        out[k] = a[np.ix_(*sl)].copy()
    return out
