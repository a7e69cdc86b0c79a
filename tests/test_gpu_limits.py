"""GPU check of the size limit of the tiled radiation kernels: they address with 32-bit
byte offsets, so a handle whose padded arrays exceed 4 GiB each refuses them and runs
the per-cell kernels, while one just below the limit accepts them. (FP64, radiation
only: about 60 GB of device memory per handle, nothing stepped.)"""
import sys

import numpy as np

import pytest

import paper_1306_0010_amd as P
import rhd_inputs as ri

pytestmark = pytest.mark.gpu


def big_handle(n):
    spec = ri.default_spec(nx=n, ny=n, nz=n, dx=1.0 / n, dy=1.0 / n, dz=1.0 / n, rad_only=True,
                           exchange="none", precision="fp64")
    return P.rhd_create(P.params_from_spec(spec))


@pytest.mark.parametrize("n,tiled_ok", [(820, False), (808, True)])
def test_tiled_kernels_need_arrays_below_4_gib(n, tiled_ok):
    print(f"[gpu case] limits {n}^3 fp64", flush=True)
    sys.stdout.flush()
    padded_bytes = (n + 4) ** 3 * 8
    assert (padded_bytes <= 2 ** 32) == tiled_ok
    h = big_handle(n)
    try:
        P.rhd_set_kernel_variant(h, P.RHD_KERNELS_PER_CELL, 8, 8)
        if tiled_ok:
            P.rhd_set_kernel_variant(h, P.RHD_KERNELS_TILED, 8, 8)
        else:
            with pytest.raises(P.RhdError) as e:
                P.rhd_set_kernel_variant(h, P.RHD_KERNELS_TILED, 8, 8)
            assert e.value.code == P.RHD_EINVAL
    finally:
        P.rhd_destroy(h)


def test_binding_checks_array_sizes_before_the_call():
    """The binding knows each handle's cell count and refuses arrays of another size
    before the C function could read or write past them."""
    print("[gpu case] binding array sizes", flush=True)
    spec = ri.default_spec(nx=8, ny=6, nz=4, dx=1 / 8, dy=1 / 6, dz=1 / 4)
    st = ri.smooth_random_state(spec, seed=3)
    h = P.rhd_create(P.params_from_spec(spec))
    n = 8 * 6 * 4
    try:
        flat = lambda k: st[k].ravel()
        mom = lambda: np.stack([st["mx"], st["my"], st["mz"]]).ravel()
        fr = lambda: np.stack([st["Fx"], st["Fy"], st["Fz"]]).ravel()
        with pytest.raises(ValueError):
            P.rhd_set_state(h, flat("rho")[:-1], mom(), flat("E"), flat("Er"), fr(),
                            flat("kP"), flat("kF"), 0)
        with pytest.raises(ValueError):
            P.rhd_set_state(h, flat("rho"), mom(), flat("E"), flat("Er"), fr()[: 3 * n - 3],
                            flat("kP"), flat("kF"), 0)
        with pytest.raises(ValueError):
            P.rhd_get_state(h, n + 1)
        with pytest.raises(ValueError):
            P.rhd_set_emission(h, np.ones(n - 1))
        P.rhd_set_state(h, flat("rho"), mom(), flat("E"), flat("Er"), fr(), flat("kP"),
                        flat("kF"), 0)
        out = P.rhd_get_state(h, n)
        assert np.allclose(out["rho"], flat("rho"))
    finally:
        P.rhd_destroy(h)
    with pytest.raises(ValueError):
        P.rhd_get_state(h, n)  # destroyed


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,rad_only", [((24, 20, 12), False), ((24, 20, 12), True),
                                            ((40, 18, 1), False), ((100, 1, 1), True)])
def test_footprint_equals_a_new_handles_device_bytes(precision, shape, rad_only):
    """rhd_footprint_bytes, which the server's budget counts, is what a created handle
    holds; per-cell opacities and an emissivity add their own arrays on top."""
    print(f"[gpu case] footprint {shape} {precision} rad_only={rad_only}", flush=True)
    nx, ny, nz = shape
    spec = ri.default_spec(nx=nx, ny=ny, nz=nz, dx=1 / nx, dy=1 / max(ny, 1), dz=1 / max(nz, 1),
                           rad_only=rad_only, exchange="none" if rad_only else "full",
                           precision=precision)
    p = P.params_from_spec(spec)
    h = P.rhd_create(p)
    try:
        assert P.rhd_device_bytes(h) == P.rhd_footprint_bytes(p)
        st = ri.smooth_random_state(spec, seed=5)
        n = nx * ny * nz
        es = 4 if precision == "mixed" else 8
        mom = np.stack([st["mx"], st["my"], st["mz"]]).ravel()
        fr = np.stack([st["Fx"], st["Fy"], st["Fz"]]).ravel()
        P.rhd_set_state(h, st["rho"].ravel(), mom, st["E"].ravel(), st["Er"].ravel(), fr,
                        st["kP"].ravel(), st["kF"].ravel(), 0)
        assert P.rhd_device_bytes(h) == P.rhd_footprint_bytes(p) + 2 * n * es
        P.rhd_set_emission(h, np.full(n, 0.5))
        assert P.rhd_device_bytes(h) == P.rhd_footprint_bytes(p) + 3 * n * es
    finally:
        P.rhd_destroy(h)
