"""GPU check of the size limit of the tiled radiation kernels: they address with 32-bit
byte offsets, so a handle whose padded arrays exceed 4 GiB each refuses them and runs
the per-cell kernels, while one just below the limit accepts them. (FP64, radiation
only: about 60 GB of device memory per handle, nothing stepped.)"""
import sys

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
