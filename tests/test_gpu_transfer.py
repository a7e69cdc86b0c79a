"""GPU checks of the host transfers (rhd_set_state, rhd_get_state): the host arrays travel
through pairs of pinned chunks (4 MiB each), converted to FP32 on the host in mixed
precision. A state copied in and straight out again must come back as the IEEE
round-to-nearest FP32 value of each input (mixed) or unchanged (FP64), at sizes below one
chunk, exactly one and several with a ragged tail; and the host conversion must equal the
device's (rhd_set_state_device, which converts with a kernel), subnormal FP32 results
included."""
import numpy as np
import pytest

import paper_1306_0010_amd as P
import rhd_inputs as ri

pytestmark = pytest.mark.gpu

CHUNK = 4 << 20  # bytes of one pinned chunk


def values(rng, n):
    """Positive and negative values over many decades, with FP32 ties, values that round
    up to the next binade, FP32 subnormals and exact zeros sprinkled in."""
    v = rng.standard_normal(n) * 10.0 ** rng.integers(-30, 30, n)
    k = max(1, n // 50)
    idx = rng.choice(n, size=5 * k, replace=False)
    f = np.float32(1.0) + np.float32(2.0 ** -23) * rng.integers(0, 1 << 10, k).astype(np.float32)
    v[idx[:k]] = f.astype(np.float64) + 2.0 ** -24          # exact ties between FP32 values
    v[idx[k:2 * k]] = 1.0 - 2.0 ** -26                        # rounds up to 1.0 in FP32
    v[idx[2 * k:3 * k]] = 1e-40 * rng.standard_normal(k)      # FP32 subnormals
    v[idx[3 * k:4 * k]] = 0.0
    v[idx[4 * k:]] = -v[idx[4 * k:]]
    return v


def make_state(spec, seed):
    n = spec["nx"] * spec["ny"] * spec["nz"]
    rng = np.random.default_rng(seed)
    return {"rho": values(rng, n), "mom": values(rng, 3 * n), "E": values(rng, n),
            "Er": values(rng, n), "Fr": values(rng, 3 * n), "kP": np.abs(values(rng, n)),
            "kF": np.abs(values(rng, n))}


def spec_for(shape, precision):
    nx, ny, nz = shape
    return ri.default_spec(nx=nx, ny=ny, nz=nz, dx=1 / nx, dy=1 / ny, dz=1 / nz,
                           precision=precision)


def put(h, st):
    P.rhd_set_state(h, st["rho"], st["mom"], st["E"], st["Er"], st["Fr"], st["kP"], st["kF"], 0)


# below one chunk; exactly one FP32 chunk (two FP64 ones); several with a ragged tail
SHAPES = [(7, 5, 3), (128, 128, 64), (150, 130, 120)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_state_comes_back_rounded_once(precision, shape):
    print(f"[gpu case] transfer round trip {shape} {precision}", flush=True)
    spec = spec_for(shape, precision)
    n = shape[0] * shape[1] * shape[2]
    es = 4 if precision == "mixed" else 8
    if shape == (128, 128, 64):
        assert n * 4 == CHUNK
    st = make_state(spec, seed=sum(shape))
    h = P.rhd_create(P.params_from_spec(spec))
    try:
        put(h, st)
        out = P.rhd_get_state(h, n)
    finally:
        P.rhd_destroy(h)
    assert n * es >= CHUNK or shape == (7, 5, 3)
    for k in ("rho", "mom", "E", "Er", "Fr"):
        want = st[k].astype(np.float32).astype(np.float64) if precision == "mixed" else st[k]
        np.testing.assert_array_equal(out[k].view(np.uint64), want.view(np.uint64), err_msg=k)


@pytest.mark.parametrize("shape", SHAPES[::2])
def test_host_conversion_equals_the_devices(shape):
    """The same FP64 values given as device arrays (converted by a kernel) and as host
    arrays (converted on the host) leave the same FP32 state, bit for bit."""
    import torch
    print(f"[gpu case] host vs device conversion {shape}", flush=True)
    spec = spec_for(shape, "mixed")
    n = shape[0] * shape[1] * shape[2]
    st = make_state(spec, seed=7 + sum(shape))
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(v).to(dev) for k, v in st.items()}
    torch.cuda.synchronize(dev)
    outs = []
    for device_path in (False, True):
        h = P.rhd_create(P.params_from_spec(spec))
        try:
            if device_path:
                P.rhd_set_state_device(h, t["rho"].data_ptr(), t["mom"].data_ptr(),
                                       t["E"].data_ptr(), t["Er"].data_ptr(), t["Fr"].data_ptr(),
                                       t["kP"].data_ptr(), t["kF"].data_ptr(), 0)
            else:
                put(h, st)
            outs.append(P.rhd_get_state(h, n))
        finally:
            P.rhd_destroy(h)
    for k in ("rho", "mom", "E", "Er", "Fr"):
        np.testing.assert_array_equal(outs[0][k].view(np.uint64), outs[1][k].view(np.uint64),
                                      err_msg=k)
