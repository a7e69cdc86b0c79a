"""HIP graphs of the radiation subcycle loop (rhd_set_graph): the captured loop replays
the same kernels with the same arguments, so every step's state must equal the state
of the same step launched kernel by kernel, bit for bit. Each replay is checked against
the eager run, with the program's own work (ledger, state copies, synchronisations)
between the replays."""
import sys

import numpy as np
import pytest

import paper_1306_0010_amd as P
import rhd_inputs as ri

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def trajectory(spec, st, chat, schedule, graph):
    """States after every step of `schedule` ((dt, nsub) pairs), with graphs on or off."""
    out = []
    with P.Solver(spec) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, 8, 8)
        s.set_graph(graph)
        s.set_state(st)
        for dt, ns in schedule:
            s.step(dt, chat, ns)
            s.sync()
            out.append(s.get_state())
            s.ledger(chat)
        stats = s.graph_stats()
    return out, stats


def assert_same_steps(a, b, label):
    for k, (x, y) in enumerate(zip(a, b)):
        for f in ri.FIELDS:
            assert np.array_equal(x[f], y[f]), (label, k, f)


def cases():
    out = []
    for shape, prec in (((48, 40, 24), "mixed"), ((40, 24, 20), "fp64"), ((64, 48, 1), "mixed"),
                        ((200, 1, 1), "fp64")):
        nx, ny, nz = shape
        spec = ri.default_spec(nx=nx, ny=ny, nz=nz, dx=1.0 / nx, dy=1.0 / ny, dz=1.0 / nz,
                               c_light=30.0, exchange="full", theta_E=0.51, bc="periodic",
                               precision=prec)
        st = ri.smooth_random_state(spec, seed=31, amp=0.1, f_amp=0.3, kappa=(2.0, 2.0),
                                    v_amp=0.1)
        out.append((f"{prec} {shape}", spec, st))
    return out


@pytest.mark.parametrize("label,spec,st", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_graph_replays_equal_eager_steps(label, spec, st):
    """Five steps of one size: one capture, four replays, each step's state equal to the
    eager run's; then steps of changing size: each new key is captured again."""
    announce(f"graph {label}")
    chat = 6.0
    dxm = min(spec["dx"] if spec["nx"] > 1 else 1e9, spec["dy"] if spec["ny"] > 1 else 1e9,
              spec["dz"] if spec["nz"] > 1 else 1e9)
    ns = 4
    dt = 0.4 * dxm / chat * ns * 0.99
    fixed = [(dt, ns)] * 5
    eager, st0 = trajectory(spec, st, chat, fixed, False)
    graph, st1 = trajectory(spec, st, chat, fixed, True)
    assert st0 == (0, 0) and st1 == (1, 4), st1
    assert_same_steps(graph, eager, label + " fixed")
    varying = [(dt, ns), (0.9 * dt, ns), (0.9 * dt, ns), (0.7 * dt, 3), (0.7 * dt, 3)]
    eager, _ = trajectory(spec, st, chat, varying, False)
    graph, st2 = trajectory(spec, st, chat, varying, True)
    assert st2 == (3, 2), st2
    assert_same_steps(graph, eager, label + " varying")
