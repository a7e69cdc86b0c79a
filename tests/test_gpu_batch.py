"""GPU checks of the batch of independent solves (the served form): a member's result
is the same bit for bit whatever else is in the batch and whenever others join or
leave; it equals what the handle computes alone to rounding; the served results equal
the one-at-a-time results to rounding; an FP64 member matches the oracle."""
import sys

import numpy as np
import pytest

import oracle
import paper_1306_0010_amd as P
import rhd_inputs as ri
from paper_1306_0010_amd import serve
from parity import assert_parity

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def problem(n, kappa, chat_over_a0, seed, precision="mixed"):
    req = dict(id=seed, nx=n[0], ny=n[1], nz=n[2], kappa=kappa, chat_over_a0=chat_over_a0,
               steps=3, arrival=0.0, seed=seed)
    return ri.c5_problem(req, precision=precision)


PROBLEMS = [((40, 24, 20), 3.0, 8.0, 11), ((33, 48, 17), 50.0, 20.0, 12), ((64, 20, 30), 300.0, 40.0, 13)]


def alone(pb, steps, rows=8, zchunk=16):
    with P.Solver(pb["spec"]) as s:
        s.set_kernel_variant(P.RHD_KERNELS_TILED, rows, zchunk)
        s.set_state(pb["state"])
        for _ in range(steps):
            dt, ns = s.suggest_dt(pb["chat"])
            s.step(dt, pb["chat"], ns)
        return s.get_state()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_members_equal_single_handles(precision):
    announce(f"batch members {precision}")
    pbs = [problem(*p, precision=precision) for p in PROBLEMS]
    ref = [alone(pb, 3) for pb in pbs]
    b = P.rhd_batch_create(8, 8, 16)
    solvers = []
    try:
        for pb in pbs:
            s = P.Solver(pb["spec"])
            s.set_state(pb["state"])
            P.rhd_batch_add(b, s.h, pb["chat"])
            solvers.append(s)
        for _ in range(3):
            ns, dts = P.rhd_batch_step(b)
            assert len(ns) == 3 and all(n >= 1 for n in ns)
        outs = [s.get_state() for s in solvers]
        for s in solvers:
            P.rhd_batch_remove(b, s.h)
    finally:
        P.rhd_batch_destroy(b)
        for s in solvers:
            s.close()
    # the batch launches other kernels (same device code) than a lone handle, so the
    # compiler may fuse multiply-adds differently: equal to rounding, not bit for bit
    for pb, o, r in zip(pbs, outs, ref):
        assert_parity(pb["spec"], o, r, 1e-13 if precision == "fp64" else 1e-6, "max",
                      label="batch member vs lone handle")


def test_member_result_does_not_depend_on_the_mix():
    """Solve A alone in a batch, and A with others joining after its first step and one
    leaving after its second: A's final state is identical bit for bit."""
    announce("alone vs mix")
    pa, pb_, pc = (problem(*p) for p in PROBLEMS)

    def run(with_others):
        b = P.rhd_batch_create(8, 8, 16)
        sv = []
        try:
            a = P.Solver(pa["spec"])
            a.set_state(pa["state"])
            sv.append(a)
            P.rhd_batch_add(b, a.h, pa["chat"])
            P.rhd_batch_step(b)
            others = []
            if with_others:
                for q in (pb_, pc):
                    s = P.Solver(q["spec"])
                    s.set_state(q["state"])
                    sv.append(s)
                    others.append(s)
                    P.rhd_batch_add(b, s.h, q["chat"])
            P.rhd_batch_step(b)
            if with_others:
                P.rhd_batch_remove(b, others[0].h)
            P.rhd_batch_step(b)
            out = a.get_state()
            for s in sv:
                if s.h is not None:
                    try:
                        P.rhd_batch_remove(b, s.h)
                    except P.RhdError:
                        pass
            return out
        finally:
            P.rhd_batch_destroy(b)
            for s in sv:
                s.close()

    x, y = run(False), run(True)
    for k in ri.FIELDS:
        assert np.array_equal(x[k], y[k]), k


def test_fp64_member_matches_oracle():
    announce("batch fp64 vs oracle")
    pb = problem((26, 18, 14), 20.0, 10.0, 21, precision="fp64")
    spec, st, chat = pb["spec"], pb["state"], pb["chat"]
    dt, ns, _ = oracle.suggest_dt(spec, st, chat)
    ref, _ = oracle.step(spec, st, dt, chat, ns)
    b = P.rhd_batch_create(4, 4, 5)
    s = P.Solver(spec)
    try:
        s.set_state(st)
        P.rhd_batch_add(b, s.h, chat)
        nsb, dtb = P.rhd_batch_step(b)
        assert nsb == [ns] and dtb[0] == pytest.approx(dt, rel=1e-13)
        gpu = s.get_state()
        P.rhd_batch_remove(b, s.h)
    finally:
        P.rhd_batch_destroy(b)
        s.close()
    assert_parity(spec, gpu, ref, 1e-12, "max", label="batch member")


def test_batch_rejects_bad_members():
    announce("batch errors")
    spec2d = ri.default_spec(nx=16, ny=16, dx=1 / 16, dy=1 / 16)
    st = ri.smooth_random_state(spec2d, seed=1)
    b = P.rhd_batch_create(1, 8, 16)
    s2 = P.Solver(spec2d)
    pm = problem(*PROBLEMS[0])
    pf = problem(*PROBLEMS[1], precision="fp64")
    s3, s4 = P.Solver(pm["spec"]), P.Solver(pf["spec"])
    try:
        with pytest.raises(P.RhdError):
            P.rhd_batch_add(b, s3.h, pm["chat"])  # no state yet
        s2.set_state(st)
        with pytest.raises(P.RhdError):
            P.rhd_batch_add(b, s2.h, 1.0)  # 2D
        s3.set_state(pm["state"])
        P.rhd_batch_add(b, s3.h, pm["chat"])
        s4.set_state(pf["state"])
        with pytest.raises(P.RhdError):
            P.rhd_batch_add(b, s4.h, pf["chat"])  # full, and precision differs
        P.rhd_batch_remove(b, s3.h)
    finally:
        P.rhd_batch_destroy(b)
        for s in (s2, s3, s4):
            s.close()


def test_destroying_a_member_removes_it_from_its_batch():
    """rhd_destroy on a batch member takes it out of the batch first: the batch shrinks
    and steps its remaining member, whose result still equals its lone run."""
    announce("destroy a batch member")
    pa, pb_ = problem(*PROBLEMS[0]), problem(*PROBLEMS[2])
    b = P.rhd_batch_create(2, 8, 16)
    sa, sb = P.Solver(pa["spec"]), P.Solver(pb_["spec"])
    try:
        sa.set_state(pa["state"])
        sb.set_state(pb_["state"])
        P.rhd_batch_add(b, sa.h, pa["chat"])
        P.rhd_batch_add(b, sb.h, pb_["chat"])
        assert P.rhd_batch_size(b) == 2
        sb.close()  # rhd_destroy of a member
        assert P.rhd_batch_size(b) == 1
        for _ in range(2):
            P.rhd_batch_step(b)
        P.rhd_batch_sync(b)
        got = sa.get_state()
    finally:
        P.rhd_batch_destroy(b)
        sa.close()
    ref = alone(pa, 2)
    assert_parity(pa["spec"], got, ref, 1e-6, "max", label="remaining member vs alone")


def test_served_results_equal_one_at_a_time_results():
    """Continuous batching with staggered arrivals and a memory budget that admits only
    part of the stream at once gives every request its one-at-a-time result (to FP32
    rounding: the two paths launch different kernels over the same device code)."""
    announce("serve small stream")
    reqs = ri.c5_requests(count=7, seed=5, sizes=(16, 24, 32, 40))
    for i, r in enumerate(reqs):
        r["steps"] = 3
        r["arrival"] = 0.002 * i
    make = lambda r: ri.c5_problem(r)
    fp = [P.rhd_footprint_bytes(P.params_from_spec(make(r)["spec"])) for r in reqs]
    budget = int(sum(sorted(fp)[-3:]))
    a, ra = serve.serve_batched(reqs, make, budget_bytes=budget, max_slots=4, keep_results=True)
    b, rb = serve.serve_serial(reqs, make, keep_results=True, variant=serve.DEFAULT_VARIANT)
    assert a["requests"] == b["requests"] == 7
    assert a["zone_updates"] == b["zone_updates"]
    assert 1 <= a["peak_active"] <= 4
    for r in reqs:
        assert_parity(make(r)["spec"], ra[r["id"]], rb[r["id"]], 1e-6, "max",
                      label=f"request {r['id']} served vs one at a time")


def test_concurrent_served_results_equal_one_at_a_time_results():
    """Serving with one handle and stream per admitted solve, steps of different solves in
    flight together, a memory budget and a slot limit: every request gets exactly its
    one-at-a-time result (same kernels, same tile shape, so bit for bit)."""
    announce("serve small stream concurrently")
    reqs = ri.c5_requests(count=7, seed=6, sizes=(16, 24, 32, 40))
    for i, r in enumerate(reqs):
        r["steps"] = 3
        r["arrival"] = 0.002 * i
    make = lambda r: ri.c5_problem(r)
    fp = [P.rhd_footprint_bytes(P.params_from_spec(make(r)["spec"])) for r in reqs]
    budget = int(sum(sorted(fp)[-3:]))
    a, ra = serve.serve_concurrent(reqs, make, budget_bytes=budget, max_slots=4,
                                   variant=serve.DEFAULT_VARIANT, keep_results=True)
    b, rb = serve.serve_serial(reqs, make, keep_results=True, variant=serve.DEFAULT_VARIANT)
    assert a["requests"] == b["requests"] == 7
    assert a["zone_updates"] == b["zone_updates"]
    assert 1 <= a["peak_active"] <= 4
    for r in reqs:
        for k in ri.FIELDS:
            assert np.array_equal(ra[r["id"]][k], rb[r["id"]][k]), (r["id"], k)


def run_batch(pbs, steps, persistent, rows=8, zchunk=16):
    b = P.rhd_batch_create(8, rows, zchunk)
    solvers, nsubs = [], []
    try:
        P.rhd_batch_set_persistent(b, persistent)
        for pb in pbs:
            s = P.Solver(pb["spec"])
            s.set_state(pb["state"])
            P.rhd_batch_add(b, s.h, pb["chat"])
            solvers.append(s)
        for _ in range(steps):
            ns, _ = P.rhd_batch_step(b)
            nsubs.append(list(ns))
        P.rhd_batch_sync(b)
        outs = [s.get_state() for s in solvers]
        for s in solvers:
            P.rhd_batch_remove(b, s.h)
    finally:
        P.rhd_batch_destroy(b)
        for s in solvers:
            s.close()
    return outs, nsubs


@pytest.mark.skip(reason="the persistent launch is switched off: twice it did not finish on the "
                         "GPU (this test's batch, three members; no end within 120-180 s), and its "
                         "cause is not found; rhd_batch_set_persistent(b, 1) returns RHD_EINVAL")
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_persistent_launch_equals_round_launches(precision):
    """The persistent launch (one launch for all subcycles of all members, per-member
    phase counters) computes every tile with the same device code as the round launches:
    the members' states agree to rounding (the two kernels may contract multiply-adds
    differently). Members span 5 to ~40 subcycles per gas step and 16^3 to 64x20x30
    cells, so members finish their subcycles at different levels of the launch."""
    announce(f"persistent vs rounds {precision}")
    probs = PROBLEMS + [((16, 16, 16), 1.0, 5.0, 14), ((24, 17, 40), 1000.0, 45.0, 15)]
    pbs = [problem(*p, precision=precision) for p in probs]
    per, ns_p = run_batch(pbs, 3, True)
    rnd, ns_r = run_batch(pbs, 3, False)
    assert ns_p == ns_r
    assert len(set(ns_p[0])) >= 3, ns_p
    for pb, a, r in zip(pbs, per, rnd):
        assert_parity(pb["spec"], a, r, 1e-13 if precision == "fp64" else 1e-6, "max",
                      label="persistent vs rounds")


def test_persistent_launch_is_refused():
    """Asking a batch or a server for the switched-off persistent launch is an error that
    changes nothing; rounds stay available. Host calls only."""
    b = P.rhd_batch_create(2, 8, 8)
    try:
        with pytest.raises(P.RhdError) as e:
            P.rhd_batch_set_persistent(b, 1)
        assert e.value.code == P.RHD_EINVAL and "switched off" in str(e.value)
        P.rhd_batch_set_persistent(b, 0)
    finally:
        P.rhd_batch_destroy(b)
    with P.Server(1 << 30, 2) as srv:
        with pytest.raises(P.RhdError) as e:
            P.rhd_server_set_persistent(srv.s, 1)
        assert e.value.code == P.RHD_EINVAL
        P.rhd_server_set_persistent(srv.s, 0)
