"""GPU checks of the native server (rhd_server_*, the served form behind the C interface):
its results equal those of the same solves in a batch bit for bit and those of lone
handles to rounding; a request larger than the memory budget is refused at submission
and the others run within the budget; cancelling a running or queued request frees its
slot and leaves every other result unchanged bit for bit; a failing request fails alone;
waiting with a time limit and destroying a busy server both return; the benchmark's own
stream, at full size, equals its requests run alone, and one served gas step of its
smallest request matches the oracle."""
import sys
import time

import numpy as np
import pytest

import paper_1306_0010_amd as P
import rhd_inputs as ri
from paper_1306_0010_amd import serve
from parity import assert_parity

pytestmark = pytest.mark.gpu


def announce(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def stream(count, seed, steps=3, sizes=(16, 24, 32, 40)):
    reqs = ri.c5_requests(count=count, seed=seed, sizes=sizes)
    for i, r in enumerate(reqs):
        r["steps"] = steps
        r["arrival"] = 0.002 * i
    return reqs


def footprint(pb):
    return P.rhd_footprint_bytes(P.params_from_spec(pb["spec"]))


def wait_until(pred, limit_s=30.0):
    t = time.perf_counter()
    while not pred():
        assert time.perf_counter() - t < limit_s, "condition not reached"
        time.sleep(0.001)


def test_native_server_results_equal_batch_results():
    """The same stream through the native server, through the Python batching loop with
    the same tile shape (bit for bit: the same batched kernels, and a member's result
    does not depend on the mix) and one request at a time (to FP32 rounding)."""
    announce("native server vs batch vs one at a time")
    reqs = stream(7, seed=7)
    make = lambda r: ri.c5_problem(r)
    budget = int(sum(sorted(footprint(make(r)) for r in reqs)[-3:]))
    a, ra = serve.serve_native(reqs, make, budget_bytes=budget, max_slots=4, keep_results=True)
    b, rb = serve.serve_batched(reqs, make, budget_bytes=budget, max_slots=4, keep_results=True)
    c, rc = serve.serve_serial(reqs, make, keep_results=True, variant=serve.DEFAULT_VARIANT)
    assert a["requests"] == b["requests"] == c["requests"] == 7
    assert a["zone_updates"] == c["zone_updates"]
    assert 1 <= a["peak_active"] <= 4 and a["peak_bytes"] <= budget
    for r in reqs:
        for k in ri.FIELDS:
            assert np.array_equal(ra[r["id"]][k], rb[r["id"]][k]), (r["id"], k)
        assert_parity(make(r)["spec"], ra[r["id"]], rc[r["id"]], 1e-6, "max",
                      label=f"request {r['id']} native server vs one at a time")


def test_served_stream_at_full_size():
    """The served-batch workload's own requests (the benchmark's stream: seeds, grids up
    to 192^3, 20 gas steps each) through the native server as the benchmark runs it, all
    queued at once: every result equals the same request run alone to FP32 rounding. The
    smallest of them, one gas step served, matches the FP64 oracle on its whole box."""
    import oracle
    announce("served stream at full size")
    reqs = [dict(r, arrival=0.0) for r in ri.c5_requests(count=8)]
    make = lambda r: ri.c5_problem(r)
    a, ra = serve.serve_native(reqs, make, keep_results=True)
    c, rc = serve.serve_serial(reqs, make, keep_results=True, variant=serve.DEFAULT_VARIANT)
    assert a["requests"] == c["requests"] == 8 and a["zone_updates"] == c["zone_updates"]
    assert max(r["nx"] * r["ny"] * r["nz"] for r in reqs) >= 128 ** 3
    for r in reqs:
        assert_parity(make(r)["spec"], ra[r["id"]], rc[r["id"]], 1e-6, "max",
                      label=f"request {r['id']} ({r['nx']}x{r['ny']}x{r['nz']}) native vs alone")
    small = dict(min(reqs, key=lambda r: r["nx"] * r["ny"] * r["nz"]), steps=1)
    pb = make(small)
    _, rs = serve.serve_native([small], make, keep_results=True)
    spec64 = dict(pb["spec"], precision="fp64")
    dt, ns, _ = oracle.suggest_dt(spec64, pb["state"], pb["chat"])
    ref, _ = oracle.step(spec64, pb["state"], dt, pb["chat"], ns)
    assert_parity(pb["spec"], rs[small["id"]], ref, 1e-5, "l1",
                  label=f"request {small['id']} one gas step vs oracle")


def test_over_budget_request_is_refused_and_the_rest_run_within_budget():
    announce("server budget")
    small = [ri.c5_problem(r) for r in stream(4, seed=8, sizes=(24,))]
    big = ri.c5_problem(stream(1, seed=9, sizes=(64,))[0])
    budget = max(footprint(pb) for pb in small) * 3 // 2
    assert footprint(big) > budget
    with P.Server(budget, 8) as srv:
        with pytest.raises(P.RhdError) as e:
            srv.submit(big["spec"], big["state"], big["chat"], 2)
        assert e.value.code == P.RHD_ENOMEM
        ids = [srv.submit(pb["spec"], pb["state"], pb["chat"], 2) for pb in small]
        for rid in ids:
            info = srv.wait(rid, 60.0)
            assert info["status"] == "done" and info["steps_done"] == 2
            assert 0.0 <= info["t_submit"] <= info["t_start"] <= info["t_done"]
            _, diag, code = srv.fetch(rid)
            assert code == P.RHD_OK and diag["steps"] == 2 and diag["nonfinite"] == 0
        st = srv.stats()
    # only one small request fits the budget at a time
    assert st["rejected"] == 1 and st["submitted"] == 4 and st["completed"] == 4
    assert st["peak_running"] == 1 and 0 < st["peak_bytes"] <= budget
    assert st["bytes_in_use"] == 0 and st["running"] == 0 and st["queued"] == 0


def test_cancel_running_and_queued_requests_leaves_others_unchanged():
    announce("server cancel")
    pbs = [ri.c5_problem(r) for r in stream(3, seed=10, sizes=(24, 32))]
    long_pb, others = pbs[0], pbs[1:]

    def run(with_long):
        out = {}
        with P.Server(1 << 40, 4) as srv:
            lid = None
            if with_long:
                lid = srv.submit(long_pb["spec"], long_pb["state"], long_pb["chat"], 1_000_000)
                wait_until(lambda: srv.poll(lid)["steps_done"] >= 2)
            ids = [srv.submit(pb["spec"], pb["state"], pb["chat"], 3) for pb in others]
            if with_long:
                wait_until(lambda: srv.poll(ids[0])["steps_done"] >= 1)
                srv.cancel(lid)
                info = srv.wait(lid, 60.0)
                assert info["status"] == "cancelled" and info["steps_done"] >= 2
                with pytest.raises(P.RhdError) as e:
                    srv.fetch(lid)
                assert e.value.code == P.RHD_ESTATE
            for i, rid in enumerate(ids):
                assert srv.wait(rid, 60.0)["status"] == "done"
                out[i], _, code = srv.fetch(rid)
                assert code == P.RHD_OK
            st = srv.stats()
            assert st["cancelled"] == (1 if with_long else 0) and st["bytes_in_use"] == 0
        return out

    ref, got = run(False), run(True)
    for i in ref:
        for k in ri.FIELDS:
            assert np.array_equal(ref[i][k], got[i][k]), (i, k)

    # a queued request is dropped at once; a finished one is forgotten by cancel
    with P.Server(1 << 40, 1) as srv:
        a = srv.submit(long_pb["spec"], long_pb["state"], long_pb["chat"], 1_000_000)
        b = srv.submit(others[0]["spec"], others[0]["state"], others[0]["chat"], 3)
        wait_until(lambda: srv.poll(a)["status"] == "running")
        assert srv.poll(b)["status"] == "queued"
        srv.cancel(b)
        assert srv.poll(b)["status"] == "cancelled"
        with pytest.raises(P.RhdError) as e:
            srv.wait(a, 0.0)
        assert e.value.code == P.RHD_ETIMEOUT
        srv.cancel(a)
        assert srv.wait(a, 60.0)["status"] == "cancelled"
        srv.cancel(a)
        with pytest.raises(P.RhdError) as e:
            srv.poll(a)
        assert e.value.code == P.RHD_EINVAL


def test_failing_request_fails_alone():
    """A request whose state holds a non-finite value fails with RHD_ENONFINITE; the
    requests beside it (FP64 and mixed, two batches) finish as if it had never come."""
    announce("server failure isolation")
    reqs = stream(3, seed=11, sizes=(16, 24))
    pbs = [ri.c5_problem(reqs[0], precision="fp64"), ri.c5_problem(reqs[1], precision="fp64"),
           ri.c5_problem(reqs[2])]
    bad = ri.copy_state(pbs[0]["state"])
    bad["Er"][1, 2, 3] = np.nan

    def run(with_bad):
        out = {}
        with P.Server(1 << 40, 4) as srv:
            bid = srv.submit(pbs[0]["spec"], bad, pbs[0]["chat"], 3) if with_bad else None
            ids = [srv.submit(pb["spec"], pb["state"], pb["chat"], 3) for pb in pbs[1:]]
            if with_bad:
                info = srv.wait(bid, 60.0)
                assert info["status"] == "failed" and info["error"] == P.RHD_ENONFINITE
                _, _, code = srv.fetch(bid)
                assert code == P.RHD_ENONFINITE
            for i, rid in enumerate(ids):
                assert srv.wait(rid, 60.0)["status"] == "done"
                out[i], diag, code = srv.fetch(rid)
                assert code == P.RHD_OK and diag["nonfinite"] == 0
            st = srv.stats()
            assert st["failed"] == (1 if with_bad else 0) and st["completed"] == 2
        return out

    ref, got = run(False), run(True)
    for i in ref:
        for k in ri.FIELDS:
            assert np.array_equal(ref[i][k], got[i][k]), (i, k)


def test_destroying_a_busy_server_returns():
    announce("server destroy while busy")
    pb = ri.c5_problem(stream(1, seed=12, sizes=(24,))[0])
    srv = P.Server(1 << 40, 2)
    rid = srv.submit(pb["spec"], pb["state"], pb["chat"], 1_000_000)
    srv.submit(pb["spec"], pb["state"], pb["chat"], 1_000_000)
    wait_until(lambda: srv.poll(rid)["steps_done"] >= 1)
    t = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t < 30.0
