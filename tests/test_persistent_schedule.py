"""CPU replay of the persistent batch launch's scheduling (k_rad_batch_persistent in
paper_1306_0010_amd/csrc/rhd_tile.hpp, its plan built in rhd.hip): the host's packed
tile lists, level table and grid size, and the device's ticket claims, level lookup and
per-member wait condition, mirrored in integers. A random interleaving of the blocks is
simulated to the end: no wait can block forever, every tile a block reads lies inside
its list, and a tile of member k at level l starts only once every tile of member k at
the levels below has finished (so the half-step and state arrays are complete)."""
import bisect
import random

import pytest

BX = 64


def balanced_chunk(L, zc):
    chunks = (L + zc - 1) // zc
    return (L + chunks - 1) // chunks


def tile_grid(n, BY, zc):
    """Tile counts (predictor, corrector) of one member, as rhdk::tile_grid."""
    ntx = (n[0] + BX - 1) // BX
    zp, zq = balanced_chunk(n[2] + 4, zc), balanced_chunk(n[2], zc)
    pred = (ntx + 1, (n[1] + 4 + BY - 1) // BY, (n[2] + 4 + zp - 1) // zp)
    corr = (ntx, (n[1] + BY - 1) // BY, (n[2] + zq - 1) // zq)
    return pred[0] * pred[1] * pred[2], corr[0] * corr[1] * corr[2]


def host_plan(members, BY, zc, resident):
    """members: list of (grid n, nsub). Mirrors batch_step_impl's sort, lists, round
    counts and the persistent launch's level table and grid."""
    order = sorted(range(len(members)), key=lambda i: -members[i][1])  # stable, by nsub desc
    tiles = [[], []]
    tp, tc, pred_end, corr_end = [], [], [], []
    for k, i in enumerate(order):
        p, c = tile_grid(members[i][0], BY, zc)
        tp.append(p)
        tc.append(c)
        tiles[0] += [k] * p
        tiles[1] += [k] * c
        pred_end.append(len(tiles[0]))
        corr_end.append(len(tiles[1]))
    nsub = [members[i][1] for i in order]
    rounds = nsub[0]
    counts = []
    for r in range(rounds):
        k = sum(1 for q in nsub if q > r)
        counts += [pred_end[k - 1], corr_end[k - 1]]
    start, acc = [], 0
    for cnt in counts:
        start.append(acc)
        acc += cnt
    start.append(acc)
    widest = max(counts)
    grid = max(1, min(acc, resident, 2 * widest))
    return dict(tiles=tiles, tp=tp, tc=tc, nsub=nsub, start=start, levels=2 * rounds,
                total=acc, grid=grid)


def plan_level(start, levels, t):
    lo, hi = 0, levels - 1
    while lo < hi:
        mid = (lo + hi + 1) >> 1
        if start[mid] <= t:
            lo = mid
        else:
            hi = mid - 1
    return lo


def simulate(plan, seed):
    rng = random.Random(seed)
    total, levels, start = plan["total"], plan["levels"], plan["start"]
    done = [0] * len(plan["tp"])
    finished_at = {}  # (member, level) -> finished tiles
    ticket = 0
    blocks = [{"state": "idle"} for _ in range(plan["grid"])]
    live = len(blocks)
    steps = 0
    while live:
        steps += 1
        assert steps < 50 * total * len(blocks) + 1000, "no progress: a wait never ends"
        b = rng.choice([q for q in blocks if q["state"] != "exit"])
        if b["state"] == "idle":
            t = ticket
            ticket += 1
            if t >= total:
                b["state"] = "exit"
                live -= 1
                continue
            l = plan_level(start, levels, t)
            assert start[l] <= t < start[l + 1]
            o = t - start[l]
            assert 0 <= o < len(plan["tiles"][l & 1])
            k = plan["tiles"][l & 1][o]
            need = (l >> 1) * (plan["tp"][k] + plan["tc"][k]) + (plan["tp"][k] if l & 1 else 0)
            b.update(state="wait", k=k, l=l, need=need)
        elif b["state"] == "wait":
            if done[b["k"]] >= b["need"]:
                k, l = b["k"], b["l"]
                for lo in range(l):  # every tile of member k below this level has finished
                    cnt = plan["tp"][k] if lo % 2 == 0 else plan["tc"][k]
                    assert finished_at.get((k, lo), 0) == cnt, (k, l, lo)
                b["state"] = "run"
        else:  # run -> finished
            done[b["k"]] += 1
            finished_at[(b["k"], b["l"])] = finished_at.get((b["k"], b["l"]), 0) + 1
            b["state"] = "idle"
    for k, ns in enumerate(plan["nsub"]):
        assert done[k] == ns * (plan["tp"][k] + plan["tc"][k])
    return steps


MIXES = [
    [((40, 24, 20), 7), ((33, 48, 17), 20), ((64, 20, 30), 38)],
    [((16, 16, 16), 5), ((24, 17, 40), 45), ((40, 24, 20), 7), ((33, 48, 17), 20),
     ((64, 20, 30), 38)],
    [((192, 32, 48), 3), ((32, 32, 32), 50), ((130, 70, 9), 1)],
    [((64, 64, 64), 12)],
]


@pytest.mark.parametrize("mix", range(len(MIXES)))
@pytest.mark.parametrize("BY,zc,resident", [(8, 16, 512), (8, 8, 7), (4, 8, 1), (16, 16, 3)])
def test_persistent_schedule_replay(mix, BY, zc, resident):
    plan = host_plan(MIXES[mix], BY, zc, resident)
    assert plan["grid"] >= 1 and all(plan["start"][l] < plan["start"][l + 1]
                                     for l in range(plan["levels"]))
    for seed in range(3):
        simulate(plan, seed)
