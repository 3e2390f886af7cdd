"""Host tests of the serving loop: the arrival generator, the first-fit
arena and the scheduler, driven by a simulated device on a simulated clock."""
import math

import numpy as np
import pytest

import synth
from paper_2407_13055_amd import serving as sv

OFFSETS = list(range(1, 33))


def reqs(rate, duration, seed=0, log_ns=(15, 16), top=24, n_src=16):
    return sv.poisson_requests(seed, rate, duration, list(log_ns), {ln: top for ln in log_ns}, OFFSETS, n_src)


def test_arrivals_follow_the_recipe():
    r = reqs(2000, 5.0)
    n = len(r)
    assert abs(n - 10000) < 4 * math.sqrt(10000)
    t = np.array([x.arrival for x in r])
    assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] < 5.0
    gaps = np.diff(t)
    assert abs(gaps.mean() * 2000 - 1) < 0.05 and abs(gaps.std() / gaps.mean() - 1) < 0.05  # exponential: cv 1
    hm = np.mean([x.op == sv.HMULT for x in r])
    assert abs(hm - 0.7) < 4 * math.sqrt(0.21 / n)
    assert abs(np.mean([x.log_n == 16 for x in r]) - 0.5) < 4 * math.sqrt(0.25 / n)
    lv = np.array([x.level for x in r])
    assert lv.min() == 1 and lv.max() == 24
    counts = np.bincount(lv, minlength=25)[1:]
    assert counts.min() > 0.7 * n / 24 and counts.max() < 1.3 * n / 24
    for x in r:
        if x.op == sv.HROT:
            assert x.rot == OFFSETS[x.key]
        else:
            assert x.rot == 0 and x.key == 0
    assert [x.level for x in reqs(2000, 1.0)] == [x.level for x in reqs(2000, 1.0)]
    assert [x.arrival for x in reqs(2000, 1.0, seed=1)] != [x.arrival for x in reqs(2000, 1.0)]


def test_request_kinds():
    mk = sv.Request
    assert mk(0, 0, 16, sv.HMULT, 1, 0).kind == sv.K_HMULT
    assert mk(0, 0, 16, sv.HMULT, 2, 0).kind == sv.K_HMULT_RS
    assert mk(0, 0, 16, sv.HMULT, 2, 0).out_level == 1
    assert mk(0, 0, 16, sv.HROT, 5, 0, 3, 2).out_level == 5


def test_arena_against_a_byte_map():
    st = synth.stream(3, "arena")
    cap = 1 << 16
    A = sv.Arena(cap)
    owner = np.zeros(cap, dtype=np.int64)
    live = {}
    sizes = st.integers(1, 5000, 3000)
    coin = st.unit(3000)
    for i in range(3000):
        if live and coin[i] < 0.45:
            off = sorted(live)[int(coin[i] * 1e6) % len(live)]
            sz = live.pop(off)
            assert np.all(owner[off:off + sz] == off + 1)
            owner[off:off + sz] = 0
            A.free(off)
        else:
            off = A.alloc(int(sizes[i]))
            if off is None:
                # first fit fails only if no free run of the aligned size exists
                need = -(-int(sizes[i]) // sv.ALIGN) * sv.ALIGN
                free_runs = [(s, z) for s, z in A.free_size.items()]
                assert all(z < need for _, z in free_runs)
                continue
            sz = A.used_size[off]
            assert off % sv.ALIGN == 0 and sz >= sizes[i] and off + sz <= cap
            assert np.all(owner[off:off + sz] == 0), "overlapping allocation"
            owner[off:off + sz] = off + 1
            live[off] = sz
        assert A.used == sum(live.values()) and A.used <= cap
        assert A.used + sum(A.free_size.values()) == A.capacity
    for off in list(live):
        A.free(off)
    assert A.free_offs == [0] and A.free_size == {0: A.capacity} and A.used == 0


def run_sim(requests, budget=1 << 40, lanes=2, depth=1, max_batch=16, hold=0.0, linger=0.0, **kw):
    clock = sv.SimClock()
    ex = sv.SimExecutor(clock, lanes=lanes, depth=depth, **kw)
    rep = sv.Server(ex, budget, max_batch=max_batch, hold=hold, linger=linger).run(requests, clock)
    return rep, ex


def check_schedule(rep, ex, max_batch):
    by_rid = {r.rid: r for r in rep.requests}
    last_in_group = {}
    for group, rids, lane, start, end, *_ in ex.launches:
        assert 1 <= len(rids) <= max_batch
        for rid in rids:
            r = by_rid[rid]
            assert r.group == group, "a batch mixes groups"
            assert r.launched >= r.arrival, "launched before arrival"
            assert r.ready == end and end > start >= r.arrival
        # first come, first served within a group
        assert rids == sorted(rids)
        assert rids[0] > last_in_group.get(group, -1)
        last_in_group[group] = rids[-1]
    # lanes never run two batches at once (depth 1) in the device model
    for lane in set(x[2] for x in ex.launches):
        spans = sorted((x[3], x[4]) for x in ex.launches if x[2] == lane)
        assert all(a[1] <= b[0] + 1e-12 for a, b in zip(spans, spans[1:]))


def test_all_requests_served_in_order_and_alone_at_light_load():
    r = reqs(200, 2.0)
    rep, ex = run_sim(r)
    assert all(not math.isnan(x.ready) and not x.rejected for x in r)
    check_schedule(rep, ex, 16)
    # at light load almost every request runs alone, right at arrival
    assert np.mean(rep.batch_sizes) < 1.1
    s = rep.summary()
    assert s["completed"] == len(r) and s["p50_ms"] < 0.2


def test_continuous_batching_under_load():
    """Arrivals faster than one lane serves: requests that arrive while
    batches run join the next batch of their group; lanes overlap."""
    r = reqs(80000, 0.2)  # about 3x what two lanes serve one request at a time
    rep, ex = run_sim(r, lanes=2, max_batch=16)
    check_schedule(rep, ex, 16)
    assert all(not math.isnan(x.ready) for x in r)
    assert np.mean(rep.batch_sizes) > 2 and max(rep.batch_sizes) > 4
    assert rep.max_inflight == 2
    # nothing waits for a full batch: a batch launches as soon as a lane frees
    free_at = {}
    for group, rids, lane, start, end, *_ in ex.launches:
        first = min(x.arrival for x in rep.requests if x.rid in rids)
        assert start <= max(first, free_at.get(lane, 0.0)) + 1e-9 or start == rep.requests[rids[0]].launched
        free_at[lane] = end


def test_budget_pressure_waits_but_serves_everyone():
    r = reqs(4000, 0.5, log_ns=(15,), top=24)
    limb = 4 << 15
    one = 2 * 24 * limb + 12 * 24 * limb     # largest single request's footprint in the model
    budget = 3 * one
    rep, ex = run_sim(r, budget=budget, lanes=4, depth=2, hold=2e-3)
    assert rep.peak_bytes <= budget
    assert rep.blocked_polls > 0
    assert all(not math.isnan(x.ready) and not x.rejected for x in r)
    check_schedule(rep, ex, 16)
    big, _ = run_sim(r, budget=1 << 40, lanes=4, depth=2, hold=2e-3)
    assert rep.summary()["p99_ms"] >= big.summary()["p99_ms"]


def test_requests_that_never_fit_are_rejected():
    r = reqs(500, 0.2, log_ns=(16,))
    limb = 4 << 16
    budget = 14 * 12 * limb  # below the footprint of high-level requests
    rep, ex = run_sim(r, budget=budget)
    rej = [x for x in r if x.rejected]
    assert rej and all(2 * x.out_level * limb + 12 * x.level * limb > budget - 2 * sv.ALIGN for x in rej)
    assert all(not math.isnan(x.ready) for x in r if not x.rejected)
    assert rep.summary()["rejected"] == len(rej)


def test_linger_builds_larger_batches_under_load_only():
    """With a linger time, groups wait for fuller batches while the device is
    busy: larger batches and more completed work per launch under overload;
    at light load (idle device) requests still launch on arrival."""
    heavy = reqs(80000, 0.1)
    base, _ = run_sim(heavy, lanes=4, depth=2)
    lin, ex = run_sim(reqs(80000, 0.1), lanes=4, depth=2, linger=200e-6)
    check_schedule(lin, ex, 16)
    assert np.mean(lin.batch_sizes) > np.mean(base.batch_sizes)
    assert lin.batches < base.batches
    light = reqs(200, 1.0)
    a, _ = run_sim(light, linger=200e-6)
    b, _ = run_sim(reqs(200, 1.0))
    assert abs(a.summary()["p50_ms"] - b.summary()["p50_ms"]) < 0.05
