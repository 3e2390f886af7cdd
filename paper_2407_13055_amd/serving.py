"""Continuous-batching request loop for HMult / HRot on one GPU.

Requests name a ring degree N, an operation (HMult, with rescale when the
level allows it, or HRot by a slot offset), a level and an input slot of a
ciphertext pool that stays resident in HBM, beside the relinearisation and
rotation keys.  The loop

* releases each request at its arrival time into a queue per
  (N, operation) group;
* whenever a stream lane has room, takes the group whose oldest request has
  waited longest and launches up to ``max_batch`` of its requests as ONE
  batched library call (every item at its own level);
* admits a batch only if its output and workspace bytes fit in the free
  part of a byte budget (first-fit arena over one device allocation);
  requests wait, in order, until completions free memory;
* polls completion events, frees the workspace at once and the outputs when
  the consumer has released them, and records per-request latency from
  arrival to the result-ready event.

Batches on different lanes run concurrently on the device, and requests that
arrive while others run join the next batch of their group: no batch waits
for a full set.  The arithmetic is the library's batched calls, which are
bit-identical per item to the single-operation calls, so a result does not
depend on the mix it ran in.

The scheduler is independent of the device: ``GpuExecutor`` launches the
library's batched calls on torch streams, ``SimExecutor`` models durations
on a simulated clock (host tests of the scheduling logic).
"""
from __future__ import annotations

import bisect
import gc
import heapq
import math
import time
from collections import deque
from dataclasses import dataclass, field

ALIGN = 256

HMULT, HROT = "hmult", "hrot"
# batch kinds: HMult + relin + rescale (level >= 2), HMult + relin (level 1), HRot
K_HMULT_RS, K_HMULT, K_HROT = "hmult_rescale", "hmult", "hrot"


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    log_n: int
    op: str                 # HMULT or HROT
    level: int
    src: int                # input slot of the resident pool
    rot: int = 0            # slot offset (HRot)
    key: int = 0            # index of the rotation key for `rot` (HRot)
    # filled in by the server
    launched: float = math.nan
    ready: float = math.nan
    batch: int = -1
    slot: int = -1
    rejected: bool = False

    @property
    def kind(self) -> str:
        if self.op == HROT:
            return K_HROT
        return K_HMULT_RS if self.level >= 2 else K_HMULT

    @property
    def group(self) -> tuple:
        return (self.log_n, self.kind)

    @property
    def out_level(self) -> int:
        return self.level - 1 if self.kind == K_HMULT_RS else self.level


def poisson_requests(seed: int, rate: float, duration: float, log_ns, n_q: dict, offsets, n_src: int,
                     p_hmult: float = 0.7) -> list:
    """Poisson arrivals at `rate` per second over [0, duration): each request
    is HMult with probability p_hmult (else HRot by an offset drawn uniformly
    from `offsets`, key index = its position there), N = 2^log_n with log_n
    uniform over `log_ns`, level uniform in [1, n_q[log_n]], input slot
    uniform in [0, n_src)."""
    import numpy as np

    import synth
    est = int(rate * duration * 1.3) + 64
    while True:
        gaps = -np.log(synth.stream(seed, "arrivals").unit(est)) / rate
        t = np.cumsum(gaps)
        if t[-1] >= duration:
            break
        est *= 2
    n = int(np.searchsorted(t, duration))
    t = t[:n]
    u_op = synth.stream(seed, "serving/op").unit(n)
    i_n = synth.stream(seed, "serving/n").integers(0, len(log_ns) - 1, n)
    u_lv = synth.stream(seed, "serving/level").unit(n)
    src = synth.stream(seed, "serving/src").integers(0, n_src - 1, n)
    i_rot = synth.stream(seed, "serving/rot").integers(0, len(offsets) - 1, n)
    out = []
    for i in range(n):
        ln = int(log_ns[int(i_n[i])])
        top = n_q[ln]
        level = min(top, 1 + int((1.0 - u_lv[i]) * top))  # u in (0, 1] -> level uniform in [1, top]
        hm = u_op[i] <= p_hmult
        k = int(i_rot[i])
        out.append(Request(i, float(t[i]), ln, HMULT if hm else HROT, level, int(src[i]),
                           0 if hm else int(offsets[k]), 0 if hm else k))
    return out


class Arena:
    """First-fit allocator of ALIGN-aligned byte ranges in [0, capacity);
    freed ranges merge with free neighbours."""

    def __init__(self, capacity: int):
        self.capacity = capacity - capacity % ALIGN
        self.free_offs = [0]                 # sorted starts of free ranges
        self.free_size = {0: self.capacity}  # start -> size
        self.used_size = {}                  # start -> size of live allocations
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        need = max(ALIGN, -(-nbytes // ALIGN) * ALIGN)
        for off in self.free_offs:
            size = self.free_size[off]
            if size >= need:
                i = bisect.bisect_left(self.free_offs, off)
                del self.free_offs[i]
                del self.free_size[off]
                if size > need:
                    bisect.insort(self.free_offs, off + need)
                    self.free_size[off + need] = size - need
                self.used_size[off] = need
                self.used += need
                self.peak = max(self.peak, self.used)
                return off
        return None

    def free(self, off: int) -> None:
        size = self.used_size.pop(off)
        self.used -= size
        i = bisect.bisect_left(self.free_offs, off)
        if i < len(self.free_offs) and self.free_offs[i] == off + size:  # merge with the next range
            size += self.free_size.pop(off + size)
            del self.free_offs[i]
        if i > 0:
            prev = self.free_offs[i - 1]
            if prev + self.free_size[prev] == off:  # merge with the previous range
                self.free_size[prev] += size
                return
        self.free_offs.insert(i, off)
        self.free_size[off] = size

    def largest_free(self) -> int:
        return max(self.free_size.values(), default=0)


@dataclass
class Batch:
    bid: int
    group: tuple
    reqs: list
    lane: int
    off_out: int
    off_ws: int
    handle: object = None
    launched: float = 0.0
    ready: float = math.nan
    live: int = 0           # requests whose outputs are still held


@dataclass
class Report:
    requests: list
    batches: int
    batch_sizes: list = field(default_factory=list)
    peak_bytes: int = 0
    budget: int = 0
    wall: float = 0.0
    max_inflight: int = 0
    blocked_polls: int = 0

    def summary(self, warmup: float = 0.0) -> dict:
        done = [r for r in self.requests if not r.rejected and r.arrival >= warmup and not math.isnan(r.ready)]
        lat = sorted(r.ready - r.arrival for r in done)
        if not lat:
            return {"completed": 0}
        wait = sorted(r.launched - r.arrival for r in done)
        span = max(r.ready for r in done) - min(r.arrival for r in done)

        def pct(p):
            return lat[min(len(lat) - 1, int(p / 100.0 * len(lat)))]
        return {"completed": len(done), "rejected": sum(r.rejected for r in self.requests),
                "ops_per_s": len(done) / span if span > 0 else float("nan"),
                "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "max_ms": 1e3 * lat[-1],
                "p50_wait_ms": 1e3 * wait[len(wait) // 2], "p99_wait_ms": 1e3 * wait[min(len(wait) - 1, int(0.99 * len(wait)))],
                "mean_batch": sum(self.batch_sizes) / max(1, len(self.batch_sizes)), "batches": self.batches,
                "max_inflight_batches": self.max_inflight, "peak_bytes": self.peak_bytes, "budget": self.budget}


class Server:
    """The request loop.  `executor` provides lanes, footprints, launches and
    completion times; `hold` is how long a consumer keeps a result before its
    memory is released (0: at once); `on_ready(req, batch)` runs when a
    request's result is ready, before its memory can be released."""

    def __init__(self, executor, budget: int, max_batch: int = 16, hold: float = 0.0, on_ready=None,
                 linger: float = 0.0):
        self.ex = executor
        self.arena = Arena(budget)
        self.max_batch = max_batch
        self.hold = hold
        self.on_ready = on_ready
        # while other batches run, a group waits up to `linger` seconds for a
        # full batch (larger batches under load); an idle device launches at once
        self.linger = linger

    def _try_launch(self, group, queue, lane, now, bid):
        """Launch up to max_batch requests of `queue` on `lane` if memory allows;
        return the batch, or None when even one request does not fit now."""
        k = min(self.max_batch, len(queue))
        while k >= 1:
            reqs = [queue[i] for i in range(k)]
            out_b, ws_b = self.ex.footprint(group, reqs)
            off_out = self.arena.alloc(out_b)
            if off_out is not None:
                off_ws = self.arena.alloc(ws_b)
                if off_ws is not None:
                    for _ in range(k):
                        queue.popleft()
                    b = Batch(bid, group, reqs, lane, off_out, off_ws, launched=now, live=k)
                    for i, r in enumerate(reqs):
                        r.launched, r.batch, r.slot = now, bid, i
                    b.handle = self.ex.launch(group, reqs, off_out, off_ws, lane)
                    return b
                self.arena.free(off_out)
            k //= 2
        return None

    def run(self, requests, clock) -> Report:
        # the loop allocates little, but a full collection over the request
        # objects stalls it for tens of milliseconds: collect before, not during
        gc.collect()
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, clock)
        finally:
            if was_enabled:
                gc.enable()

    def _run(self, requests, clock) -> Report:
        reqs = sorted(requests, key=lambda r: r.arrival)
        queues = {}
        rep = Report(reqs, 0, budget=self.arena.capacity)
        inflight = []            # launched batches not yet complete
        releases = []            # heap (time, bid, batch) of held outputs
        lane_load = [0] * self.ex.lanes
        nxt, finished, bid = 0, 0, 0
        total = len(reqs)
        t_start = clock.now()
        while finished < total:
            now = clock.now()
            while nxt < total and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                out_b, ws_b = self.ex.footprint(r.group, [r])
                if -(-out_b // ALIGN) * ALIGN + -(-ws_b // ALIGN) * ALIGN > self.arena.capacity:
                    r.rejected = True  # can never fit the budget
                    finished += 1
                    continue
                queues.setdefault(r.group, deque()).append(r)
            progressed = False
            for b in list(inflight):
                t = self.ex.poll(b.handle)
                if t is None:
                    continue
                progressed = True
                inflight.remove(b)
                lane_load[b.lane] -= 1
                b.ready = t
                self.arena.free(b.off_ws)
                for r in b.reqs:
                    r.ready = t
                    if self.on_ready is not None:
                        self.on_ready(r, b)
                finished += len(b.reqs)
                self.ex.retire(b.handle)
                heapq.heappush(releases, (now + self.hold, b.bid, b))
            while releases and releases[0][0] <= now:
                _, _, b = heapq.heappop(releases)
                self.arena.free(b.off_out)
                progressed = True
            blocked = False
            while not blocked:
                lane = min(range(self.ex.lanes), key=lambda i: lane_load[i])
                if lane_load[lane] >= self.ex.depth:
                    break
                busy = bool(inflight)
                ready_groups = [(q[0].arrival, g) for g, q in queues.items()
                                if q and (not busy or len(q) >= self.max_batch or now - q[0].arrival >= self.linger)]
                if not ready_groups:
                    break
                _, g = min(ready_groups)
                b = self._try_launch(g, queues[g], lane, now, bid)
                if b is None:
                    blocked = True
                    rep.blocked_polls += 1
                    break
                bid += 1
                progressed = True
                inflight.append(b)
                lane_load[lane] += 1
                rep.batches += 1
                rep.batch_sizes.append(len(b.reqs))
                rep.max_inflight = max(rep.max_inflight, len(inflight))
            if not progressed and finished < total:
                nexts = []
                if nxt < total:
                    nexts.append(reqs[nxt].arrival)
                if releases:
                    nexts.append(releases[0][0])
                if self.linger > 0:
                    nexts.extend(t for t in (q[0].arrival + self.linger for q in queues.values() if q) if t > now)
                t_done = self.ex.next_completion()
                if t_done is not None:
                    nexts.append(t_done)
                clock.idle(min(nexts) if nexts else None)
        while releases:
            _, _, b = heapq.heappop(releases)
            self.arena.free(b.off_out)
        self.ex.finish()
        rep.peak_bytes = self.arena.peak
        rep.wall = clock.now() - t_start
        return rep


class RealClock:
    """Seconds since `start()`, host monotonic clock; idling spins."""

    def __init__(self):
        self.t0 = time.perf_counter()

    def start(self, t0: float) -> None:
        self.t0 = t0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def idle(self, until) -> None:
        pass


class SimClock:
    """Simulated time: idling jumps to the next event."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def idle(self, until) -> None:
        if until is None:
            raise RuntimeError("simulated run has nothing left to wait for")
        self.t = max(self.t, until)


class SimExecutor:
    """Device model for host tests: a batch on a lane starts when the lane's
    previous batch ends and lasts fixed + per_level * sum(levels) seconds
    (scaled by N / 2^16); footprints as the library's, with a stand-in
    workspace of `ws_limbs` limbs per item level."""

    def __init__(self, clock: SimClock, lanes: int = 2, depth: int = 1, fixed: float = 50e-6,
                 per_level: float = 4e-6, ws_limbs: int = 12):
        self.clock, self.lanes, self.depth = clock, lanes, depth
        self.fixed, self.per_level, self.ws_limbs = fixed, per_level, ws_limbs
        self.lane_free = [0.0] * lanes
        self.pending = {}   # handle -> end time
        self.launches = []  # (group, [rid], lane, start, end, off_out, off_ws, out_bytes, ws_bytes)
        self.seq = 0

    def footprint(self, group, reqs):
        log_n, kind = group
        top = max(r.level for r in reqs)
        out_level = top - 1 if kind == K_HMULT_RS else top
        limb = 4 << log_n
        return len(reqs) * 2 * out_level * limb, len(reqs) * self.ws_limbs * top * limb

    def launch(self, group, reqs, off_out, off_ws, lane):
        scale = 2.0 ** (group[0] - 16)
        start = max(self.clock.now(), self.lane_free[lane])
        end = start + scale * (self.fixed + self.per_level * sum(r.level for r in reqs))
        self.lane_free[lane] = end
        self.seq += 1
        self.pending[self.seq] = end
        ob, wb = self.footprint(group, reqs)
        self.launches.append((group, [r.rid for r in reqs], lane, start, end, off_out, off_ws, ob, wb))
        return self.seq

    def poll(self, h):
        end = self.pending[h]
        return end if end <= self.clock.now() else None

    def retire(self, h):
        del self.pending[h]

    def next_completion(self):
        return min(self.pending.values(), default=None)

    def finish(self):
        pass


class GpuExecutor:
    """Launches batches through the library on `lanes` torch streams (default
    priority), `depth` batches in flight per lane.  Outputs and workspaces
    are carved from one device allocation of `capacity` bytes; items go
    through pinned host buffers, one per lane slot, reused only after the
    batch that used them completed.  Completion times are the batches'
    events, placed on the host clock through an anchor event."""

    def __init__(self, ck, torch, ctxs: dict, pools: dict, keys: dict, capacity: int, lanes: int = 4,
                 depth: int = 2, max_batch: int = 16):
        self.ck, self.torch = ck, torch
        self.ctxs, self.pools, self.keys = ctxs, pools, keys
        self.lanes, self.depth, self.max_batch = lanes, depth, max_batch
        self.arena = torch.empty(capacity, dtype=torch.uint8, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.items_h = [[torch.zeros((max_batch, 4), dtype=torch.int32, pin_memory=True) for _ in range(depth)]
                        for _ in range(lanes)]
        self.items_d = [[torch.zeros((max_batch, 4), dtype=torch.int32, device="cuda") for _ in range(depth)]
                        for _ in range(lanes)]
        self.slot_busy = [[False] * depth for _ in range(lanes)]
        self.anchor = None
        self.clock = None
        self.finished = []
        self.n_launch = 0

    def start(self, clock: RealClock) -> None:
        """Anchor device time to the host clock (call right before the run):
        every lane runs a marker first, so the anchor is not delayed by a
        stream's first use."""
        torch = self.torch
        for s in self.streams:
            torch.cuda.Event().record(s)
        torch.cuda.synchronize()
        self.clock = clock
        self.anchor = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        self.anchor.record(self.streams[0])
        torch.cuda.synchronize()
        self.anchor_uncertainty = time.perf_counter() - t0
        clock.start(t0)
        self.finished = []

    def finish(self) -> None:
        """Place every completion on the host clock: device event times are
        mapped linearly through the start anchor and an end anchor (the two
        clocks run at slightly different rates), and kept within [launch,
        the host time the loop saw the completion]."""
        torch = self.torch
        torch.cuda.synchronize()
        end = torch.cuda.Event(enable_timing=True)
        t_end = self.clock.now()
        end.record(self.streams[0])
        torch.cuda.synchronize()
        g_end = self.anchor.elapsed_time(end) / 1e3
        scale = t_end / g_end if g_end > 0 else 1.0
        for reqs, ev in self.finished:
            t = self.anchor.elapsed_time(ev) / 1e3 * scale
            for r in reqs:
                r.ready = min(r.ready, max(r.launched, t))
        self.clock_scale = scale

    def out_level_of(self, kind, top):
        return top - 1 if kind == K_HMULT_RS else top

    def footprint(self, group, reqs):
        log_n, kind = group
        C = self.ctxs[log_n]
        top = max(r.level for r in reqs)
        op = self.ck.OP_HROT if kind == K_HROT else self.ck.OP_HMULT
        out_b = len(reqs) * 2 * self.out_level_of(kind, top) * (4 << log_n)
        return out_b, len(reqs) * C.workspace_size(op, top)

    def view(self, off, nbytes):
        return self.arena[off:off + nbytes]

    def out_tensor(self, b):
        """Output slots of a batch: [n][2][out_level(max level)][N] int32."""
        log_n, kind = b.group
        top = max(r.level for r in b.reqs)
        ol = self.out_level_of(kind, top)
        n = len(b.reqs)
        return self.view(b.off_out, n * 2 * ol * (4 << log_n)).view(self.torch.int32).view(n, 2, ol, 1 << log_n)

    def result(self, b, i):
        """Item i's result [2][out_level_i][N] (a view into the arena)."""
        r = b.reqs[i]
        return self.out_tensor(b)[i, :, :r.out_level]

    def launch(self, group, reqs, off_out, off_ws, lane):
        torch = self.torch
        log_n, kind = group
        C = self.ctxs[log_n]
        slot = self.slot_busy[lane].index(False)
        self.slot_busy[lane][slot] = True
        n = len(reqs)
        h = self.items_h[lane][slot]
        hv = h.numpy()
        for i, r in enumerate(reqs):
            hv[i, 0], hv[i, 1], hv[i, 2], hv[i, 3] = r.level, r.key, r.rot, r.src
        s = self.streams[lane]
        d = self.items_d[lane][slot]
        top = max(r.level for r in reqs)
        ol = self.out_level_of(kind, top)
        out_b, ws_b = self.footprint(group, reqs)
        out = self.view(off_out, out_b).view(torch.int32).view(n, 2, ol, 1 << log_n)
        ws = self.view(off_ws, ws_b)
        with torch.cuda.stream(s):
            d[:n].copy_(h[:n], non_blocking=True)
        A, B = self.pools[log_n]
        rlk, rks = self.keys[log_n]
        if kind == K_HROT:
            C.hrot_batch(A, d[:n], top, rks, out, ws=ws, stream=s)
        elif kind == K_HMULT_RS:
            C.hmult_rescale_batch(A, B, d[:n], top, rlk, out, ws=ws, stream=s)
        else:
            C.hmult_batch(A, B, d[:n], top, rlk, out, ws=ws, stream=s)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        self.n_launch += 1
        return (lane, slot, ev, reqs)

    def poll(self, h):
        """Host time at which the loop sees the batch complete (refined by finish())."""
        lane, slot, ev, reqs = h
        if not ev.query():
            return None
        self.finished.append((reqs, ev))
        return self.clock.now()

    def retire(self, h):
        lane, slot, _, _ = h
        self.slot_busy[lane][slot] = False

    def next_completion(self):
        return None
