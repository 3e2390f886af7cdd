"""Autotuner of a context's launch shapes.

The knobs (``Context.tune``) change only how work is cut into work-groups:
the number of BConv targets each work-group of the fused BConv + NTT column
pass accumulates (ModUp and ModDown separately: more targets reuse each
loaded input more, fewer give more work-groups), the column-tile order
across the 8 XCDs, how many residues each thread of the stand-alone NTT
row passes holds (16 with one LDS exchange, or 4 with one wave per row and
three exchanges: four times the waves to hide memory latency), and the
column-pass tile (8, 16 or 32 columns: a quarter, half or whole 128-byte
row; narrower tiles give more work-groups); the residues each KeyMult thread holds (16, or 4 with one wave per row and
64-bit digit sums), and the residues each thread of key switching's column
passes holds (16 with one LDS exchange, or 4 with radix-4 rounds); the
row-pass, KeyMult and column-pass widths of single-operation launches are
tuned apart, on the single operation alone.  Results are
bit-identical for every setting, so the tuner only times: each candidate
runs the workloads below on uniformly random residues, and the fastest
total wins.  The winner is cached in a JSON
file keyed by device name and parameter set, and reused without timing.

Workloads: one HMult + relinearisation + rescale at the top level (the
latency of a single operation) and one batched call of `batch` pairs at
levels spread evenly over [2, L] (throughput).  A retune rebuilds the launch
plans, so graphs captured before it must be captured again.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import OP_HMULT

KNOBS = ("bconv_tpw_up", "bconv_tpw_down", "xcd_pair", "rows_per_thread", "col_threads", "rows_per_thread_single",
         "keymult_rows", "keymult_rows_single", "cols_per_thread", "cols_per_thread_single")
# 512-thread column tiles cover whole 128-byte rows, so the XCD grouping of
# the tiles of one line does not apply to them; the 4-residue column passes
# have tiles of their own (col_threads does not apply to them)
CANDIDATES = [{"bconv_tpw_up": u, "bconv_tpw_down": d, "xcd_pair": x, "rows_per_thread": e, "col_threads": ct,
               "rows_per_thread_single": 0, "keymult_rows": km, "keymult_rows_single": 0, "cols_per_thread": cw,
               "cols_per_thread_single": 0}
              for u in (1, 2, 4) for d in (1, 2, 4) for e in (16, 4) for cw in (16, 4)
              for ct in ((128, 256, 512) if cw == 16 else (256,))
              for x in ((1, 0) if ct != 512 else (1,)) for km in (16, 4)]


def default_cache() -> str:
    return os.environ.get("CKKS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ckks_hip",
                                                             "tuning.json")


def cache_key(ctx, device_name: str) -> str:
    h = hashlib.sha256(json.dumps([list(map(int, ctx.q)), list(map(int, ctx.p))]).encode()).hexdigest()[:12]
    return "%s|logn=%d|nq=%d|np=%d|%s" % (device_name, ctx.log_n, ctx.n_q, len(ctx.p), h)


def _random_residues(torch, mods, lead, n, gen):
    m = torch.tensor([int(q) for q in mods], dtype=torch.int64, device="cuda").view(len(mods), 1)
    x = torch.randint(0, 1 << 62, (*lead, len(mods), n), generator=gen, device="cuda", dtype=torch.int64)
    return (x % m).to(torch.int32)


def autotune(ctx, batch: int = 16, reps: int = 10, cache: str | None = None, force: bool = False,
             candidates=None) -> dict:
    """Pick the fastest knob setting for `ctx` (cached); leaves it applied.
    Returns {"tuning", "source": "cache" | "timed", "table": [...]}"""
    import torch
    cache = cache or default_cache()
    key = cache_key(ctx, torch.cuda.get_device_name())
    db = {}
    if os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if not force and key in db:
        ctx.tune(**db[key]["tuning"])
        return {"tuning": db[key]["tuning"], "source": "cache", "table": db[key].get("table", [])}

    L, n = ctx.n_q, ctx.n
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2407)
    a = _random_residues(torch, ctx.q, (batch, 2), n, gen)
    b = _random_residues(torch, ctx.q, (batch, 2), n, gen)
    rlk = _random_residues(torch, list(ctx.q) + list(ctx.p), (ctx.dnum, 2), n, gen)
    levels = [2 + (i * (L - 2)) // max(1, batch - 1) for i in range(batch)] if L >= 2 else []
    out1 = torch.empty((2, max(1, L - 1), n), dtype=torch.int32, device="cuda")
    outb = torch.empty((batch, 2, max(1, L - 1), n), dtype=torch.int32, device="cuda")
    ws1 = torch.empty(ctx.workspace_size(OP_HMULT, L), dtype=torch.uint8, device="cuda")
    wsb = torch.empty(batch * ctx.workspace_size(OP_HMULT, L), dtype=torch.uint8, device="cuda")
    items = ctx.batch_items(levels) if levels else None

    def run():
        ctx.hmult_rescale(a[0], b[0], rlk, L, out1, ws=ws1)
        if items is not None:
            ctx.hmult_rescale_batch(a, b, items, L, rlk, outb, ws=wsb)

    table = []
    for cand in (candidates or CANDIDATES):
        ctx.tune(**cand)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        table.append({**cand, "us": 1e6 * (time.perf_counter() - t0) / reps})
    best = min(table, key=lambda r: r["us"])
    tuning = {k: best[k] for k in KNOBS}
    # then the row-pass and KeyMult widths of single-operation launches
    # alone, timed on the single operation (a lone HMult has few waves; a
    # batch has many)
    single = []
    for e in (16, 4):
        for km in (16, 4):
            for cw in (16, 4):
                ctx.tune(**{**tuning, "rows_per_thread_single": e, "keymult_rows_single": km,
                            "cols_per_thread_single": cw})
                ctx.hmult_rescale(a[0], b[0], rlk, L, out1, ws=ws1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(4 * reps):
                    ctx.hmult_rescale(a[0], b[0], rlk, L, out1, ws=ws1)
                torch.cuda.synchronize()
                single.append((1e6 * (time.perf_counter() - t0) / (4 * reps), e, km, cw))
                table.append({**tuning, "rows_per_thread_single": e, "keymult_rows_single": km,
                              "cols_per_thread_single": cw, "us_single": single[-1][0]})
    _, tuning["rows_per_thread_single"], tuning["keymult_rows_single"], tuning["cols_per_thread_single"] = min(single)
    ctx.tune(**tuning)
    db[key] = {"tuning": tuning, "table": table, "workload": "hmult_rescale level %d + batch of %d" % (L, batch)}
    os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    tmp = cache + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, cache)
    return {"tuning": tuning, "source": "timed", "table": table}
