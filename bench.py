#!/usr/bin/env python3
"""Benchmark of the key-switching hot path on one MI355X.

Workload (headline): HMult with relinearisation followed by rescale on one
ciphertext pair per operation, N = 2^16, 24 ciphertext primes of 30 bits,
8 special primes of 31 bits (digit width 8, dnum 3), uniformly random
residues (every kernel is data-independent).  Each step is one such
operation on the next of 16 distinct ciphertext pairs (384 MiB, more than
the 256 MB last-level cache), with one resident relinearisation key.

Prints one compact JSON line last on stdout: throughput (ops/s), the
roofline of the dominant kernel (the operation's algorithmic bytes over that
kernel's average duration, timed live with HIP events), the whole-operation
HBM and ALU fractions, HMult-only and HRot timings, short summaries of the
batched, rotation and serving runs, and the CPU oracle timed single-threaded
and on all host threads.  The full record (per-kernel timings, the tuner's
table, serving runs, 25-30 prime system sections) goes to a details file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HMult+relin ops/s at N=2^16 L=24 (32-bit RNS), batched vs plain; % HBM BW"
LOG_N, N_Q, N_P = 16, 24, 8
LIMB = 4 << LOG_N  # bytes per limb
HBM_PEAK_GBS = 8000.0
N_PAIRS = 16


def alg_bytes_per_kernel(level: int, alpha: int, beta: int) -> dict:
    """Algorithmic HBM bytes per launch of each kernel of HMult+relin+rescale
    (every operand read once, every result written once), in limbs x LIMB."""
    up_rows = beta * (level + alpha) - level
    limbs = {
        "modup_intt_rows": 2 * level + level,              # a_a, a_b in; INTT rows out
        "modup_intt_cols": level + level,                  # in; lifted out
        "modup_bconv_ntt_cols": level + up_rows,           # lifted digits in; new ModUp rows out
        "keymult": up_rows + 2 * beta * (level + alpha) + 4 * level + 2 * level + 2 * alpha,
        "moddown_intt_cols": 2 * alpha + 2 * alpha,
        "moddown_bconv_ntt_cols": 2 * alpha + 2 * level,
        "moddown_ntt_rows_combine": 2 * level + 2 * level + 2 * level,
        "rescale_intt_rows": 2 + 2,
        "rescale_intt_cols": 2 + 2,
        "rescale_ntt_cols": 2 + 2 * (level - 1),
        "rescale_ntt_rows_combine": 3 * 2 * (level - 1),
    }
    return {k: v * LIMB for k, v in limbs.items()}


def op_alg_bytes(level: int, alpha: int, beta: int, rescale: bool) -> int:
    """Whole-operation algorithmic bytes: inputs 4l + evk rows 2 beta (l+alpha)
    + output 2l (2(l-1) after rescale) limbs."""
    out = 2 * (level - 1) if rescale else 2 * level
    return (4 * level + 2 * beta * (level + alpha) + out) * LIMB


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "ntt_core.h", "modarith.h"):
        h.update(open(os.path.join(ROOT, "paper_2407_13055_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# kernels of one HMult+relin+rescale in dispatch order (each pass in any of
# its widths), with the names the library's own timer gives them
HMULT_RS_SEQUENCE = ((("k_inv_rows<8, ckks::MapByPtr, ckks::LdOwn<(ckks::Own)0>",
                       "k_inv_rows4<8, ckks::MapByPtr, ckks::LdOwn<(ckks::Own)0>"), "modup_intt_rows"),
                     (("k_inv_cols<8", "k_inv_cols4<8"), "modup_intt_cols"),
                     (("k_bconv_ntt_cols<8", "k_bconv_ntt_cols4<8"), "modup_bconv_ntt_cols"),
                     (("k_keymult<8, (ckks::Own)0", "k_keymult4<8, (ckks::Own)0"), "keymult"),
                     (("k_inv_cols<8", "k_inv_cols4<8"), "moddown_intt_cols"),
                     (("k_bconv_ntt_cols<8", "k_bconv_ntt_cols4<8"), "moddown_bconv_ntt_cols"),
                     (("k_fwd_rows<8", "k_fwd_rows4<8"), "moddown_ntt_rows_combine"))
# issue rate of mixed integer VALU code on gfx950, in wave64 instructions
# per CU per cycle: a microbenchmark of radix-2 Shoup butterflies (3 32-bit
# multiplies, 5-6 adds, min) sustains 0.95-0.98 at full occupancy, 32-bit
# multiplies and 64-bit multiply-adds alone 0.97, plain 32-bit adds alone
# 1.77 (they pair up); the ALU floor takes 1.0
VALU_MIX_PEAK = 1.0
VALU_PEAK_WAVE_INSTR = 256 * 2.4e9 * VALU_MIX_PEAK


def _op_sequences(rows):
    """Start indices of complete HMult+rescale sequences in a dispatch list
    [(kernel name, ...)]."""
    n = len(HMULT_RS_SEQUENCE)
    return [i for i in range(len(rows) - n + 1)
            if all(any(sub in rows[i + k][0] for sub in alts) for k, (alts, _) in enumerate(HMULT_RS_SEQUENCE))]


def summarize_op(kt_dir: str, fetch_dir: str, write_dir: str, sq_dir: str, name: str, copy_bytes: int,
                 cmd: str) -> None:
    """Whole-operation profile of HMult+relin+rescale from four rocprofv3
    runs of the same command: --kernel-trace (durations), --pmc FETCH_SIZE,
    --pmc WRITE_SIZE (KiB per dispatch) and --pmc SQ_INSTS_VALU.  Every
    complete 7-kernel sequence is averaged per position.  The byte counters
    are scaled by what they read for a plain device copy of copy_bytes
    (random data) in the same runs."""
    import csv
    import glob

    def dispatches(d, counter=None):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv" if counter is None else
                                        "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if counter is None:
                    rows.append((r["Kernel_Name"], int(r["Dispatch_Id"]),
                                 (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
                elif r["Counter_Name"] == counter:
                    rows.append((r["Kernel_Name"], int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        rows.sort(key=lambda x: x[1])
        return rows

    def per_position(rows):
        idx = _op_sequences(rows)
        n = len(HMULT_RS_SEQUENCE)
        return [sum(rows[i + k][2] for i in idx) / max(1, len(idx)) for k in range(n)], len(idx), \
            [rows[idx[0] + k][0].split("(")[0].replace("void ", "") if idx else "?" for k in range(n)]

    def copy_scale(d, counter):
        v = [x for k, _, x in dispatches(d, counter) if "CUDAFunctorOnSelf_add" in k]
        v = [x for x in v if x > 0.25 * copy_bytes / 1024] or v
        return (copy_bytes / 1024) / (sorted(v)[len(v) // 2]) if v else float("nan"), len(v)

    dur, n_kt, names = per_position(dispatches(kt_dir))
    fetch, n_f, _ = per_position(dispatches(fetch_dir, "FETCH_SIZE"))
    write, n_w, _ = per_position(dispatches(write_dir, "WRITE_SIZE"))
    valu, n_v, _ = per_position(dispatches(sq_dir, "SQ_INSTS_VALU"))
    fs, nfc = copy_scale(fetch_dir, "FETCH_SIZE")
    wsc, nwc = copy_scale(write_dir, "WRITE_SIZE")
    kb = alg_bytes_per_kernel(N_Q, N_P, 3)
    path = os.path.join(ROOT, "profiles", "op_%s.txt" % name)
    tot = {"us": 0.0, "f": 0.0, "w": 0.0, "v": 0.0, "alg": 0.0}
    with open(path, "w") as f:
        f.write("# One HMult+relin+rescale at N=2^16, 24+8 primes, dnum 3: its 7 kernels in dispatch order\n")
        f.write("# command (four rocprofv3 runs: --kernel-trace; --pmc FETCH_SIZE; --pmc WRITE_SIZE; --pmc SQ_INSTS_VALU):\n")
        f.write("#   %s\n" % cmd)
        f.write("# sequences averaged: trace %d, fetch %d, write %d, valu %d; byte counters scaled by a %d-byte\n"
                "# random-data device copy in the same runs: fetch x%.4f (%d), write x%.4f (%d)\n"
                % (n_kt, n_f, n_w, n_v, copy_bytes, fs, nfc, wsc, nwc))
        f.write("# %-26s %8s %10s %10s %10s %11s %6s  %s\n" % ("kernel", "avg_us", "fetch_B", "write_B", "alg_B",
                                                             "valu_instr", "valu%", "instance"))
        lines = []
        for k, (_, label) in enumerate(HMULT_RS_SEQUENCE):
            fb, wb = fetch[k] * 1024 * fs, write[k] * 1024 * wsc
            util = 100 * valu[k] / (dur[k] * 1e-6) / VALU_PEAK_WAVE_INSTR if dur[k] else float("nan")
            f.write("#   %-26s %8.2f %10.0f %10.0f %10.0f %11.0f %6.1f  %s\n" % (label, dur[k], fb, wb,
                                                                             kb.get(label, 0), valu[k], util, names[k]))
            lines.append("kernel_%s: us=%.3f traffic_bytes=%.0f valu_instr=%.0f\n" % (label, dur[k], fb + wb, valu[k]))
            tot["us"] += dur[k]; tot["f"] += fb; tot["w"] += wb; tot["v"] += valu[k]; tot["alg"] += kb.get(label, 0)
        f.writelines(lines)
        f.write("kernels_us: %.2f\n" % tot["us"])
        f.write("traffic_bytes_per_op: %.0f\n" % (tot["f"] + tot["w"]))
        f.write("kernel_alg_bytes_per_op: %.0f\n" % tot["alg"])
        f.write("op_alg_bytes: %.0f\n" % op_alg_bytes(N_Q, N_P, 3, True))
        f.write("valu_wave_instr_per_op: %.0f\n" % tot["v"])
        f.write("alu_floor_us: %.2f\n" % (tot["v"] / VALU_PEAK_WAVE_INSTR * 1e6))
        f.write("source_sha256: %s\n" % source_hash())
    print(open(path).read())


def op_profile(name: str) -> dict:
    """Fields of profiles/op_NAME.txt, or {} when absent or taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", "op_%s.txt" % name)
    if not os.path.exists(path):
        return {}
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != source_hash():
        return {}
    return fields


def kernel_profile(prof: dict, kernel: str) -> dict:
    v = prof.get("kernel_" + kernel)
    return {k: float(x) for k, x in (kv.split("=") for kv in v.split())} if v else {}


def batched_vs_plain(C, ck, torch, synth, q, p, n_pairs: int, reps: int) -> dict:
    """64 pairs at levels drawn uniformly from [4, 24]: HMult+relin+rescale as
    n_pairs plain calls, and as one batched call captured in a hipGraph."""
    n, L, beta_of = C.n, N_Q, (lambda lv: -(-lv // N_P))
    levels = synth.stream(0, "levels").integers(4, L, n_pairs).tolist()
    st = synth.stream(0, "bench/batch")

    def cts():
        t = torch.empty((n_pairs, 2, L, n), dtype=torch.int32, device="cuda")
        for i in range(n_pairs):
            for h in range(2):
                t[i, h] = ck.to_device(st.residues(q, n))
        return t

    A, B = cts(), cts()
    rlk = torch.stack([torch.stack([ck.to_device(st.residues(q + p, n)) for _ in range(2)]) for _ in range(C.dnum)])
    out = torch.empty((n_pairs, 2, L - 1, n), dtype=torch.int32, device="cuda")
    items = C.batch_items(levels)
    ws = torch.empty(n_pairs * C.workspace_size(ck.OP_HMULT, L), dtype=torch.uint8, device="cuda")
    ws1 = torch.empty(C.workspace_size(ck.OP_HMULT, L), dtype=torch.uint8, device="cuda")
    outs1 = [torch.empty((2, lv - 1, n), dtype=torch.int32, device="cuda") for lv in levels]

    def plain():
        for i, lv in enumerate(levels):
            C.hmult_rescale(A[i], B[i], rlk, lv, outs1[i], ws=ws1)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.hmult_rescale_batch(A, B, items, L, rlk, out, ws=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        C.hmult_rescale_batch(A, B, items, L, rlk, out, ws=ws, stream=s)

    for _ in range(2):
        plain()
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    alg = sum((4 * lv + 2 * beta_of(lv) * (lv + N_P) + 2 * (lv - 1)) * LIMB for lv in levels)
    return {"workload": "%d HMult+relin+rescale pairs, levels uniform in [4, 24], N=2^16, dnum by level" % n_pairs,
            "pairs": n_pairs, "levels_mean": sum(levels) / len(levels),
            "plain_ops_per_s": n_pairs / t_plain, "batched_graph_ops_per_s": n_pairs / t_batch,
            "speedup": t_plain / t_batch, "batched_us_per_batch": 1e6 * t_batch,
            "batched_alg_bytes": alg, "batched_hbm_frac": alg / t_batch / 1e9 / HBM_PEAK_GBS}


def batched_top_level(C, ck, torch, cts, rlk, reps: int) -> dict:
    """The headline shape batched: the 16 distinct pairs at level 24 as one
    HMult+relin+rescale batch captured in a hipGraph (the key is read once
    per batch)."""
    L, n_pairs = N_Q, N_PAIRS
    A = torch.stack([cts[2 * i] for i in range(n_pairs)])
    B = torch.stack([cts[2 * i + 1] for i in range(n_pairs)])
    out = torch.empty((n_pairs, 2, L - 1, C.n), dtype=torch.int32, device="cuda")
    items = C.batch_items([L] * n_pairs)
    ws = torch.empty(n_pairs * C.workspace_size(ck.OP_HMULT, L), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.hmult_rescale_batch(A, B, items, L, rlk, out, ws=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        C.hmult_rescale_batch(A, B, items, L, rlk, out, ws=ws, stream=s)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    beta = C.dnum
    alg = (n_pairs * (4 * L + 2 * (L - 1)) + 2 * beta * (L + N_P)) * LIMB
    return {"workload": "%d HMult+relin+rescale pairs at level 24, one batched call in a hipGraph" % n_pairs,
            "ops_per_s": n_pairs / t, "us_per_op": 1e6 * t / n_pairs, "alg_bytes": alg,
            "hbm_frac": alg / t / 1e9 / HBM_PEAK_GBS}


def mechanisms(C, ck, torch, cts, rk, reps: int) -> dict:
    """HAdd, PAdd, PMult (element-wise, HBM-bound) and HConj at level 24 on
    distinct resident operands, one stream, plain launches."""
    L, beta = N_Q, C.dnum
    n_ops = len(cts) // 2
    pts = [cts[2 * i + 1][0] for i in range(n_ops)]  # [24][N] residues stand in for encoded plaintexts
    out = torch.empty((2, L, C.n), dtype=torch.int32, device="cuda")
    ws = torch.empty(C.workspace_size(ck.OP_HROT, L), dtype=torch.uint8, device="cuda")
    ops = {
        "hadd": (lambda i: C.hadd(cts[2 * (i % n_ops)], cts[2 * (i % n_ops) + 1], L, out), 6 * L),
        "padd": (lambda i: C.padd(cts[2 * (i % n_ops)], pts[i % n_ops], L, out), 5 * L),
        "pmult": (lambda i: C.pmult(cts[2 * (i % n_ops)], pts[i % n_ops], L, out), 5 * L),
        "hconj": (lambda i: C.hconj(cts[2 * (i % n_ops)], L, rk, out, ws=ws), 4 * L + 2 * beta * (L + N_P)),
    }
    res = {}
    for name, (fn, limbs) in ops.items():
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(reps):
            fn(i)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        res[name] = {"us": 1e6 * t, "alg_bytes": limbs * LIMB, "hbm_frac": limbs * LIMB / t / 1e9 / HBM_PEAK_GBS}
    return res


def rational_rescale(ck, torch, synth, reps: int) -> dict:
    """Rational rescaling in the 25-30 prime system at N=2^16 (Table 2's
    construction): each transition of the 2^40 cycle and one bootstrapping
    level, on uniformly random resident ciphertexts; a windowed context's
    precomputed four-pass plan (`us`) and the general path over arbitrary
    prime sets (`general_path_us`)."""
    from paper_2407_13055_amd import primes
    full, wins = primes.context_primes(LOG_N)
    p = ck.prime_chain(31, LOG_N, 1)
    C = ck.Context(LOG_N, full, p, windows=[(w[0], len(w)) for w in wins])  # precomputed transitions
    G = ck.Context(LOG_N, full, p)                                           # general prime-set path
    res = _rational_rescale_levels(C, ck, torch, synth, full, wins, reps)
    gen = _rational_rescale_levels(G, ck, torch, synth, full, wins, reps)
    for k, v in gen.items():
        res[k]["general_path_us"] = v["us"]
    C.close()
    G.close()
    return res


def prime_system(ck, torch, synth, reps: int, alpha: int = 4, tuned: bool = True) -> dict:
    """HMult + relinearisation on the 25-30 prime system at N=2^16: a windowed
    context over the 15 Table 2 primes (inverted-terminal order) plus alpha
    special primes, one key over P * Q_max for every level; per level, HMult
    alone, HMult followed by rational rescaling to the level below, and HMult
    with ModDown merged into that rescaling (one call)."""
    from paper_2407_13055_amd import primes
    full, wins = primes.context_primes(LOG_N)
    p = ck.prime_chain(31, LOG_N, alpha)
    C = ck.Context(LOG_N, full, p, windows=[(w[0], len(w)) for w in wins])
    if tuned:
        from paper_2407_13055_amd import tune
        tune.autotune(C, batch=16, reps=3)
    n = C.n
    rlk = synth.device_residues(0, "bench/ps/rlk", full + p, (C.dnum, 2), n, torch)
    res = {"alpha": alpha, "dnum": C.dnum, "tuning": C.tuning, "levels": {}}
    for lv in range(1, len(wins)):
        ids, below = wins[lv], wins[lv - 1]
        L = len(ids)
        mods = [full[i] for i in ids]
        a = synth.device_residues(0, "bench/ps/a/%d" % lv, mods, (2,), n, torch)
        b = synth.device_residues(0, "bench/ps/b/%d" % lv, mods, (2,), n, torch)
        h = torch.empty((2, L, n), dtype=torch.int32, device="cuda")
        o = torch.empty((2, len(below), n), dtype=torch.int32, device="cuda")
        ws = torch.empty(C.workspace_size(ck.OP_HMULT, L), dtype=torch.uint8, device="cuda")
        wr = torch.empty(C.workspace_size(ck.OP_RESCALE_RATIONAL, 0, L, len(below)), dtype=torch.uint8,
                         device="cuda")

        def hm():
            C.hmult(a, b, rlk, L, h, ws=ws)

        def hm_rs():
            C.hmult(a, b, rlk, L, h, ws=ws)
            C.rescale_rational(h, ids, below, o, ws=wr)

        def hm_merged():
            C.hmult_rescale(a, b, rlk, L, o, ws=ws)
        out = {"limbs": L, "window_start": ids[0]}
        for name, fn in (("hmult_us", hm), ("hmult_rescale_us", hm_rs), ("hmult_rescale_merged_us", hm_merged)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            out[name] = 1e6 * (time.perf_counter() - t0) / reps
        res["levels"][str(lv)] = out
    C.close()
    return res


def _rational_rescale_levels(C, ck, torch, synth, full, wins, reps: int) -> dict:
    n = C.n
    res = {}
    for frm in (4, 3, 2, 1, 8):
        ids_in, ids_out = wins[frm], wins[frm - 1]
        ct = synth.device_residues(0, "bench/rr/%d" % frm, [full[i] for i in ids_in], (2,), n, torch)
        out = torch.empty((2, len(ids_out), n), dtype=torch.int32, device="cuda")
        ws = torch.empty(C.workspace_size(ck.OP_RESCALE_RATIONAL, 0, len(ids_in), len(ids_out)), dtype=torch.uint8,
                         device="cuda")
        C.rescale_rational(ct, ids_in, ids_out, out, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            C.rescale_rational(ct, ids_in, ids_out, out, ws=ws)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        alg = (2 * len(ids_in) + 2 * len(ids_out)) * LIMB
        res["%d->%d" % (frm, frm - 1)] = {"limbs_in": len(ids_in), "limbs_out": len(ids_out), "us": 1e6 * t,
                                          "hbm_frac": alg / t / 1e9 / HBM_PEAK_GBS}
    return res


def rotations(C, ck, torch, synth, q, p, reps: int) -> dict:
    """32 distinct offsets from [1, 2^15 - 1] with 32 resident rotation keys:
    (i) one ciphertext at level 24, hoisted (one shared ModUp) vs 32 plain
    HRot; (ii) 32 ciphertexts at levels uniform in [8, 24], offset i for
    ciphertext i, one batched call in a hipGraph vs 32 plain HRot."""
    n, L = C.n, N_Q
    offs = synth.stream(0, "offsets").distinct(1, (1 << 15) - 1, 32).tolist()
    keys = synth.device_residues(0, "bench/rot/keys", q + p, (32, C.dnum, 2), n, torch)
    cts = synth.device_residues(0, "bench/rot/cts", q, (32, 2), n, torch)
    levels = synth.stream(0, "bench/rot/levels").integers(8, L, 32).tolist()
    ws1 = torch.empty(C.workspace_size(ck.OP_HROT, L), dtype=torch.uint8, device="cuda")
    outs = torch.empty((32, 2, L, n), dtype=torch.int32, device="cuda")
    items_h = C.batch_items([L] * 32, list(range(32)), offs)
    ws_h = torch.empty(C.workspace_size(ck.OP_HROT_HOISTED, L, 32), dtype=torch.uint8, device="cuda")
    items_b = C.batch_items(levels, list(range(32)), offs)
    ws_b = torch.empty(32 * C.workspace_size(ck.OP_HROT, L), dtype=torch.uint8, device="cuda")
    outb = torch.empty((32, 2, L, n), dtype=torch.int32, device="cuda")

    def plain_one():
        for i in range(32):
            C.hrot(cts[0], L, offs[i], keys[i], outs[i], ws=ws1)

    def hoisted():
        C.hrot_hoisted(cts[0], L, items_h, keys, outs, ws=ws_h)

    outs_many = [torch.empty((2, lv, n), dtype=torch.int32, device="cuda") for lv in levels]

    def plain_many():
        for i in range(32):
            C.hrot(cts[i], levels[i], offs[i], keys[i], outs_many[i], ws=ws1)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.hrot_batch(cts, items_b, L, keys, outb, ws=ws_b, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        C.hrot_batch(cts, items_b, L, keys, outb, ws=ws_b, stream=s)

    def tm(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # sum of plaintext-weighted rotations (one ModUp, one ModDown) vs the
    # hoisted rotations followed by 32 PMult and 31 HAdd
    pts = synth.device_residues(0, "bench/rot/pts", q + p, (32,), n, torch)
    acc = torch.empty((2, L, n), dtype=torch.int32, device="cuda")
    tmp = torch.empty((2, L, n), dtype=torch.int32, device="cuda")
    ws_s = torch.empty(C.workspace_size(ck.OP_HROT_SUM, L), dtype=torch.uint8, device="cuda")

    def lt_sum():
        C.hrot_sum_hoisted(cts[0], L, items_h, keys, pts, acc, ws=ws_s)

    def lt_composed():
        C.hrot_hoisted(cts[0], L, items_h, keys, outs, ws=ws_h)
        C.pmult(outs[0], pts[0], L, acc)
        for i in range(1, 32):
            C.pmult(outs[i], pts[i], L, tmp)
            C.hadd(acc, tmp, L, acc)

    t_p1, t_h = tm(plain_one), tm(hoisted)
    t_pm, t_b = tm(plain_many), tm(g.replay)
    t_ls, t_lc = tm(lt_sum), tm(lt_composed)
    # hoisted == plain, bit for bit, on this workload
    ref = torch.empty_like(outs)
    for i in range(32):
        C.hrot(cts[0], L, offs[i], keys[i], ref[i], ws=ws1)
    hoisted()
    torch.cuda.synchronize()
    same = bool(torch.equal(ref, outs))
    beta = C.dnum
    alg_h = (2 * L + 32 * 2 * beta * (L + N_P) + 32 * 2 * L) * LIMB
    return {"hoisted": {"workload": "1 ct at level 24, 32 offsets, 32 keys", "plain_us": 1e6 * t_p1,
                        "hoisted_us": 1e6 * t_h, "speedup": t_p1 / t_h, "identical_to_plain": same,
                        "alg_bytes": alg_h, "hbm_frac": alg_h / t_h / 1e9 / HBM_PEAK_GBS},
            "batched": {"workload": "32 cts, levels uniform in [8, 24], offset i with key i",
                        "plain_us": 1e6 * t_pm, "batched_graph_us": 1e6 * t_b, "speedup": t_pm / t_b},
            "weighted_sum": {"workload": "sum of 32 plaintext-weighted rotations of 1 ct at level 24",
                             "one_moddown_us": 1e6 * t_ls, "hoisted_then_pmult_hadd_us": 1e6 * t_lc,
                             "speedup": t_lc / t_ls,
                             "alg_bytes": (4 * L + 32 * (2 * beta * (L + N_P) + (L + N_P))) * LIMB,
                             "hbm_frac": (4 * L + 32 * (2 * beta * (L + N_P) + (L + N_P))) * LIMB / t_ls / 1e9
                             / HBM_PEAK_GBS}}


def serving(ck, torch, synth, seconds: float, warmup: float, rate: float, budget: float, hold: float,
            n_sample: int = 200, tuned: bool = True, linger: float = 0.0, lanes: int = 4, depth: int = 2) -> dict:
    """Continuous batching of Poisson-arriving HMult (70%, with rescale when
    the level is >= 2) and HRot (30%, offset from a 32-set) requests,
    N in {2^15, 2^16}, level uniform in [1, 24]; keys (relinearisation + 32
    rotation keys per N) and a pool of 16 input ciphertext pairs per N stay
    resident.  Latency is arrival to result-ready event on the host clock.
    With linger > 0 a group waits up to that long for a full batch while
    other batches are in flight.  n_sample requests' results are kept and rerun alone (single-op calls)."""
    from paper_2407_13055_amd import serving as sv
    log_ns, n_src = (15, 16), 16
    offs = synth.stream(0, "offsets").distinct(1, (1 << 15) - 1, 32).tolist()
    ctxs, pools, keys = {}, {}, {}
    for ln in log_ns:
        q, p = ck.prime_chain(30, ln, N_Q), ck.prime_chain(31, ln, N_P)
        C = ck.Context(ln, q, p)
        if tuned:
            from paper_2407_13055_amd import tune
            tune.autotune(C, batch=16, reps=3)
        ctxs[ln] = C
        n = 1 << ln
        pools[ln] = (synth.device_residues(0, "serve/a/%d" % ln, q, (n_src, 2), n, torch),
                     synth.device_residues(0, "serve/b/%d" % ln, q, (n_src, 2), n, torch))
        keys[ln] = (synth.device_residues(0, "serve/rlk/%d" % ln, q + p, (C.dnum, 2), n, torch),
                    synth.device_residues(0, "serve/rk/%d" % ln, q + p, (32, C.dnum, 2), n, torch))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # blocks cached from earlier runs would count as used
    free, _ = torch.cuda.mem_get_info()
    capacity = int(min(budget, free - (8 << 30)))
    reqs = sv.poisson_requests(0, rate, warmup + seconds, list(log_ns), {ln: N_Q for ln in log_ns}, offs, n_src)
    sample = set(synth.stream(0, "serving/sample").distinct(0, len(reqs) - 1, min(n_sample, len(reqs))).tolist())
    ex = sv.GpuExecutor(ck, torch, ctxs, pools, keys, capacity, lanes=lanes, depth=depth)
    kept = {}

    def on_ready(r, b):
        if r.rid in sample:
            kept[r.rid] = ex.result(b, r.slot).clone()
            torch.cuda.current_stream().synchronize()  # before the arena range can be reused

    clock = sv.RealClock()
    ex.start(clock)
    rep = sv.Server(ex, capacity, max_batch=ex.max_batch, hold=hold, on_ready=on_ready,
                    linger=linger).run(reqs, clock)
    torch.cuda.synchronize()
    out = rep.summary(warmup)
    out.update({"offered_req_per_s": rate, "seconds": seconds, "warmup_s": warmup, "budget_bytes": int(budget),
                "arena_bytes": capacity, "hold_s": hold, "linger_s": linger, "lanes": ex.lanes, "depth": ex.depth,
                "max_batch": ex.max_batch})
    same = 0
    by_rid = {r.rid: r for r in reqs}
    for rid, got in kept.items():
        r = by_rid[rid]
        C = ctxs[r.log_n]
        A, B = pools[r.log_n]
        rlk, rks = keys[r.log_n]
        o = torch.empty((2, r.out_level, C.n), dtype=torch.int32, device="cuda")
        if r.kind == sv.K_HROT:
            C.hrot(A[r.src], r.level, r.rot, rks[r.key], o)
        elif r.kind == sv.K_HMULT_RS:
            C.hmult_rescale(A[r.src], B[r.src], rlk, r.level, o)
        else:
            C.hmult(A[r.src], B[r.src], rlk, r.level, o)
        same += bool(torch.equal(o, got))
    out["alone_vs_mix"] = {"checked": len(kept), "identical": same}
    for C in ctxs.values():
        C.close()
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return os.uname().machine


def _host_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(n, 1)


def cpu_baseline(q, p, runs: int = 5) -> dict:
    """The oracle on the headline operation (HMult+relin+rescale, N=2^16,
    24+8 primes): the median of `runs` runs single-threaded and the median of
    `runs` runs with its limb loops on every host thread this process may use
    (the oracle's -fopenmp build; same results)."""
    import numpy as np

    import oracle
    import synth
    P = oracle.Params(LOG_N, q, p)
    st = synth.stream(1, "bench/cpu")
    a = np.stack([st.residues(q, P.n), st.residues(q, P.n)])
    b = np.stack([st.residues(q, P.n), st.residues(q, P.n)])
    rlk = np.stack([np.stack([st.residues(q + p, P.n), st.residues(q + p, P.n)]) for _ in range(P.dnum)])

    def median_s(threads):
        used = oracle.use_threads(threads)
        ts = []
        for _ in range(runs):
            t0 = time.perf_counter()
            oracle.rescale(P, oracle.hmult(P, a, b, rlk, N_Q), N_Q)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2], used

    t1, _ = median_s(1)
    threads = _host_threads()
    tn, used = median_s(threads)
    oracle.use_threads(1)
    return {"value": 1.0 / tn, "unit": "ops/s", "cores": used, "kind": "oracle",
            "sample": "HMult+relin+rescale at N=2^16, 24+8 primes, dnum 3: median of %d runs on %d threads "
                      "(OpenMP over limbs) and of %d single-thread runs" % (runs, used, runs),
            "single_thread_ops_per_s": 1.0 / t1, "median_s": tn, "single_thread_median_s": t1,
            "nproc": os.cpu_count(), "model": _cpu_model()}


def compact_line(res: dict, details_path) -> dict:
    """The one-line record: headline, roofline, whole-operation ceilings, CPU
    baseline and short summaries of the batched / rotation / serving runs
    (everything else is in the details file)."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "roofline", "whole_op", "hmult_relin_us", "hrot_us",
            "hmult_then_rescale_us", "cpu_baseline")
    out = {k: res[k] for k in keep if k in res}
    out["tuning"] = res.get("tuning", {}).get("applied")

    def r3(x):
        return None if x is None else round(float(x), 3)
    if "batched" in res:
        b, t = res["batched"], res.get("batched_top_level", {})
        out["batched"] = {"pairs": res["batched"].get("pairs"), "levels": "U{4..24}",
                          "plain_ops_per_s": r3(b["plain_ops_per_s"]),
                          "graph_ops_per_s": r3(b["batched_graph_ops_per_s"]), "speedup": r3(b["speedup"]),
                          "hbm_frac": r3(b["batched_hbm_frac"]),
                          "top_level_16_us_per_op": r3(t.get("us_per_op")),
                          "top_level_16_speedup": r3(t.get("speedup_vs_plain"))}
    if "rotations" in res:
        ro = res["rotations"]
        out["rotations"] = {"hoisted_32_speedup": r3(ro["hoisted"]["speedup"]),
                            "hoisted_identical": ro["hoisted"]["identical_to_plain"],
                            "batched_32_speedup": r3(ro["batched"]["speedup"]),
                            "weighted_sum_speedup": r3(ro["weighted_sum"]["speedup"])}
    if "serving" in res:
        sv = res["serving"]
        out["serving"] = {k: sv.get(k) for k in ("ops_per_s", "p50_ms", "p99_ms", "mean_batch", "arena_bytes")}
        out["serving"]["alone_vs_mix"] = "%d/%d" % (sv["alone_vs_mix"]["identical"], sv["alone_vs_mix"]["checked"])
    out["details"] = details_path
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-runs", type=int, default=5, help="oracle runs per CPU-baseline leg (median)")
    ap.add_argument("--details", default=None, metavar="PATH",
                    help="write the full record here (default: $CKKS_BENCH_DETAILS, else "
                         "bench_results/bench_details.json)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-pair batched comparison")
    ap.add_argument("--batch-pairs", type=int, default=64)
    ap.add_argument("--batch-reps", type=int, default=20)
    ap.add_argument("--no-rotations", action="store_true", help="skip the 32-rotation comparisons")
    ap.add_argument("--no-prime-system", action="store_true",
                    help="skip the 25-30 prime system sections (rational rescaling, windowed HMult)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes (no autotuning)")
    ap.add_argument("--tuning", default="", metavar="UP,DOWN,XCD,ROWS,COLTHREADS,ROWS1,KM,KM1,COLS,COLS1",
                    help="apply these launch shapes instead of autotuning (ckks_tuning fields in order)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop runs")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="also run a plain device copy of BYTES of random data (counter calibration)")
    ap.add_argument("--summarize-op", nargs=6, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "SQ_DIR", "NAME", "CMD"),
                    help="write profiles/op_NAME.txt from four rocprofv3 runs of CMD and exit")
    args = ap.parse_args()
    if args.summarize_op:
        kd, fd, wd, sd, name, cmd = args.summarize_op
        summarize_op(kd, fd, wd, sd, name, args.copy_probe or (256 << 20), cmd)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on exactly one GPU (the library has no multi-GPU component); "
              "got --gpus %d / WORLD_SIZE %d" % (args.gpus, world), file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2407_13055_amd as ck
    import synth

    q, p = ck.prime_chain(30, LOG_N, N_Q), ck.prime_chain(31, LOG_N, N_P)
    C = ck.Context(LOG_N, q, p)
    n, level, alpha, beta = C.n, N_Q, N_P, C.dnum
    tuned = None
    if args.tuning:
        C.tune(*(int(v) for v in args.tuning.split(",")))
    elif not args.no_tune:
        from paper_2407_13055_amd import tune
        print("bench: autotuning launch shapes", file=sys.stderr, flush=True)
        tuned = tune.autotune(C, batch=16, reps=5)
    dev = "cuda"

    def residues(st, mods):
        return ck.to_device(st.residues(mods, n), dev)

    st = synth.stream(0, "bench/inputs")
    cts = [torch.stack([residues(st, q), residues(st, q)]) for _ in range(2 * N_PAIRS)]
    rlk = torch.stack([torch.stack([residues(st, q + p), residues(st, q + p)]) for _ in range(beta)])
    rk = torch.stack([torch.stack([residues(st, q + p), residues(st, q + p)]) for _ in range(beta)])
    out = torch.empty((2, level, n), dtype=torch.int32, device=dev)
    rs = torch.empty((2, level - 1, n), dtype=torch.int32, device=dev)
    ws = torch.empty(max(C.workspace_size(ck.OP_HMULT, level), C.workspace_size(ck.OP_RESCALE)),
                     dtype=torch.uint8, device=dev)

    def hmult_rescale(i):
        C.hmult_rescale(cts[2 * (i % N_PAIRS)], cts[2 * (i % N_PAIRS) + 1], rlk, level, rs, ws=ws)

    def hmult_then_rescale(i):
        C.hmult(cts[2 * (i % N_PAIRS)], cts[2 * (i % N_PAIRS) + 1], rlk, level, out, ws=ws)
        C.rescale(out, rs, ws=ws)

    def hmult_only(i):
        C.hmult(cts[2 * (i % N_PAIRS)], cts[2 * (i % N_PAIRS) + 1], rlk, level, out, ws=ws)

    def hrot(i):
        C.hrot(cts[i % (2 * N_PAIRS)], level, 1, rk, out, ws=ws)

    def timed(fn, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            fn(i)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for i in range(args.warmup):
        hmult_rescale(i)
        hrot(i)
    print("bench: warmup done", file=sys.stderr, flush=True)
    t_main = timed(hmult_rescale, args.steps)
    t_hm = timed(hmult_only, args.steps)
    t_seq = timed(hmult_then_rescale, args.steps)
    t_hr = timed(hrot, args.steps)
    # host-side enqueue cost of one step (no synchronisation inside)
    torch.cuda.synchronize()
    h0 = time.perf_counter()
    for i in range(args.steps):
        hmult_rescale(i)
    t_host = time.perf_counter() - h0
    torch.cuda.synchronize()
    print("bench: timed regions done", file=sys.stderr, flush=True)

    # live per-kernel timing (HIP events on the launch stream), same workload
    C.profile_start(max_launches=16 * args.steps + 64)
    timed(hmult_rescale, args.steps)
    C.profile_stop()
    prof = C.profile_report()
    kb = alg_bytes_per_kernel(level, alpha, beta)
    per_kernel = {k: {"launches": c, "avg_us": 1e3 * ms / c,
                      "alg_GBs": (kb[k] / (ms / c * 1e-3) / 1e9) if k in kb else None}
                  for k, (c, ms) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][1])
    dom_avg_s = prof[dom][1] / prof[dom][0] * 1e-3
    ms_step = 1e3 * t_main / args.steps
    op_bytes = op_alg_bytes(level, alpha, beta, rescale=True)
    # one launch of the dominant kernel serves one operation: its algorithmic
    # bytes are the operation's (inputs, key rows used, output)
    achieved = op_bytes / dom_avg_s / 1e9
    # counter figures of the same kernels (profiles/op_*.txt, when taken on these sources)
    oprof = op_profile("hmult_rescale_n16_l24")
    dprof = kernel_profile(oprof, dom)
    traffic = dprof.get("traffic_bytes")
    op_traffic = float(oprof["traffic_bytes_per_op"]) if oprof else None
    alu_floor = float(oprof["alu_floor_us"]) if oprof else None
    res = {
        "metric": METRIC,
        "value": args.steps / t_main,
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "HMult+relin+rescale, one ciphertext pair per op (plain per-op launches), "
                               "N=2^16, 24 x 30-bit q + 8 x 31-bit p, dnum 3, 16 distinct pairs cycled",
                   "log_n": LOG_N, "level": level, "alpha": alpha, "dnum": beta, "distinct_pairs": N_PAIRS},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": op_bytes,
                     "avg_us": dom_avg_s * 1e6, "kernel_model_bytes": kb.get(dom),
                     "kernel_model_frac": (kb[dom] / dom_avg_s / 1e9 / HBM_PEAK_GBS) if dom in kb else None,
                     "valu_util": (dprof["valu_instr"] / (dom_avg_s * VALU_PEAK_WAVE_INSTR)) if dprof else None},
        "whole_op": {"us": ms_step * 1e3, "alg_bytes": op_bytes, "achieved_GBs": op_bytes / (ms_step * 1e-3) / 1e9,
                     "hbm_frac": op_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "hbm_floor_us": op_bytes / HBM_PEAK_GBS / 1e3,
                     "alu_floor_us": alu_floor,
                     "alu_frac": (alu_floor / (ms_step * 1e3)) if alu_floor else None,
                     "traffic": op_traffic,
                     "traffic_over_alg": (op_traffic / op_bytes) if op_traffic else None},
        "hmult_relin_us": 1e6 * t_hm / args.steps,
        "hmult_relin_hbm_frac": op_alg_bytes(level, alpha, beta, False) / (t_hm / args.steps) / 1e9 / HBM_PEAK_GBS,
        "hrot_us": 1e6 * t_hr / args.steps,
        "hmult_then_rescale_us": 1e6 * t_seq / args.steps,
        "host_enqueue_us_per_step": 1e6 * t_host / args.steps,
        "kernels": per_kernel,
        "tuning": {"applied": C.tuning,
                   "source": tuned["source"] if tuned else ("given" if args.tuning else "default"),
                   "candidates_us": tuned["table"] if tuned else []},
    }
    if not args.no_batched:
        res["batched"] = batched_vs_plain(C, ck, torch, synth, q, p, args.batch_pairs, args.batch_reps)
        res["batched_top_level"] = batched_top_level(C, ck, torch, cts, rlk, args.batch_reps)
        res["batched_top_level"]["speedup_vs_plain"] = res["batched_top_level"]["ops_per_s"] / res["value"]
    res["mechanisms"] = mechanisms(C, ck, torch, cts, rk, 200)
    if not args.no_prime_system:
        print("bench: 25-30 prime system", file=sys.stderr, flush=True)
        res["rational_rescale"] = rational_rescale(ck, torch, synth, 100)
        res["prime_system_25_30"] = prime_system(ck, torch, synth, 100, tuned=not args.no_tune)
    if not args.no_rotations:
        print("bench: rotations", file=sys.stderr, flush=True)
        res["rotations"] = rotations(C, ck, torch, synth, q, p, args.batch_reps)
    if not args.no_serving:
        print("bench: serving", file=sys.stderr, flush=True)
        res["serving"] = serving(ck, torch, synth, args.serve_seconds, 1.0, args.serve_rate, 200e9, 0.0,
                                 tuned=not args.no_tune)
        print("bench: serving under a 1 GB budget", file=sys.stderr, flush=True)
        res["serving_1GB"] = serving(ck, torch, synth, 3.0, 0.5, args.serve_rate, 1e9, 0.05, n_sample=50)
        print("bench: serving at 10x the arrival rate", file=sys.stderr, flush=True)
        res["serving_overload"] = serving(ck, torch, synth, 2.0, 0.5, 10 * args.serve_rate, 200e9, 0.0, n_sample=50)
        print("bench: serving at 10x the arrival rate, 200 us linger", file=sys.stderr, flush=True)
        res["serving_overload_linger"] = serving(ck, torch, synth, 2.0, 0.5, 10 * args.serve_rate, 200e9, 0.0,
                                                 n_sample=50, linger=200e-6)
    if args.copy_probe:
        src = torch.randint(0, 1 << 30, (args.copy_probe // 4,), dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):  # one elementwise kernel reading and writing copy_probe bytes each
            torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        print("bench: CPU oracle runs", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(q, p, args.cpu_runs)
    details = args.details or os.environ.get("CKKS_BENCH_DETAILS") or os.path.join("bench_results",
                                                                                  "bench_details.json")
    try:
        os.makedirs(os.path.dirname(os.path.abspath(details)), exist_ok=True)
        with open(details, "w") as f:
            json.dump(res, f, indent=1)
        print("bench: full record in %s" % details, file=sys.stderr, flush=True)
    except OSError as e:
        print("bench: could not write %s (%s)" % (details, e), file=sys.stderr, flush=True)
        details = None
    print(json.dumps(compact_line(res, details)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
