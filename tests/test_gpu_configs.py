"""GPU parity at the benchmark's own configurations, against the oracle:

* N = 2^15 with the 24 + 8 prime chain (the serving loop's smaller ring):
  HMult, HMult + rescale, HRot and the batched calls at levels 24, 9, 1;
* the batched HMult + rescale of many pairs at N = 2^16 (24 + 8 primes), one
  item per digit count (1, 2 and 3 digits) plus levels of the benchmark's own
  draw, run as the benchmark runs it: one batched call captured in a hipGraph
  and replayed;
* rotations by offsets of the benchmark's 32-offset set at N = 2^16, hoisted
  (one shared ModUp) and batched over ciphertexts at levels in [8, 24].

Each case runs under the default launch shapes (the autotuner's pick on
MI355X), under the all-16-residue shapes and under mixes of the two (the
kernels differ per setting; results must not).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402

# launch shapes: the defaults (the tuner's pick on MI355X: 16 residues per
# thread in batched row passes, one wave per row in KeyMult and in
# single-operation row passes, Col4 column passes), the all-16 shapes, and
# mixes of the two; every entry but the first names each knob
_ALL16 = {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 256,
          "rows_per_thread_single": 16, "keymult_rows": 16, "keymult_rows_single": 16, "cols_per_thread": 16,
          "cols_per_thread_single": 16}
TUNINGS = [
    {},
    _ALL16,
    {**_ALL16, "col_threads": 128, "rows_per_thread_single": 4},
    {**_ALL16, "bconv_tpw_up": 1, "bconv_tpw_down": 1, "rows_per_thread": 4, "rows_per_thread_single": 4},
    {**_ALL16, "col_threads": 128, "rows_per_thread_single": 4, "keymult_rows": 4, "keymult_rows_single": 4},
    {**_ALL16, "bconv_tpw_down": 4, "rows_per_thread": 4, "rows_per_thread_single": 4, "keymult_rows": 4,
     "keymult_rows_single": 4, "cols_per_thread": 4, "cols_per_thread_single": 0},
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()


def apply(C, t):
    if t:
        C.tune(**t)
    else:
        C.tune()


def rand_cts(P, n, level, name):
    st = synth.stream(21, name)
    return np.stack([np.stack([st.residues(P.q[:level], P.n), st.residues(P.q[:level], P.n)]) for _ in range(n)])


def rand_keys(P, n, name):
    st = synth.stream(21, name)
    mods = P.q + P.p
    return np.stack([np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
                     for _ in range(n)])


def same(got, want, what):
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d mismatches, first at %s" % (what, len(bad), bad[:4].tolist())


@pytest.fixture(scope="module")
def params_15():
    """N = 2^15 with the 2^17-chain: 24 x 30-bit q, 8 x 31-bit p (dnum 3)."""
    return oracle.Params(15, oracle.prime_chain(30, 16, 24), oracle.prime_chain(31, 16, 8))


def test_n15_single_and_batched(params_15):
    P = params_15
    C = ck.Context(P.log_n, P.q, P.p)
    L = P.n_q
    levels = [24, 9, 1]
    n = len(levels)
    a, b = rand_cts(P, n, L, "n15/a"), rand_cts(P, n, L, "n15/b")
    rlk = rand_keys(P, 1, "n15/rlk")[0]
    rk = rand_keys(P, 1, "n15/rk")[0]
    k = 5
    g = oracle.galois_element(k, P.log_n)
    say("n15: oracle")
    w_hm = [oracle.hmult(P, a[i], b[i], rlk, lv) for i, lv in enumerate(levels)]
    w_rs = [oracle.rescale(P, w_hm[i], lv) if lv >= 2 else None for i, lv in enumerate(levels)]
    w_rot = [oracle.hrot(P, a[i], lv, g, rk) for i, lv in enumerate(levels)]
    A, B, R, K = ck.to_device(a), ck.to_device(b), ck.to_device(rlk), ck.to_device(rk)
    for t in TUNINGS:
        apply(C, t)
        for i, lv in enumerate(levels):
            say("n15 single", t, "level", lv)
            o = torch.empty((2, lv, P.n), dtype=torch.int32, device="cuda")
            C.hmult(A[i], B[i], R, lv, o)
            r = torch.empty((2, lv, P.n), dtype=torch.int32, device="cuda")
            C.hrot(A[i], lv, k, K, r)
            torch.cuda.synchronize()
            same(ck.to_host(o), w_hm[i], "hmult level %d %s" % (lv, t))
            same(ck.to_host(r), w_rot[i], "hrot level %d %s" % (lv, t))
            if lv >= 2:
                rs = torch.empty((2, lv - 1, P.n), dtype=torch.int32, device="cuda")
                C.hmult_rescale(A[i], B[i], R, lv, rs)
                torch.cuda.synchronize()
                same(ck.to_host(rs), w_rs[i], "hmult_rescale level %d %s" % (lv, t))
        say("n15 batched", t)
        rs_lv = [24, 9, 2]  # rescaling needs level >= 2
        w_b = [w_rs[0], w_rs[1], oracle.rescale(P, oracle.hmult(P, a[2], b[2], rlk, 2), 2)]
        ob = torch.zeros((n, 2, L - 1, P.n), dtype=torch.int32, device="cuda")
        C.hmult_rescale_batch(A, B, C.batch_items(rs_lv), L, R, ob)
        oh = torch.zeros((n, 2, L, P.n), dtype=torch.int32, device="cuda")
        C.hmult_batch(A, B, C.batch_items(levels), L, R, oh)
        orot = torch.zeros((n, 2, L, P.n), dtype=torch.int32, device="cuda")
        C.hrot_batch(A, C.batch_items(levels, [0] * n, [k] * n), L, K[None], orot)
        torch.cuda.synchronize()
        gb, gh, gr = ck.to_host(ob), ck.to_host(oh), ck.to_host(orot)
        for i in range(n):
            same(gb[i][:, :rs_lv[i] - 1], w_b[i], "hmult_rescale_batch item %d %s" % (i, t))
            same(gh[i][:, :levels[i]], w_hm[i], "hmult_batch item %d %s" % (i, t))
            same(gr[i][:, :levels[i]], w_rot[i], "hrot_batch item %d %s" % (i, t))
    C.close()


def bench_levels(n):
    """The benchmark's draw of batch levels (uniform in [4, 24])."""
    return synth.stream(0, "levels").integers(4, 24, 64).tolist()[:n]


def test_config2_batch_in_graph(params_full):
    """Batched HMult + rescale at N = 2^16 as the benchmark runs it (one call
    captured in a hipGraph, replayed), every item against the oracle."""
    P = params_full
    C = ck.Context(P.log_n, P.q, P.p)
    L = P.n_q
    levels = [24, 4, 12] + bench_levels(3)  # 3, 1 and 2 digits, then the benchmark's first draws
    n = len(levels)
    a, b = rand_cts(P, n, L, "cfg2/a"), rand_cts(P, n, L, "cfg2/b")
    rlk = rand_keys(P, 1, "cfg2/rlk")[0]
    say("config 2: oracle", levels)
    want = [oracle.rescale(P, oracle.hmult(P, a[i], b[i], rlk, lv), lv) for i, lv in enumerate(levels)]
    A, B, R = ck.to_device(a), ck.to_device(b), ck.to_device(rlk)
    items = C.batch_items(levels)
    out = torch.zeros((n, 2, L - 1, P.n), dtype=torch.int32, device="cuda")
    for t in TUNINGS:
        apply(C, t)
        ws = torch.empty(n * C.workspace_size(ck.OP_HMULT, L), dtype=torch.uint8, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            C.hmult_rescale_batch(A, B, items, L, R, out, ws=ws, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            C.hmult_rescale_batch(A, B, items, L, R, out, ws=ws, stream=s)
        for rep in range(2):
            out.zero_()
            torch.cuda.synchronize()
            say("config 2 replay", rep, t)
            g.replay()
            torch.cuda.synchronize()
            got = ck.to_host(out)
            for i, lv in enumerate(levels):
                same(got[i][:, :lv - 1], want[i], "item %d level %d replay %d %s" % (i, lv, rep, t))
        del g
    C.close()


def test_config3_rotations(params_full):
    """Offsets of the benchmark's 32-set at N = 2^16: hoisted rotations of one
    level-24 ciphertext and batched rotations at levels in [8, 24]."""
    P = params_full
    C = ck.Context(P.log_n, P.q, P.p)
    L = P.n_q
    offs = synth.stream(0, "offsets").distinct(1, (1 << 15) - 1, 32).tolist()
    sel = [0, 7, 19, 31]
    rots = [offs[i] for i in sel]
    n = len(rots)
    keys = rand_keys(P, n, "cfg3/keys")
    ct = rand_cts(P, n, L, "cfg3/ct")
    lv_b = [24, 8] + synth.stream(0, "bench/rot/levels").integers(8, 24, 32).tolist()[:2]
    gs = [oracle.galois_element(r, P.log_n) for r in rots]
    say("config 3: oracle", rots, lv_b)
    w_h = [oracle.hrot(P, ct[0], L, gs[i], keys[i]) for i in range(n)]
    w_b = [oracle.hrot(P, ct[i], lv_b[i], gs[i], keys[i]) for i in range(n)]
    CT, K = ck.to_device(ct), ck.to_device(keys)
    for t in TUNINGS:
        apply(C, t)
        say("config 3 hoisted / batched", t)
        outs = torch.zeros((n, 2, L, P.n), dtype=torch.int32, device="cuda")
        C.hrot_hoisted(CT[0], L, C.batch_items([L] * n, list(range(n)), rots), K, outs)
        ob = torch.zeros((n, 2, L, P.n), dtype=torch.int32, device="cuda")
        C.hrot_batch(CT, C.batch_items(lv_b, list(range(n)), rots), L, K, ob)
        torch.cuda.synchronize()
        gh, gb = ck.to_host(outs), ck.to_host(ob)
        for i in range(n):
            same(gh[i], w_h[i], "hoisted k=%d %s" % (rots[i], t))
            same(gb[i][:, :lv_b[i]], w_b[i], "batched k=%d level %d %s" % (rots[i], lv_b[i], t))
    C.close()
