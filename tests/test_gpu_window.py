"""GPU parity of key switching over windows of the prime list (Sec. 3.2,
3.3): a windowed context whose levels are the Table 2 levels of the 25-30
prime system (inverted-terminal order), every level using one key over
P * Q_max.  HMult, HMult with ModDown merged into rational rescaling to
the level below, HRot (plain and hoisted), HConj and the element-wise
mechanisms are bit-exact against the oracle at N = 2^12 and 2^16, for digit
widths that make windows start inside a key digit; an encryption multiplied
on the GPU and rescaled rationally to the level below (separately and
merged) decrypts to the product; batched calls mix windows per item; calls
that need prefix levels are refused."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402

N_LEVELS = len(oracle.TABLE2_LEVELS)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_sys = {}


def system(log_n, alpha):
    """(context, full list, special primes, windows by Table 2 level)."""
    if (log_n, alpha) not in _sys:
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        taus, qs = oracle.prime_system_25_30(log_n)
        full = list(taus[::-1]) + list(qs)
        p = oracle.prime_chain(31, log_n, alpha)
        wins = []
        for lv in range(N_LEVELS):
            mods = oracle.level_primes(taus, qs, lv)
            wins.append((full.index(mods[0]), len(mods)))
        _sys[(log_n, alpha)] = (ck.Context(log_n, full, p, windows=wins), full, p, wins)
    return _sys[(log_n, alpha)]


def random_key(full, p, log_n, name, n=None):
    st = synth.stream(80, "gpu/win/key/" + name)
    mods = full + p
    dnum = -(-len(full) // len(p))
    one = lambda: np.stack([np.stack([st.residues(mods, 1 << log_n), st.residues(mods, 1 << log_n)])
                            for _ in range(dnum)])
    return one() if n is None else np.stack([one() for _ in range(n)])


def window_ct(full, start, length, log_n, name):
    st = synth.stream(81, "gpu/win/ct/" + name)
    mods = full[start:start + length]
    return np.stack([st.residues(mods, 1 << log_n), st.residues(mods, 1 << log_n)])


@pytest.mark.parametrize("log_n,alpha,levels", [(12, 2, tuple(range(N_LEVELS))), (12, 3, tuple(range(N_LEVELS))),
                                                (12, 5, tuple(range(N_LEVELS))), (16, 3, tuple(range(N_LEVELS))),
                                                (16, 2, tuple(range(N_LEVELS))), (16, 4, tuple(range(N_LEVELS)))])
def test_hmult_over_windows_matches_oracle(log_n, alpha, levels):
    C, full, p, wins = system(log_n, alpha)
    key = random_key(full, p, log_n, "rlk/%d/%d" % (log_n, alpha))
    dkey = ck.to_device(key)
    for lv in levels:
        start, length = wins[lv]
        a = window_ct(full, start, length, log_n, "a/%d/%d" % (log_n, lv))
        b = window_ct(full, start, length, log_n, "b/%d/%d" % (log_n, lv))
        say("hmult N=2^%d alpha=%d level %d window [%d, %d)" % (log_n, alpha, lv, start, start + length))
        out = torch.zeros((2, length, 1 << log_n), dtype=torch.int32, device="cuda")
        C.hmult(ck.to_device(a), ck.to_device(b), dkey, length, out)
        torch.cuda.synchronize()
        want = oracle.hmult_window(full, p, start, length, a, b, key, log_n)
        assert np.array_equal(ck.to_host(out), want), (log_n, alpha, lv)


@pytest.mark.parametrize("log_n,alpha,levels", [(12, 2, tuple(range(1, N_LEVELS))),
                                                (12, 3, tuple(range(1, N_LEVELS))),
                                                (16, 3, tuple(range(1, N_LEVELS))),
                                                (16, 4, tuple(range(1, N_LEVELS)))])
def test_merged_hmult_rescale_over_windows_matches_oracle(log_n, alpha, levels):
    """ckks_hmult_rescale on a windowed context: one ModDown merged into the
    rational rescaling to the window below, every Table 2 transition
    (1 -> 0 shares no prime, 8 -> 7 drops one at each end)."""
    C, full, p, wins = system(log_n, alpha)
    key = random_key(full, p, log_n, "mrlk/%d/%d" % (log_n, alpha))
    dkey = ck.to_device(key)
    for lv in levels:
        (s0, l0), (s1, l1) = wins[lv], wins[lv - 1]
        a = window_ct(full, s0, l0, log_n, "ma/%d/%d" % (log_n, lv))
        b = window_ct(full, s0, l0, log_n, "mb/%d/%d" % (log_n, lv))
        say("hmult_rescale (merged) N=2^%d alpha=%d level %d -> %d" % (log_n, alpha, lv, lv - 1))
        out = torch.zeros((2, l1, 1 << log_n), dtype=torch.int32, device="cuda")
        C.hmult_rescale(ck.to_device(a), ck.to_device(b), dkey, l0, out)
        torch.cuda.synchronize()
        want = oracle.hmult_rescale_window(full, p, s0, l0, s1, l1, a, b, key, log_n)
        assert np.array_equal(ck.to_host(out), want), (log_n, alpha, lv)


@pytest.mark.parametrize("log_n,alpha,levels", [(12, 3, (0, 4, 7)), (16, 2, (5,))])
def test_hrot_and_hconj_over_windows_match_oracle(log_n, alpha, levels):
    C, full, p, wins = system(log_n, alpha)
    key = random_key(full, p, log_n, "rk/%d/%d" % (log_n, alpha))
    dkey = ck.to_device(key)
    for lv in levels:
        start, length = wins[lv]
        ct = window_ct(full, start, length, log_n, "rot/%d/%d" % (log_n, lv))
        dct = ck.to_device(ct)
        out = torch.zeros((2, length, 1 << log_n), dtype=torch.int32, device="cuda")
        say("hrot / hconj N=2^%d alpha=%d level %d" % (log_n, alpha, lv))
        C.hrot(dct, length, 11, dkey, out)
        torch.cuda.synchronize()
        g = oracle.galois_element(11, log_n)
        assert np.array_equal(ck.to_host(out), oracle.hrot_window(full, p, start, length, ct, g, key, log_n)), lv
        C.hconj(dct, length, dkey, out)
        torch.cuda.synchronize()
        g = oracle.conj_galois(log_n)
        assert np.array_equal(ck.to_host(out), oracle.hrot_window(full, p, start, length, ct, g, key, log_n)), lv


def test_hoisted_rotations_over_a_window_match_oracle():
    """Hoisted HRot (one shared ModUp) at a window that starts inside a key
    digit, three rotations with their own keys."""
    log_n, alpha, lv = 12, 3, 6
    C, full, p, wins = system(log_n, alpha)
    start, length = wins[lv]
    assert start % alpha != 0
    keys = random_key(full, p, log_n, "hoist", n=3)
    rots = [1, 7, 300]
    ct = window_ct(full, start, length, log_n, "hoist")
    outs = torch.zeros((3, 2, length, 1 << log_n), dtype=torch.int32, device="cuda")
    say("hrot_hoisted level", lv)
    C.hrot_hoisted(ck.to_device(ct), length, C.batch_items([length] * 3, [0, 1, 2], rots), ck.to_device(keys), outs)
    torch.cuda.synchronize()
    got = ck.to_host(outs)
    for i, k in enumerate(rots):
        want = oracle.hrot_window(full, p, start, length, ct, oracle.galois_element(k, log_n), keys[i], log_n)
        assert np.array_equal(got[i], want), k


def test_elementwise_over_a_window_matches_oracle():
    log_n, alpha, lv = 12, 3, 5
    C, full, p, wins = system(log_n, alpha)
    start, length = wins[lv]
    mods = full[start:start + length]
    a = window_ct(full, start, length, log_n, "ew/a")
    b = window_ct(full, start, length, log_n, "ew/b")
    pt = synth.stream(82, "gpu/win/pt").residues(mods, 1 << log_n)
    Pw = oracle.Params(log_n, mods, p)
    da, db, dp = ck.to_device(a), ck.to_device(b), ck.to_device(pt)
    out = torch.zeros((2, length, 1 << log_n), dtype=torch.int32, device="cuda")
    say("elementwise level", lv)
    for fn, x, want in ((C.hadd, db, oracle.hadd(Pw, a, b, length)), (C.padd, dp, oracle.padd(Pw, a, pt, length)),
                        (C.pmult, dp, oracle.pmult(Pw, a, pt, length))):
        fn(da, x, length, out)
        torch.cuda.synchronize()
        assert np.array_equal(ck.to_host(out), want), fn.__name__


def test_windowed_hmult_then_rational_rescale_decrypts():
    """Encrypt u, v at 2^40 over level 6's window (oracle, real keys over
    P * Q_max), HMult and rescale to level 5 on the GPU (HMult then rational
    rescaling, and the merged call), decrypt u * v at 2^80 * Q_5 / Q_6."""
    log_n, alpha, lv = 12, 3, 6
    C, full, p, wins = system(log_n, alpha)
    P = oracle.Params(log_n, full, p)
    s = synth.stream(83, "gpu/win/secret").ternary(P.n, 64)
    st = synth.stream(83, "gpu/win/rlk")
    rlk = oracle.relin_key(P, s, np.stack([st.residues(full + p, P.n) for _ in range(P.dnum)]),
                           np.stack([st.gaussian(P.n) for _ in range(P.dnum)]))
    (s0, l0), (s1, l1) = wins[lv], wins[lv - 1]
    mi, mo = full[s0:s0 + l0], full[s1:s1 + l1]

    def enc(u, name):
        e = synth.stream(83, "gpu/win/enc/" + name)
        a = e.residues(mi, P.n)
        s_ntt = oracle.to_ntt(s, mi, log_n)
        m = oracle.encode(u, log_n, 2.0 ** 40) + e.gaussian(P.n)
        return np.stack([oracle.add_mod(oracle.neg_mod(oracle.mul_mod(a, s_ntt, mi), mi),
                                        oracle.to_ntt(m, mi, log_n), mi), a])
    u = synth.stream(83, "gpu/win/u").complex_slots(P.n // 2)
    v = synth.stream(83, "gpu/win/v").complex_slots(P.n // 2)
    h = torch.zeros((2, l0, P.n), dtype=torch.int32, device="cuda")
    out = torch.zeros((2, l1, P.n), dtype=torch.int32, device="cuda")
    say("windowed hmult + rational rescale, level", lv)
    ca, cb, drlk = ck.to_device(enc(u, "u")), ck.to_device(enc(v, "v")), ck.to_device(rlk)
    C.hmult(ca, cb, drlk, l0, h)
    C.rescale_rational(h, list(range(s0, s0 + l0)), list(range(s1, s1 + l1)), out)
    merged = torch.zeros_like(out)
    C.hmult_rescale(ca, cb, drlk, l0, merged)
    torch.cuda.synchronize()
    scale = 2.0 ** 80 * math.prod(mo) / math.prod(mi)
    Po = oracle.Params(log_n, mo, p)
    for res in (out, merged):
        got = oracle.decrypt(Po, ck.to_host(res), s, scale)
        assert np.max(np.abs(got - u * v)) <= 2.0 ** -12


def test_windowed_context_refusals():
    log_n, alpha = 12, 3
    C, full, p, wins = system(log_n, alpha)
    n = 1 << log_n
    start, length = wins[5]
    ct = torch.zeros((2, length, n), dtype=torch.int32, device="cuda")
    key = torch.zeros((C.dnum, 2, len(full) + alpha, n), dtype=torch.int32, device="cuda")
    out = torch.zeros((2, length, n), dtype=torch.int32, device="cuda")
    low = wins[0][1]
    c0 = torch.zeros((2, low, n), dtype=torch.int32, device="cuda")
    with pytest.raises(ck.CkksError):
        C.hmult_rescale(c0, c0, key, low, c0.clone())                       # no window below the lowest
    with pytest.raises(ck.CkksError):
        C.rescale(ct, out[:, :length - 1].contiguous())                     # no single rescaling
    with pytest.raises(ck.CkksError):
        C.hmult(ct, ct, key, 4, out[:, :4].contiguous())                        # no window has 4 limbs
    with pytest.raises(ck.CkksError):
        C.hmult(ct, ct, key, wins[4][1], out[:, :wins[4][1]].contiguous())    # inputs above the level
    a = torch.zeros((1, 2, low, n), dtype=torch.int32, device="cuda")
    with pytest.raises(ck.CkksError):
        C.hmult_rescale_batch(a, a, C.batch_items([low]), low, key, a.clone())   # no window below max_level
    with pytest.raises(ck.CkksError):
        ck.Context(log_n, full, p, windows=[(0, 3), (2, 3)])                 # two windows of 3 limbs
    with pytest.raises(ck.CkksError):
        ck.Context(log_n, full, p, windows=[(13, 3)])                        # past the end of the list
    for bad in ([(0, 0)], [(-1, 3)], [(0, 65)], [(2 ** 31 - 2, 3)], []):   # empty, negative, too long, overflow
        with pytest.raises(ck.CkksError):
            ck.Context(log_n, full, p, windows=bad)


@pytest.mark.parametrize("log_n,alpha", [(12, 3), (16, 2)])
def test_rescale_rational_on_a_windowed_context_matches_oracle(log_n, alpha):
    """ckks_rescale_rational between a window and the window below takes the
    context's precomputed four-pass plan; any other pair of prime sets takes
    the general path.  Both bit-exact against the oracle."""
    C, full, p, wins = system(log_n, alpha)
    cases = [(lv, lv - 1) for lv in range(1, N_LEVELS)] + [(4, 2), (8, 5)]
    for frm, to in cases:
        (s0, l0), (s1, l1) = wins[frm], wins[to]
        mi, mo = full[s0:s0 + l0], full[s1:s1 + l1]
        ct = window_ct(full, s0, l0, log_n, "rr/%d/%d" % (frm, to))
        out = torch.zeros((2, l1, 1 << log_n), dtype=torch.int32, device="cuda")
        say("rescale_rational N=2^%d window level %d -> %d" % (log_n, frm, to))
        C.rescale_rational(ck.to_device(ct), list(range(s0, s0 + l0)), list(range(s1, s1 + l1)), out)
        torch.cuda.synchronize()
        assert np.array_equal(ck.to_host(out), oracle.rescale_rational(ct, mi, mo, log_n)), (frm, to)


def test_rotation_sum_over_a_window_matches_oracle():
    """Weighted rotation sum (one ModUp, one ModDown) at a window that starts
    inside a key digit; plaintexts indexed by prime id over the whole list."""
    log_n, alpha, lv = 12, 3, 7
    C, full, p, wins = system(log_n, alpha)
    start, length = wins[lv]
    assert start % alpha != 0
    keys = random_key(full, p, log_n, "sum", n=3)
    rots = [2, 9, 1000]
    ct = window_ct(full, start, length, log_n, "sum")
    st = synth.stream(84, "gpu/win/sum/pts")
    pts = np.stack([st.residues(full + p, 1 << log_n) for _ in range(3)])
    out = torch.zeros((2, length, 1 << log_n), dtype=torch.int32, device="cuda")
    say("hrot_sum_hoisted level", lv)
    C.hrot_sum_hoisted(ck.to_device(ct), length, C.batch_items([length] * 3, [0, 1, 2], rots), ck.to_device(keys),
                       ck.to_device(pts), out)
    torch.cuda.synchronize()
    gs = [oracle.galois_element(k, log_n) for k in rots]
    want = oracle.hrot_sum_window(full, p, start, length, ct, gs, list(keys), list(pts), log_n)
    assert np.array_equal(ck.to_host(out), want)


@pytest.mark.parametrize("log_n,alpha", [(12, 3), (16, 2)])
def test_batched_calls_over_windows_match_oracle(log_n, alpha):
    """Batched HMult, HMult + merged rational rescaling and HRot on a
    windowed context: items at different windows in one launch (slot i holds
    item i's ciphertext in its first limbs), bit-exact per item; an item
    whose limb count names no window is skipped (its output untouched)."""
    C, full, p, wins = system(log_n, alpha)
    n = 1 << log_n
    by_len = {l: (st, l) for st, l in wins}
    top = wins[-1][1]
    lens = [wins[lv][1] for lv in (8, 3, 5, 1, 6)] + [4]          # 4 limbs: no such window
    m = len(lens)
    key = random_key(full, p, log_n, "batch/%d/%d" % (log_n, alpha))
    rks = random_key(full, p, log_n, "batch/rk/%d/%d" % (log_n, alpha), n=m)
    A = np.zeros((m, 2, top, n), dtype=np.uint32)
    B = np.zeros((m, 2, top, n), dtype=np.uint32)
    for i, l in enumerate(lens):
        st = by_len[l][0] if l in by_len else 0
        A[i, :, :l] = window_ct(full, st, l, log_n, "batch/a/%d" % i)
        B[i, :, :l] = window_ct(full, st, l, log_n, "batch/b/%d" % i)
    dA, dB, dkey = ck.to_device(A), ck.to_device(B), ck.to_device(key)
    rots = [3, 77, 1, 500, 9, 2]

    say("hmult_batch windows", lens)
    out = torch.zeros((m, 2, top, n), dtype=torch.int32, device="cuda")
    C.hmult_batch(dA, dB, C.batch_items(lens), top, dkey, out)
    torch.cuda.synchronize()
    got = ck.to_host(out)
    for i, l in enumerate(lens):
        if l not in by_len:
            assert not got[i].any(), "item %d at a limb count with no window was not skipped" % i
            continue
        want = oracle.hmult_window(full, p, by_len[l][0], l, A[i, :, :l], B[i, :, :l], key, log_n)
        assert np.array_equal(got[i, :, :l], want), (i, l)

    say("hmult_rescale_batch (merged) windows", lens)
    below = {wins[k][1]: wins[k - 1] for k in range(1, len(wins))}
    out_l = below[top][1]
    outr = torch.zeros((m, 2, out_l, n), dtype=torch.int32, device="cuda")
    C.hmult_rescale_batch(dA, dB, C.batch_items(lens), top, dkey, outr)
    torch.cuda.synchronize()
    got = ck.to_host(outr)
    for i, l in enumerate(lens):
        if l not in below:
            assert not got[i].any(), i
            continue
        (s0, l0), (s1, l1) = by_len[l], below[l]
        want = oracle.hmult_rescale_window(full, p, s0, l0, s1, l1, A[i, :, :l], B[i, :, :l], key, log_n)
        assert np.array_equal(got[i, :, :l1], want), (i, l)

    say("hrot_batch windows", lens)
    outh = torch.zeros((m, 2, top, n), dtype=torch.int32, device="cuda")
    C.hrot_batch(dA, C.batch_items(lens, list(range(m)), rots), top, ck.to_device(rks), outh)
    torch.cuda.synchronize()
    got = ck.to_host(outh)
    for i, l in enumerate(lens):
        if l not in by_len:
            assert not got[i].any(), i
            continue
        g = oracle.galois_element(rots[i], log_n)
        want = oracle.hrot_window(full, p, by_len[l][0], l, A[i, :, :l], g, rks[i], log_n)
        assert np.array_equal(got[i, :, :l], want), (i, l)


def test_windowed_batch_graph_replays():
    """A batched merged HMult + rescaling on a windowed context captured in
    a graph, replayed three times with rewritten items (windows) and inputs,
    eager work and synchronization between the replays; every replay
    bit-exact against the oracle."""
    log_n, alpha = 12, 3
    C, full, p, wins = system(log_n, alpha)
    n = 1 << log_n
    by_len = {l: st for st, l in wins}
    below = {wins[k][1]: wins[k - 1] for k in range(1, len(wins))}
    top = wins[-1][1]
    m = 3
    key = random_key(full, p, log_n, "graph")
    dkey = ck.to_device(key)
    a_d = torch.zeros((m, 2, top, n), dtype=torch.int32, device="cuda")
    b_d = torch.zeros_like(a_d)
    items = C.batch_items([top] * m)
    out = torch.zeros((m, 2, below[top][1], n), dtype=torch.int32, device="cuda")
    ws = torch.empty(m * C.workspace_size(ck.OP_HMULT, top), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.hmult_rescale_batch(a_d, b_d, items, top, dkey, out, ws=ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        C.hmult_rescale_batch(a_d, b_d, items, top, dkey, out, ws=ws, stream=s)
    for rep in range(3):
        lvs = synth.stream(85, "gpu/win/graph/%d" % rep).distinct(1, len(wins) - 1, m).tolist()
        lens = [wins[lv][1] for lv in lvs]
        A = np.zeros((m, 2, top, n), dtype=np.uint32)
        B = np.zeros_like(A)
        for i, l in enumerate(lens):
            A[i, :, :l] = window_ct(full, by_len[l], l, log_n, "graph/a/%d/%d" % (rep, i))
            B[i, :, :l] = window_ct(full, by_len[l], l, log_n, "graph/b/%d/%d" % (rep, i))
        a_d.copy_(ck.to_device(A))
        b_d.copy_(ck.to_device(B))
        items.copy_(C.batch_items(lens))
        torch.cuda.synchronize()
        say("windowed graph replay", rep, lens)
        g.replay()
        torch.cuda.synchronize()
        got = ck.to_host(out)
        for i, l in enumerate(lens):
            (s1, l1) = below[l]
            want = oracle.hmult_rescale_window(full, p, by_len[l], l, s1, l1, A[i, :, :l], B[i, :, :l], key, log_n)
            assert np.array_equal(got[i, :, :l1], want), (rep, i, l)
