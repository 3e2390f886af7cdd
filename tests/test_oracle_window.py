"""Pins for key switching over a window of the prime list with one key over
P * Q_max (Sec. 3.2, 3.3): the digit pieces partition the window; a window
at the start of the list is the ordinary prefix-level key switching (the C
implementation); HMult and HRot over every window of the Table 2
construction decrypt to the product / rotation, including windows that cut
a key digit, and HMult followed by rational rescaling decrypts at the scale
of the level below."""
import math

import numpy as np
import pytest

import oracle
import synth

LOG_N = 12
N_LEVELS = len(oracle.TABLE2_LEVELS)


def system(alpha):
    taus, qs = oracle.prime_system_25_30(LOG_N)
    full = list(taus[::-1]) + list(qs)
    p = oracle.prime_chain(31, LOG_N, alpha)
    return taus, qs, full, p


def window_of(full, mods):
    start = full.index(mods[0])
    assert full[start:start + len(mods)] == list(mods)
    return start, len(mods)


@pytest.mark.parametrize("alpha,start,length", [(1, 0, 5), (2, 3, 9), (3, 1, 13), (3, 4, 2), (4, 2, 11), (5, 0, 15)])
def test_window_digits_partition(alpha, start, length):
    pieces = oracle.window_digits(alpha, start, length)
    covered = [i for _, lo, hi in pieces for i in range(lo, hi)]
    assert covered == list(range(start, start + length))
    for jk, lo, hi in pieces:
        assert lo < hi and lo // alpha == jk and (hi - 1) // alpha == jk  # inside key digit jk


def keys(full, p, seed, rot=None):
    P = oracle.Params(LOG_N, full, p)
    s = synth.stream(seed, "win/secret").ternary(P.n, 64)
    mods = full + p
    st = synth.stream(seed, "win/key/%s" % rot)
    a = np.stack([st.residues(mods, P.n) for _ in range(P.dnum)])
    e = np.stack([st.gaussian(P.n) for _ in range(P.dnum)])
    if rot is None:
        return P, s, oracle.relin_key(P, s, a, e)
    return P, s, oracle.rotation_key(P, s, rot, a, e)


@pytest.mark.parametrize("alpha,length", [(1, 3), (2, 5), (3, 4)])
def test_prefix_window_is_the_prefix_level(alpha, length):
    """start = 0: the window functions (numpy composition) reproduce the C
    implementation of prefix-level HMult and HRot bit for bit."""
    q = oracle.prime_chain(30, LOG_N, 6)
    p = oracle.prime_chain(31, LOG_N, alpha)
    P = oracle.Params(LOG_N, q, p)
    st = synth.stream(70, "win/prefix/%d" % alpha)
    mods = q + p
    key = np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
    a = np.stack([st.residues(q[:length], P.n), st.residues(q[:length], P.n)])
    b = np.stack([st.residues(q[:length], P.n), st.residues(q[:length], P.n)])
    assert np.array_equal(oracle.hmult_window(q, p, 0, length, a, b, key, LOG_N), oracle.hmult(P, a, b, key, length))
    g = oracle.galois_element(3, LOG_N)
    assert np.array_equal(oracle.hrot_window(q, p, 0, length, a, g, key, LOG_N), oracle.hrot(P, a, length, g, key))


def encrypt(mods, u, scale, s, name):
    st = synth.stream(71, "win/enc/" + name)
    m = oracle.encode(u, LOG_N, scale)
    a = st.residues(mods, 1 << LOG_N)
    s_ntt = oracle.to_ntt(s, mods, LOG_N)
    b = oracle.add_mod(oracle.neg_mod(oracle.mul_mod(a, s_ntt, mods), mods),
                       oracle.to_ntt(m + st.gaussian(1 << LOG_N), mods, LOG_N), mods)
    return np.stack([b, a])


def decrypt(mods, p, ct, s, scale):
    return oracle.decrypt(oracle.Params(LOG_N, list(mods), p), ct, s, scale)


@pytest.mark.parametrize("alpha,levels", [(2, tuple(range(1, 9))), (3, tuple(range(1, 9)))])
def test_hmult_over_table2_windows_decrypts(alpha, levels):
    """Table 2 levels 1-8 (level 0 cannot hold a 2^80 product): encrypt u, v
    at 2^40 over the level's window, HMult with the one key over P * Q_max,
    decrypt u * v at 2^80; rescale rationally to the level below and decrypt
    at 2^80 * Q_{l-1} / Q_l.  With alpha = 2 the windows starting at an odd
    prime (levels 5, 7), with alpha = 3 most windows, start inside a key
    digit."""
    taus, qs, full, p = system(alpha)
    P, s, rlk = keys(full, p, 72)
    u = synth.stream(72, "win/u").complex_slots(P.n // 2)
    v = synth.stream(72, "win/v").complex_slots(P.n // 2)
    cut = 0
    for lv in levels:
        mods = oracle.level_primes(taus, qs, lv)
        start, length = window_of(full, mods)
        cut += start % alpha != 0
        ca = encrypt(mods, u, 2.0 ** 40, s, "u/%d" % lv)
        cb = encrypt(mods, v, 2.0 ** 40, s, "v/%d" % lv)
        h = oracle.hmult_window(full, p, start, length, ca, cb, rlk, LOG_N)
        assert np.max(np.abs(decrypt(mods, p, h, s, 2.0 ** 80) - u * v)) <= 2.0 ** -12, lv
        below = oracle.level_primes(taus, qs, lv - 1)
        r = oracle.rescale_rational(h, mods, below, LOG_N)
        scale = 2.0 ** 80 * math.prod(below) / math.prod(mods)
        assert np.max(np.abs(decrypt(below, p, r, s, scale) - u * v)) <= 2.0 ** -12, lv
    assert cut >= 2


def test_hrot_over_windows_decrypts():
    """HRot by k over every Table 2 window (alpha = 3: most cut a key digit)
    decrypts to the slots rotated left by k."""
    taus, qs, full, p = system(3)
    k = 5
    P, s, rk = keys(full, p, 73, rot=k)
    u = synth.stream(73, "win/rot/u").complex_slots(P.n // 2)
    g = oracle.galois_element(k, LOG_N)
    for lv in range(N_LEVELS):
        mods = oracle.level_primes(taus, qs, lv)
        start, length = window_of(full, mods)
        ct = encrypt(mods, u, 2.0 ** 40, s, "rot/%d" % lv)
        out = oracle.hrot_window(full, p, start, length, ct, g, rk, LOG_N)
        assert np.max(np.abs(decrypt(mods, p, out, s, 2.0 ** 40) - np.roll(u, -k))) <= 2.0 ** -12, lv


def test_wrong_key_digit_fails_to_decrypt():
    """Sanity of the pin itself: the same window with the key's digits taken
    as if the window started at prime 0 does not decrypt."""
    taus, qs, full, p = system(2)
    P, s, rlk = keys(full, p, 74)
    u = synth.stream(74, "win/bad/u").complex_slots(P.n // 2)
    mods = oracle.level_primes(taus, qs, 5)
    start, length = window_of(full, mods)
    assert start % 2 == 1
    ca = encrypt(mods, u, 2.0 ** 40, s, "bad/a")
    cb = encrypt(mods, u, 2.0 ** 40, s, "bad/b")
    # the list rotated so the window starts at 0: key row i (not start + i)
    # and key digit i // alpha serve window prime i
    bad = oracle.hmult_window(full[start:] + full[:start], p, 0, length, ca, cb, rlk, LOG_N)
    assert np.max(np.abs(decrypt(mods, p, bad, s, 2.0 ** 80) - u * u)) > 1.0


@pytest.mark.parametrize("alpha,levels", [(2, tuple(range(1, 9))), (3, tuple(range(1, 9)))])
def test_merged_hmult_rescale_decrypts(alpha, levels):
    """HMult with ModDown merged into rational rescaling: encryptions of u, v
    at 2^40 over a level's window come out over the window below and decrypt
    to u * v at 2^80 * Q_{l-1} / Q_l.  Covers level 1 -> 0 (no prime in
    common) and 8 -> 7 (a prime dropped at each end)."""
    taus, qs, full, p = system(alpha)
    P, s, rlk = keys(full, p, 75)
    u = synth.stream(75, "win/m/u").complex_slots(P.n // 2)
    v = synth.stream(75, "win/m/v").complex_slots(P.n // 2)
    for lv in levels:
        mods = oracle.level_primes(taus, qs, lv)
        below = oracle.level_primes(taus, qs, lv - 1)
        (s0, l0), (s1, l1) = window_of(full, mods), window_of(full, below)
        ca = encrypt(mods, u, 2.0 ** 40, s, "m/u/%d" % lv)
        cb = encrypt(mods, v, 2.0 ** 40, s, "m/v/%d" % lv)
        out = oracle.hmult_rescale_window(full, p, s0, l0, s1, l1, ca, cb, rlk, LOG_N)
        scale = 2.0 ** 80 * math.prod(below) / math.prod(mods)
        assert np.max(np.abs(decrypt(below, p, out, s, scale) - u * v)) <= 2.0 ** -12, lv


@pytest.mark.parametrize("alpha,lv", [(2, 5), (3, 2), (3, 8)])
def test_merged_is_sequential_up_to_rounding(alpha, lv):
    """For arbitrary residues and key, the merged result and HMult followed
    by rational rescaling differ in every coefficient by at most the two
    roundings' error: |merged - sequential| <= alpha + |D| + 4 (exact CRT of
    the difference over the output primes)."""
    taus, qs, full, p = system(alpha)
    mods, below = oracle.level_primes(taus, qs, lv), oracle.level_primes(taus, qs, lv - 1)
    (s0, l0), (s1, l1) = window_of(full, mods), window_of(full, below)
    st = synth.stream(76, "win/seq/%d/%d" % (alpha, lv))
    dnum = -(-len(full) // alpha)
    key = np.stack([np.stack([st.residues(full + p, 1 << LOG_N), st.residues(full + p, 1 << LOG_N)])
                    for _ in range(dnum)])
    a = np.stack([st.residues(mods, 1 << LOG_N), st.residues(mods, 1 << LOG_N)])
    b = np.stack([st.residues(mods, 1 << LOG_N), st.residues(mods, 1 << LOG_N)])
    merged = oracle.hmult_rescale_window(full, p, s0, l0, s1, l1, a, b, key, LOG_N)
    seq = oracle.rescale_rational(oracle.hmult_window(full, p, s0, l0, a, b, key, LOG_N), mods, below, LOG_N)
    n_drop = len([m for m in mods if m not in below])
    for h in range(2):
        diff = oracle.add_mod(merged[h], oracle.neg_mod(seq[h], below), below)
        c = oracle.crt_centered(oracle.intt(diff, below, LOG_N)[:, :256], below)
        assert max(abs(x) for x in c) <= alpha + n_drop + 4, (h, max(abs(x) for x in c))


def test_prefix_window_rotation_sum_is_the_prefix_level():
    """start = 0: the window rotation sum reproduces the C implementation of
    the prefix-level weighted rotation sum bit for bit."""
    q = oracle.prime_chain(30, LOG_N, 5)
    p = oracle.prime_chain(31, LOG_N, 2)
    P = oracle.Params(LOG_N, q, p)
    st = synth.stream(77, "win/sum")
    mods = q + p
    keys = [np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
            for _ in range(2)]
    pts = [st.residues(mods, P.n) for _ in range(2)]
    ct = np.stack([st.residues(q[:4], P.n), st.residues(q[:4], P.n)])
    gs = [oracle.galois_element(k, LOG_N) for k in (3, 100)]
    assert np.array_equal(oracle.hrot_sum_window(q, p, 0, 4, ct, gs, keys, pts, LOG_N),
                          oracle.hrot_sum_hoisted(P, ct, 4, gs, keys, pts))
