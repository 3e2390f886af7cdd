"""Pins for the 25-30 prime system and rational rescaling (Sec. 3.2, 3.3,
Table 2, the rescaling sequence of Sec. 5.1): the moduli and scales Table 2
prints, contiguous inverted-terminal windows, the exact rounding error of
rational rescaling against big-integer arithmetic, and decryption after
rescaling an encryption."""
import math

import numpy as np
import pytest

import oracle
import synth

# log2 Q per level as printed in Table 2 (levels 0..8)
TABLE2_LOG2Q = [50, 90, 130, 170, 210, 265, 320, 375, 430]


@pytest.mark.parametrize("log_n", [12, 15, 16])
def test_table2_moduli_and_scales(log_n):
    taus, qs = oracle.prime_system_25_30(log_n)
    assert all(abs(math.log2(t) - 25) < 0.2 and (t - 1) % (2 << log_n) == 0 for t in taus)
    assert all(q < 1 << 30 and (q - 1) % (2 << log_n) == 0 for q in qs)
    logq = [math.log2(math.prod(oracle.level_primes(taus, qs, lv))) for lv in range(len(TABLE2_LOG2Q))]
    for lv, want in enumerate(TABLE2_LOG2Q):
        assert abs(logq[lv] - want) < 0.35, (lv, logq[lv])  # Table 2 prints nominal bit counts
    # Sec. 3.2: the scale stays within 2^39.9 .. 2^40.1.  At N = 2^16 the
    # NTT-friendly primes near 2^25 are about 0.1 bit apart, so the best
    # terminal primes reach 0.12 bit there.
    tol = 0.1 if log_n <= 15 else 0.12
    for lv in range(1, len(TABLE2_LOG2Q)):
        delta = logq[lv] - logq[lv - 1]
        assert abs(delta - (40 if lv <= 4 else 55)) < tol, (lv, delta)


def test_levels_are_contiguous_windows():
    taus, qs = oracle.prime_system_25_30(12)
    full = list(taus[::-1]) + list(qs)
    for lv in range(len(oracle.TABLE2_LEVELS)):
        w = oracle.level_primes(taus, qs, lv)
        start = full.index(w[0])
        assert full[start:start + len(w)] == w


def crt(x, mods):
    return oracle.crt_centered(x, mods)


@pytest.mark.parametrize("frm", [4, 3, 2, 1, 5])
def test_rational_rescale_rounding_is_exact(frm):
    """out = Q_A X / Q_D + u with |u| <= (|D| + 1) / 2 + 1 for every coefficient,
    X the centred CRT value of the input (big-integer check, coefficient
    domain, modulo Q_out)."""
    log_n = 12
    taus, qs = oracle.prime_system_25_30(log_n)
    mi, mo = oracle.level_primes(taus, qs, frm), oracle.level_primes(taus, qs, frm - 1)
    drop = [m for m in mi if m not in mo]
    add = [m for m in mo if m not in mi]
    st = synth.stream(61, "rr/%d" % frm)
    ct = np.stack([st.residues(mi, 1 << log_n), st.residues(mi, 1 << log_n)])
    out = oracle.rescale_rational(ct, mi, mo, log_n)
    qa, qd, qout = math.prod(add), math.prod(drop), math.prod(mo)
    bound = (len(drop) + 1) / 2 + 1
    for h in range(2):
        x = crt(oracle.intt(ct[h], mi, log_n)[:, :64], mi)
        y = crt(oracle.intt(out[h], mo, log_n)[:, :64], mo)
        for xv, yv in zip(x, y):
            d = (yv * qd - xv * qa) % (qout * qd)
            d = d - qout * qd if d > qout * qd // 2 else d
            assert abs(d) <= bound * qd, (frm, d / qd)


def encrypt_big(mods, log_n, u, scale_bits, s, name):
    """Encryption of u at scale 2^scale_bits over `mods`, with the message
    encoded at 2^40 and multiplied by 2^(scale_bits - 40) exactly (the scale
    exceeds what a 64-bit coefficient holds)."""
    n = 1 << log_n
    st = synth.stream(62, "rr/enc/" + name)
    m = [int(c) << (scale_bits - 40) for c in oracle.encode(u, log_n, 2.0 ** 40)]
    e = st.gaussian(n)
    coef = np.stack([np.array([(m[j] + int(e[j])) % q for j in range(n)], dtype=np.uint32) for q in mods])
    a = st.residues(mods, n)
    s_ntt = oracle.to_ntt(s, mods, log_n)
    b = oracle.add_mod(oracle.neg_mod(oracle.mul_mod(a, s_ntt, mods), mods), oracle.ntt(coef, mods, log_n), mods)
    return np.stack([b, a])


@pytest.mark.parametrize("frm,scale_bits", [(4, 80), (3, 80), (2, 80), (5, 95)])
def test_rational_rescale_decrypts(frm, scale_bits):
    """Encrypt at 2^80 (2^95 on a bootstrapping level), rescale to the level
    below: the scale becomes 2^scale_bits * Q_{l-1} / Q_l (about 2^40) and
    the slots decrypt to u within 2^-12."""
    log_n = 12
    taus, qs = oracle.prime_system_25_30(log_n)
    mi, mo = oracle.level_primes(taus, qs, frm), oracle.level_primes(taus, qs, frm - 1)
    s = synth.stream(63, "rr/secret").ternary(1 << log_n, 64)
    u = synth.stream(63, "rr/msg").complex_slots(1 << (log_n - 1))
    ct = encrypt_big(mi, log_n, u, scale_bits, s, str(frm))
    out = oracle.rescale_rational(ct, mi, mo, log_n)
    Po = oracle.Params(log_n, mo, [oracle.prime_chain(31, log_n, 1)[0]])
    scale = 2.0 ** scale_bits * math.prod(mo) / math.prod(mi)
    got = oracle.decrypt(Po, out, s, scale)
    assert np.max(np.abs(got - u)) <= 2.0 ** -12


@pytest.mark.parametrize("log_n", [12, 16])
def test_library_prime_system_matches_the_oracle(log_n):
    """The package's own prime-system construction (used by the benchmark)
    and the oracle's are independent implementations of the same selection."""
    from paper_2407_13055_amd import primes
    assert primes.prime_system_25_30(log_n) == oracle.prime_system_25_30(log_n)
    taus, qs = oracle.prime_system_25_30(log_n)
    full, wins = primes.context_primes(log_n)
    for lv, ids in enumerate(wins):
        assert [full[i] for i in ids] == oracle.level_primes(taus, qs, lv)
