"""Pins for the automorphism (Sec. 2.2 Eq. 4): the coefficient form is the
substitution X -> X^g, the NTT-domain form is Eq. 4's column permutation,
and on encoded messages it rotates slots."""
import numpy as np
import pytest

import oracle
import synth


def brev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


def substitute(a, g, q):
    """a(X^g) mod (X^N + 1, q) by plain polynomial arithmetic."""
    n = len(a)
    out = [0] * n
    for i, c in enumerate(a):
        e = i * g
        sign = -1 if (e // n) % 2 else 1
        out[e % n] = (out[e % n] + sign * int(c)) % q
    return out


@pytest.mark.parametrize("log_n", [4, 6])
def test_coefficient_form_is_substitution(log_n):
    q = oracle.prime_chain(24, log_n, 1)[0]
    a = synth.stream(11, "aut/coef").residues([q], 1 << log_n)
    for k in (1, 2, 3):
        g = oracle.galois_element(k, log_n)
        assert oracle.automorph_coef(a, [q], log_n, g)[0].tolist() == substitute(a[0], g, q)
    g = 2 * (1 << log_n) - 1  # conjugation element
    assert oracle.automorph_coef(a, [q], log_n, g)[0].tolist() == substitute(a[0], g, q)


def test_ntt_form_matches_coefficient_form(params_small):
    P = params_small
    mods = P.q
    a = synth.stream(12, "aut/ntt").residues(mods, P.n)
    for k in (1, 5, 1000, P.n // 2 - 1):
        g = oracle.galois_element(k, P.log_n)
        via_coef = oracle.ntt(oracle.automorph_coef(oracle.intt(a, mods, P.log_n), mods, P.log_n, g), mods, P.log_n)
        assert np.array_equal(oracle.automorph_ntt(a, P.log_n, g), via_coef)


def test_ntt_form_is_eq4_permutation():
    """Eq. 4 moves natural-order column i to j = ((2i+1) 5^-r mod 2N - 1)/2."""
    log_n = 5
    n = 1 << log_n
    x = np.arange(n, dtype=np.uint32)[None, :]  # bit-reversed storage of distinct labels
    for r in (1, 2, 7):
        out = oracle.automorph_ntt(x, log_n, oracle.galois_element(r, log_n))[0]
        inv5r = pow(pow(5, r, 2 * n), -1, 2 * n)
        for i in range(n):
            j = (((2 * i + 1) * inv5r) % (2 * n) - 1) // 2
            assert out[brev(j, log_n)] == x[0, brev(i, log_n)]


def test_rotation_of_slots(params_small):
    P = params_small
    z = synth.stream(13, "aut/slots").complex_slots(P.n // 2)
    scale = 2.0 ** 40
    m = oracle.encode(z, P.log_n, scale)
    mods = [P.q[0], P.q[1]]
    for k in (1, 3, 100):
        g = oracle.galois_element(k, P.log_n)
        r = oracle.automorph_coef(oracle.reduce_signed(m, mods, P.log_n), mods, P.log_n, g)
        coef = np.array(oracle.crt_centered(r, mods), dtype=np.float64)
        got = oracle.decode(coef, P.log_n, scale)
        assert np.max(np.abs(got - np.roll(z, -k))) < 2.0 ** -20
