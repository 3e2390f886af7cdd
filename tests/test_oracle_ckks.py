"""Mechanism-level pins for the oracle: encoding, key identities, the
key-switching error bound, and decrypt(HMult) / decrypt(HRot) against fp64
plaintext arithmetic within 2^-12."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import Keys


def test_encode_matches_canonical_embedding_definition():
    """m(zeta^(5^j)) = scale * z_j, evaluated by brute force at N = 8."""
    log_n, n = 3, 8
    z = synth.stream(14, "enc/def").complex_slots(n // 2)
    m = oracle.encode(z, log_n, 2.0 ** 30)
    zeta = np.exp(1j * np.pi / n)
    for j in range(n // 2):
        root = zeta ** pow(5, j, 2 * n)
        val = sum(float(m[k]) * root ** k for k in range(n))
        assert abs(val / 2.0 ** 30 - z[j]) < 2.0 ** -26


def test_encode_decode_round_trip(params_full):
    z = synth.stream(15, "enc/rt").complex_slots(params_full.n // 2)
    m = oracle.encode(z, params_full.log_n, 2.0 ** 30)
    assert np.max(np.abs(oracle.decode(m.astype(np.float64), params_full.log_n, 2.0 ** 30) - z)) < 2.0 ** -20


@pytest.fixture(scope="module")
def keys_small(params_small):
    return Keys(params_small, 0, rot_ks=(1, 5))


@pytest.fixture(scope="module")
def keys_mid(params_mid):
    return Keys(params_mid, 0, rot_ks=(1, 3))


def test_switch_key_identity(keys_small, keys_mid):
    """evk_j.b + evk_j.a * s - g_j * s^2 = e_j exactly (a small integer poly)."""
    for K in (keys_small, keys_mid):
        P = K.P
        mods = P.q + P.p
        s_ntt = oracle.to_ntt(K.s, mods, P.log_n)
        s2 = oracle.mul_mod(s_ntt, s_ntt, mods)
        for j in range(P.dnum):
            v = oracle.add_mod(K.rlk[j, 0], oracle.mul_mod(K.rlk[j, 1], s_ntt, mods), mods)
            for i in P.digits(P.n_q)[j]:
                gs = (s2[i].astype(np.uint64) * (P.P % P.q[i]) % P.q[i]).astype(np.uint32)
                v[i] = ((v[i].astype(np.uint64) + P.q[i] - gs) % P.q[i]).astype(np.uint32)
            e = oracle.crt_centered(oracle.intt(v, mods, P.log_n)[:, :64], mods)
            assert max(abs(x) for x in e) <= 19


@pytest.mark.parametrize("which", ["small", "mid"])
def test_keyswitch_error_bound(which, keys_small, keys_mid):
    """u0 + u1 s - d s^2 stays below the key-switching error bound
    sum_j |D_j| D_j/2 * 6 sigma sqrt(N) / P + (ceil(alpha/2)+1/2)(h+1)."""
    K = keys_small if which == "small" else keys_mid
    P = K.P
    level = P.n_q
    d = synth.stream(16, "ks/d").residues(P.q[:level], P.n)
    u0, u1 = oracle.keyswitch(P, d, level, K.rlk)
    mods = P.q[:level]
    s_ntt = oracle.to_ntt(K.s, mods, P.log_n)
    s2 = oracle.mul_mod(s_ntt, s_ntt, mods)
    v = oracle.add_mod(u0, oracle.mul_mod(u1, s_ntt, mods), mods)
    v = oracle.add_mod(v, oracle.neg_mod(oracle.mul_mod(d, s2, mods), mods), mods)
    err = oracle.crt_centered(oracle.intt(v, mods, P.log_n), mods)
    bound = sum(len(dg) * math.prod(P.q[i] for i in dg) / 2 for dg in P.digits(level)) * 6 * 3.2 * math.sqrt(P.n) / P.P
    bound += (-(-P.alpha // 2) + 0.5) * 65
    assert max(abs(x) for x in err) <= bound
    assert max(abs(x) for x in err) > 0


def _check_hmult(K, scale, level, tol=2.0 ** -12):
    P = K.P
    st = synth.stream(0, "msg")
    u, v = st.complex_slots(P.n // 2), st.complex_slots(P.n // 2)
    ca, cb = K.encrypt(u, scale, level, "a"), K.encrypt(v, scale, level, "b")
    out = oracle.hmult(P, ca, cb, K.rlk, level)
    got = oracle.decrypt(P, out, K.s, scale * scale)
    err = np.max(np.abs(got - u * v))
    assert err <= tol, err
    if level >= 2:
        rs = oracle.rescale(P, out, level)
        got = oracle.decrypt(P, rs, K.s, scale * scale / P.q[level - 1])
        err = np.max(np.abs(got - u * v))
        assert err <= tol, err
    return out


def test_hmult_decrypts(keys_small, keys_mid):
    _check_hmult(keys_small, 2.0 ** 28, 3)
    _check_hmult(keys_mid, 2.0 ** 30, 7)
    _check_hmult(keys_mid, 2.0 ** 30, 5)


def test_hrot_decrypts_and_hoisted_matches_plain(keys_small, keys_mid):
    for K, scale, level in ((keys_small, 2.0 ** 28, 3), (keys_mid, 2.0 ** 30, 6)):
        P = K.P
        u = synth.stream(0, "msg/rot").complex_slots(P.n // 2)
        ct = K.encrypt(u, scale, level, "rot")
        ks = sorted(K.rot)
        outs = []
        for k in ks:
            g = oracle.galois_element(k, P.log_n)
            out = oracle.hrot(P, ct, level, g, K.rot[k])
            got = oracle.decrypt(P, out, K.s, scale)
            assert np.max(np.abs(got - np.roll(u, -k))) <= 2.0 ** -12
            outs.append(out)
        hoisted = oracle.hrot_hoisted(P, ct, level, [oracle.galois_element(k, P.log_n) for k in ks],
                                      [K.rot[k] for k in ks])
        for i in range(len(ks)):
            assert np.array_equal(hoisted[i], outs[i])


@pytest.mark.slow
def test_hmult_decrypts_full_size(params_full):
    """N=2^16, 24 ciphertext primes, 8 special primes, dnum 3, scale 2^30."""
    K = Keys(params_full, 0)
    _check_hmult(K, 2.0 ** 30, 24)


def test_elementwise_mechanisms_decrypt(keys_small, keys_mid):
    """HAdd, PAdd and PMult (then rescale) decrypt to u + v, u + v and u * v
    within 2^-12 of the fp64 plaintext results (Sec. 2.1)."""
    for K, scale, level in ((keys_small, 2.0 ** 28, 3), (keys_mid, 2.0 ** 30, 7)):
        P = K.P
        st = synth.stream(0, "msg/ew")
        u, v = st.complex_slots(P.n // 2), st.complex_slots(P.n // 2)
        cu, cv = K.encrypt(u, scale, level, "ew/u"), K.encrypt(v, scale, level, "ew/v")
        got = oracle.decrypt(P, oracle.hadd(P, cu, cv, level), K.s, scale)
        assert np.max(np.abs(got - (u + v))) <= 2.0 ** -12
        pt = oracle.to_ntt(oracle.encode(v, P.log_n, scale), P.q[:level], P.log_n)
        got = oracle.decrypt(P, oracle.padd(P, cu, pt, level), K.s, scale)
        assert np.max(np.abs(got - (u + v))) <= 2.0 ** -12
        pm = oracle.pmult(P, cu, pt, level)
        got = oracle.decrypt(P, oracle.rescale(P, pm, level), K.s, scale * scale / P.q[level - 1])
        assert np.max(np.abs(got - u * v)) <= 2.0 ** -12
        # exact algebra: HAdd with the negation is the zero ciphertext; PMult by 1 is the identity
        neg = np.stack([oracle.neg_mod(cu[h], P.q[:level]) for h in range(2)])
        assert not np.any(oracle.hadd(P, cu, neg, level))
        one = np.ones((level, P.n), dtype=np.uint32)
        assert np.array_equal(oracle.pmult(P, cu, one, level), cu)


def test_hconj_decrypts_and_is_an_involution_of_slots(params_small, params_mid):
    """decrypt(HConj(Enc(u))) = conj(u) within 2^-12; the Galois element
    2N-1 conjugates every slot of the canonical embedding."""
    for P, scale, level in ((params_small, 2.0 ** 28, 3), (params_mid, 2.0 ** 30, 6)):
        K = Keys(P, 0, conj=True)
        u = synth.stream(0, "msg/conj").complex_slots(P.n // 2)
        ct = K.encrypt(u, scale, level, "conj")
        got = oracle.decrypt(P, oracle.hconj(P, ct, level, K.conj), K.s, scale)
        assert np.max(np.abs(got - np.conj(u))) <= 2.0 ** -12
        m = oracle.encode(u, P.log_n, scale)
        mc = oracle.automorph_coef(oracle.reduce_signed(m.astype(np.int64), P.q[:1], P.log_n), P.q[:1], P.log_n,
                                   oracle.conj_galois(P.log_n))
        dec = oracle.decode(np.array([float(x) for x in oracle.crt_centered(mc, P.q[:1])]), P.log_n, scale)
        assert np.max(np.abs(dec - np.conj(u))) <= 2.0 ** -20


def test_hrot_sum_hoisted_pins(keys_small, keys_mid):
    """Sum of plaintext-weighted rotations with one ModUp and one ModDown
    (Eq. 5): one rotation weighted by 1 is HRot exactly; a rotation weighted
    by 0 adds nothing; the result decrypts (after rescale) to
    sum_i v_i * (u << k_i) within 2^-12."""
    for K, scale, level in ((keys_small, 2.0 ** 28, 3), (keys_mid, 2.0 ** 30, 6)):
        P = K.P
        mods = P.q + P.p
        ks = sorted(K.rot)
        gs = [oracle.galois_element(k, P.log_n) for k in ks]
        u = synth.stream(0, "msg/lt").complex_slots(P.n // 2)
        ct = K.encrypt(u, scale, level, "lt")
        ones = np.ones((len(mods), P.n), dtype=np.uint32)
        zeros = np.zeros_like(ones)
        one = oracle.hrot_sum_hoisted(P, ct, level, gs[:1], [K.rot[ks[0]]], [ones])
        assert np.array_equal(one, oracle.hrot(P, ct, level, gs[0], K.rot[ks[0]]))
        two = oracle.hrot_sum_hoisted(P, ct, level, gs[:2], [K.rot[ks[0]], K.rot[ks[1]]], [ones, zeros])
        assert np.array_equal(two, one)
        vs = [synth.stream(0, "msg/lt/v%d" % i).complex_slots(P.n // 2) for i in range(len(ks))]
        pts = [oracle.to_ntt(oracle.encode(v, P.log_n, scale), mods, P.log_n) for v in vs]
        out = oracle.hrot_sum_hoisted(P, ct, level, gs, [K.rot[k] for k in ks], pts)
        got = oracle.decrypt(P, oracle.rescale(P, out, level), K.s, scale * scale / P.q[level - 1])
        want = sum(v * np.roll(u, -k) for v, k in zip(vs, ks))
        assert np.max(np.abs(got - want)) <= 2.0 ** -12
