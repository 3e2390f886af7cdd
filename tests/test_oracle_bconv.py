"""Pins for BConv (Eq. 2), ModUp and ModDown (Sec. 2.3) against exact CRT
arithmetic in Python integers."""
import math

import numpy as np
import pytest

import oracle
import synth


def crt_centered_col(res, mods):
    """Centred CRT value of one coefficient (Python ints; textbook CRT)."""
    M = math.prod(mods)
    x = 0
    for r, m in zip(res, mods):
        mh = M // m
        x += int(r) * mh * pow(mh % m, -1, m)
    x %= M
    return x - M if 2 * x > M else x


def test_bconv_single_prime_is_centred_reduction():
    """|S| = 1: BConv is the textbook reduction of the centred representative."""
    s = oracle.prime_chain(28, 10, 1)
    t = oracle.prime_chain(31, 10, 3)
    x = synth.stream(4, "bconv/one").residues(s, 1 << 10)
    out = oracle.bconv(x, s, t, 10)
    cent = np.where(2 * x[0].astype(np.int64) < s[0], x[0].astype(np.int64), x[0].astype(np.int64) - s[0])
    for i, m in enumerate(t):
        assert np.array_equal(out[i], (cent % m).astype(np.uint32))


@pytest.mark.parametrize("n_in,n_out", [(3, 4), (8, 5)])
def test_bconv_is_crt_plus_small_multiple(n_in, n_out):
    """out_t = X + u*S (mod t) for one integer u per coefficient with
    |u| <= ceil(|S|/2), X the centred CRT value of the input: an
    approximate CRT whose overflow is a small multiple of S."""
    log_n = 9
    primes = oracle.prime_chain(30, log_n, n_in + n_out)
    s, t = primes[:n_in], primes[n_in:]
    x = synth.stream(5, "bconv/crt/%d" % n_in).residues(s, 1 << log_n)
    out = oracle.bconv(x, s, t, log_n)
    S = math.prod(s)
    umax = -(-n_in // 2)
    seen_neg = seen_pos = False
    for c in range(1 << log_n):
        X = crt_centered_col(x[:, c], s)
        us = [u for u in range(-n_in, n_in + 1)
              if all(int(out[i, c]) == (X + u * S) % m for i, m in enumerate(t))]
        assert len(us) == 1 and abs(us[0]) <= umax, (c, us)
        seen_neg |= us[0] < 0
        seen_pos |= us[0] > 0
    assert seen_neg and seen_pos  # the centred lift makes the overflow two-sided


def test_bconv_is_odd():
    """Centred lift makes BConv odd: BConv(-x) = -BConv(x)."""
    log_n = 8
    primes = oracle.prime_chain(30, log_n, 6)
    s, t = primes[:3], primes[3:]
    x = synth.stream(6, "bconv/odd").residues(s, 1 << log_n)
    a = oracle.bconv(x, s, t, log_n)
    b = oracle.bconv(oracle.neg_mod(x, s), s, t, log_n)
    assert np.array_equal(b, oracle.neg_mod(a, t))


def test_moddown_of_p_multiple_is_exact(params_mid):
    """ModDown(P * x) = x: the P-rows are zero, so the conversion term vanishes."""
    P = params_mid
    for level in (P.n_q, 4, 1):
        x = synth.stream(7, "moddown/exact/%d" % level).residues(P.q[:level], P.n)
        y = np.zeros((level + P.alpha, P.n), dtype=np.uint32)
        for i in range(level):
            y[i] = (x[i].astype(np.uint64) * (P.P % P.q[i]) % P.q[i]).astype(np.uint32)
        assert np.array_equal(oracle.moddown(P, y, level), x)


def test_moddown_is_approximate_division_by_p(params_mid):
    """ModDown(Y) = (Y - [Y]_P)/P - u exactly, [Y]_P the centred residue of Y
    mod P and |u| <= ceil(alpha/2): division by P with a small error."""
    P = params_mid
    level = 5
    mods = P.mods_qp(level)
    y = synth.stream(8, "moddown/div").residues(mods, P.n)
    out = oracle.moddown(P, y, level)
    yc = oracle.intt(y, mods, P.log_n)
    oc = oracle.intt(out, P.q[:level], P.log_n)
    Pp = P.P
    Q = math.prod(P.q[:level])
    umax = -(-P.alpha // 2)
    for c in range(0, P.n, 37):
        Y = crt_centered_col(yc[:, c], mods)
        Yp = crt_centered_col(yc[level:, c], P.p)
        base = (Y - Yp) // Pp
        assert (Y - Yp) % Pp == 0
        got = crt_centered_col(oc[:, c], P.q[:level])
        assert any((base - u - got) % Q == 0 for u in range(-umax, umax + 1)), c


def test_modup_keeps_digit_and_extends_by_bconv(params_mid):
    P = params_mid
    level = 7
    d = synth.stream(9, "modup").residues(P.q[:level], P.n)
    for j, dig in enumerate(P.digits(level)):
        up = oracle.modup(P, d, level, j)
        assert up.shape == (level + P.alpha, P.n)
        for i in dig:
            assert np.array_equal(up[i], d[i])
        # every other row is BConv of the digit's coefficients, then NTT
        dig_mods = [P.q[i] for i in dig]
        rows = [i for i in range(level) if i not in dig] + list(range(level, level + P.alpha))
        row_mods = [P.mods_qp(level)[r] for r in rows]
        coef = oracle.intt(d[list(dig)], dig_mods, P.log_n)
        want = oracle.ntt(oracle.bconv(coef, dig_mods, row_mods, P.log_n), row_mods, P.log_n)
        assert np.array_equal(up[rows], want)
        # ... and agrees with the digit's centred CRT value mod every new prime, up to u*D
        up_c = oracle.intt(up, P.mods_qp(level), P.log_n)
        D = math.prod(dig_mods)
        for c in range(0, P.n, 101):
            X = crt_centered_col(up_c[list(dig), c], dig_mods)
            us = [u for u in range(-len(dig), len(dig) + 1)
                  if all(int(up_c[r, c]) == (X + u * D) % m for r, m in zip(rows, row_mods))]
            assert len(us) == 1 and abs(us[0]) <= -(-len(dig) // 2)


@pytest.mark.parametrize("level", [3, 2])
def test_rescale_is_rounded_division(params_small, params_mid, level):
    """Rescale = round(X / q_{l-1}) exactly (centred X; q odd, so no ties)."""
    for P in (params_small, params_mid):
        ct = synth.stream(10, "rescale/%d" % level).residues(P.q[:level], P.n)
        ct = np.stack([ct, ct[::-1].copy() % np.array(P.q[:level], dtype=np.uint32)[:, None]])
        out = oracle.rescale(P, ct, level)
        ql = P.q[level - 1]
        for poly in range(2):
            xc = oracle.intt(ct[poly], P.q[:level], P.log_n)
            oc = oracle.intt(out[poly], P.q[:level - 1], P.log_n)
            Q1 = math.prod(P.q[:level - 1])
            for c in range(0, P.n, 53):
                X = crt_centered_col(xc[:, c], P.q[:level])
                r = (2 * X + ql) // (2 * ql)  # round to nearest
                assert (crt_centered_col(oc[:, c], P.q[:level - 1]) - r) % Q1 == 0
