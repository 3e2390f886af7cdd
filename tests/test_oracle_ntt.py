"""Pins for the oracle's negacyclic NTT (Sec. 2.2): the definition evaluated
by brute force on tiny N, the negacyclic convolution theorem against a
schoolbook product, and round trips at full size."""
import numpy as np
import pytest

import oracle
import synth


def brev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def direct_ntt(a, q, log_n, psi):
    """A[k] = a(psi^(2*brev(k)+1)): evaluation at the odd powers of psi,
    stored at bit-reversed positions -- brute force, O(N^2)."""
    n = 1 << log_n
    out = [0] * n
    for k in range(n):
        root = pow(psi, 2 * brev(k, log_n) + 1, q)
        out[k] = sum(int(a[j]) * pow(root, j, q) for j in range(n)) % q
    return out


def schoolbook_negacyclic(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            v = int(a[i]) * int(b[j])
            if i + j < n:
                c[i + j] += v
            else:
                c[i + j - n] -= v
    return [x % q for x in c]


@pytest.mark.parametrize("log_n,bits", [(3, 12), (4, 20), (5, 24), (6, 22)])
def test_ntt_matches_definition(log_n, bits):
    q = oracle.prime_chain(bits, log_n, 1)[0]
    psi = oracle.find_psi(q, log_n)
    a = synth.stream(1, "ntt/def/%d" % log_n).residues([q], 1 << log_n)
    got = oracle.ntt(a, [q], log_n)[0].tolist()
    assert got == direct_ntt(a[0], q, log_n, psi)
    assert oracle.intt(np.array([got], dtype=np.uint32), [q], log_n)[0].tolist() == a[0].tolist()


@pytest.mark.parametrize("log_n,bits", [(6, 22), (8, 24), (9, 28)])
def test_negacyclic_convolution_theorem(log_n, bits):
    q = oracle.prime_chain(bits, log_n, 1)[0]
    st = synth.stream(2, "ntt/conv/%d" % log_n)
    a, b = st.residues([q], 1 << log_n), st.residues([q], 1 << log_n)
    prod = oracle.mul_mod(oracle.ntt(a, [q], log_n), oracle.ntt(b, [q], log_n), [q])
    got = oracle.intt(prod, [q], log_n)[0].tolist()
    assert got == schoolbook_negacyclic(a[0], b[0], q)


def test_round_trip_full_size(params_full, params_small):
    for P in (params_small, params_full):
        mods = [P.q[0], P.p[-1]]
        a = synth.stream(3, "ntt/rt").residues(mods, P.n)
        f = oracle.ntt(a, mods, P.log_n)
        assert not np.array_equal(f, a)
        assert np.array_equal(oracle.intt(f, mods, P.log_n), a)


def test_monomial_maps_to_roots(params_small):
    """NTT(X) holds psi^(2 brev(k)+1) at position k -- the evaluation points themselves."""
    P = params_small
    q = P.q[0]
    x = np.zeros((1, P.n), dtype=np.uint32)
    x[0, 1] = 1
    psi = oracle.find_psi(q, P.log_n)
    got = oracle.ntt(x, [q], P.log_n)[0]
    for k in [0, 1, 2, 3, 100, P.n - 1]:
        assert int(got[k]) == pow(psi, 2 * brev(k, P.log_n) + 1, q)
