"""Pins for the oracle's prime generator and root finder (Sec. 2.2 Eq. 3)."""
import os

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def trial_division_prime(n: int) -> bool:
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def test_is_prime_matches_trial_division_small():
    for n in range(0, 5000):
        assert oracle.is_prime(n) == trial_division_prime(n), n


def test_is_prime_matches_trial_division_31bit():
    st = synth.stream(0, "primes/random")
    cands = (st.u64(60) % np.uint64(1 << 31)).astype(np.int64) | 1
    for n in cands.tolist():
        assert oracle.is_prime(n) == trial_division_prime(n), n
    for n in [2147483647, 2147483649, 1073741827, 1073741825, 3215031751]:  # 3215031751: strong pseudoprime to 2,3,5,7
        assert oracle.is_prime(n) == trial_division_prime(n), n


def test_paper_single_prime_below_2p20():
    """Sec. 3.1: for N=2^16 only one prime below 2^20 is 1 mod 2N."""
    fields = {}
    for line in open(os.path.join(GOLDEN, "ntt_prime_below_2p20.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            fields[k] = int(v)
    step = 2 << fields["log_n"]
    found = oracle.primes_below(fields["bound"], step)
    assert len(found) == fields["count"]
    brute = [c for c in range(step + 1, fields["bound"], step) if trial_division_prime(c)]
    assert found == brute == [786433]


def test_prime_chain_is_the_largest_descending():
    for bits, log_n, count in [(28, 12, 3), (30, 12, 1), (30, 16, 24), (31, 16, 8), (30, 13, 7)]:
        chain = oracle.prime_chain(bits, log_n, count)
        step = 2 << log_n
        assert chain == sorted(chain, reverse=True)
        assert all(c < (1 << bits) and c % step == 1 for c in chain)
        assert all(trial_division_prime(c) for c in chain)
        # no skipped candidate: every 1-mod-2N number between 2^bits and the last
        # chain member that is not in the chain is composite
        c = ((1 << bits) - 2) // step * step + 1
        while c >= chain[-1]:
            assert (c in chain) == trial_division_prime(c), c
            c -= step


def test_psi_is_smallest_2n_th_root_of_minus_one():
    for q, log_n in [(97, 3), (257, 7), (7681, 8), (268369921, 12), (1073479681, 16), (2147352577, 16)]:
        n = 1 << log_n
        psi = oracle.find_psi(q, log_n)
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1
        assert all(pow(g, n, q) != q - 1 for g in range(2, psi))
