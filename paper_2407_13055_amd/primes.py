"""RNS prime construction for the 25-30 prime system (Sec. 3.2, Table 2):
fixed lists of terminal primes tau_i (about 25 bits) and main primes q_i
(30 bits), and the levels' prime windows in the inverted-terminal order
(Sec. 3.3).  Host-side utility: the context takes the window list
[tau_{T-1}..tau_0, q_0..q_{M-1}] as its ciphertext primes and every level is
a contiguous run of prime ids in it."""
from __future__ import annotations

import itertools
import math
from functools import lru_cache

# (terminal primes, main primes) per level of the exemplar construction:
# levels 0-4 follow the 2^40 rescaling cycle, 5-8 are bootstrapping levels
# with double rescaling at 2^55
LEVELS = ((2, 0), (0, 3), (4, 1), (2, 4), (0, 7), (1, 8), (2, 9), (3, 10), (4, 11))
SCALES = (40, 40, 40, 40, 55, 55, 55, 55)


def _is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (bases 2..41)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _below(bits: int, log_n: int, count: int) -> list:
    step = 2 << log_n
    c, out = ((1 << bits) - 2) // step * step + 1, []
    while len(out) < count:
        if _is_prime(c):
            out.append(c)
        c -= step
    return out


def _near(bits: int, log_n: int, count: int) -> list:
    step, c = 2 << log_n, 1 << bits
    lo, hi, out = (c // step) * step + 1, (c // step + 1) * step + 1, []
    while len(out) < count:
        for cand in (lo, hi):
            if _is_prime(cand):
                out.append(cand)
        lo, hi = lo - step, hi + step
    return sorted(out[:count], key=lambda p: abs(math.log2(p) - bits))


def window(taus, qs, level: int, levels=LEVELS) -> list:
    """Primes of `level` in the inverted-terminal order [tau_{t-1}..tau_0, q_0..q_{m-1}]."""
    t, m = levels[level]
    return list(taus[:t][::-1]) + list(qs[:m])


@lru_cache(maxsize=None)
def prime_system_25_30(log_n: int, levels=LEVELS, scales=SCALES, tau_bits: int = 25, q_bits: int = 30):
    """(taus, qs): the main primes are the largest NTT-friendly primes below
    2^q_bits; the terminal primes are the NTT-friendly primes near 2^tau_bits
    (either side) whose order keeps every ratio Q_l / Q_{l-1} closest to its
    scale."""
    n_tau = max(t for t, _ in levels)
    qs = _below(q_bits, log_n, max(m for _, m in levels))
    best, best_err = None, None
    for taus in itertools.permutations(_near(tau_bits, log_n, n_tau + 8), n_tau):
        lq = [sum(math.log2(p) for p in window(taus, qs, lv, levels)) for lv in range(len(levels))]
        err = max(abs(lq[lv] - lq[lv - 1] - scales[lv - 1]) for lv in range(1, len(levels)))
        if best_err is None or err < best_err:
            best, best_err = taus, err
    return tuple(best), tuple(qs)


def context_primes(log_n: int):
    """Ciphertext prime list of a context for the 25-30 system and the level
    windows as prime ids into it."""
    taus, qs = prime_system_25_30(log_n)
    full = list(taus[::-1]) + list(qs)
    return full, [[full.index(p) for p in window(taus, qs, lv)] for lv in range(len(LEVELS))]
