"""CPU oracle for the 32-bit RNS-CKKS key-switching path of Cheddar (arXiv 2407.13055).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does and
shares no code with it.

The ring arithmetic (NTT, BConv, ModUp, KeyMult, ModDown, rescale, HMult,
HRot, automorphism) lives in plain C (``ckks_oracle.c``, exact uint64
arithmetic); this module wraps it with numpy arrays and adds the host-only
pieces of CKKS that the GPU never runs: key generation, encoding (canonical
embedding, Sec. 2.1), encryption (Eq. 1, secret-key form) and decryption with
an exact CRT in Python integers.

Random draws (secret, errors, uniform masks, messages) are inputs: the caller
takes them from the seeded generator in ``synth`` and passes them in.

Parity pins (what fixes each function independently of itself) are in
``tests/test_oracle_*.py``; functions without one are marked there.
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libckks_oracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "libckks_oracle_omp.so")
MAX_PRIMES = 64


class _CParams(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int32), ("n_q", ctypes.c_int32), ("n_p", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mod", ctypes.c_uint64 * MAX_PRIMES)]


_lib = None
_lib_path = _LIB_PATH


def use_threads(n: int) -> int:
    """Timing only (the benchmark's CPU baseline): n > 1 switches to the
    -fopenmp build of the same C source, whose limb loops run on n host
    threads; n <= 1 returns to the one-thread checker.  Results are the same
    (limbs are independent).  Returns the threads in effect."""
    global _lib, _lib_path
    want = _LIB_OMP_PATH if n > 1 else _LIB_PATH
    if want != _lib_path:
        _lib, _lib_path = None, want
    return int(lib().orc_set_threads(max(int(n), 1)))


def lib():
    """Load (building first if absent) the oracle's C library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_lib_path)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        P = ctypes.POINTER(_CParams)
        i = ctypes.c_int
        sig = {
            "orc_is_prime": ([ctypes.c_uint64], i),
            "orc_prime_chain": ([i, i, i, u64p], i),
            "orc_primes_below": ([ctypes.c_uint64, ctypes.c_uint64, u64p, i], i),
            "orc_find_psi": ([ctypes.c_uint64, i], ctypes.c_uint64),
            "orc_ntt": ([u32p, u64p, i, i], None),
            "orc_intt": ([u32p, u64p, i, i], None),
            "orc_bconv": ([u32p, u64p, i, u32p, u64p, i, i], None),
            "orc_modup": ([P, u32p, i, i, u32p], None),
            "orc_moddown": ([P, u32p, i, u32p], None),
            "orc_keyswitch": ([P, u32p, i, u32p, u32p, u32p], None),
            "orc_rescale": ([P, u32p, i, u32p], None),
            "orc_hmult": ([P, u32p, i, u32p, i, u32p, i, u32p], None),
            "orc_automorph_ntt": ([u32p, u32p, i, i, ctypes.c_uint64], None),
            "orc_automorph_coef": ([u32p, u32p, u64p, i, i, ctypes.c_uint64], None),
            "orc_hrot": ([P, u32p, i, i, ctypes.c_uint64, u32p, u32p], None),
            "orc_hrot_hoisted": ([P, u32p, i, i, i, u64p, ctypes.c_void_p, u32p], None),
            "orc_hrot_sum_hoisted": ([P, u32p, i, i, i, u64p, ctypes.c_void_p, ctypes.c_void_p, u32p], None),
            "orc_reduce_signed": ([i64p, u64p, i, i, u32p], None),
            "orc_set_threads": ([i], i),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


# --------------------------------------------------------------------------
# parameters and primes
# --------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(int(n)))


def prime_chain(bits: int, log_n: int, count: int) -> list[int]:
    """The `count` largest primes below 2^bits that are 1 mod 2N, descending
    (NTT-friendly condition, Sec. 2.2 Eq. 3)."""
    out = np.zeros(count, dtype=np.uint64)
    got = lib().orc_prime_chain(bits, log_n, count, out)
    if got != count:
        raise ValueError("only %d such primes below 2^%d" % (got, bits))
    return [int(x) for x in out]


def primes_below(bound: int, step: int, max_out: int = 1 << 16) -> list[int]:
    out = np.zeros(max_out, dtype=np.uint64)
    total = lib().orc_primes_below(bound, step, out, max_out)
    return [int(x) for x in out[:min(total, max_out)]]


def find_psi(q: int, log_n: int) -> int:
    return int(lib().orc_find_psi(q, log_n))


@dataclass
class Params:
    """RNS-CKKS parameters: ring degree 2^log_n, ciphertext primes q, special
    primes p (their number alpha is also the key-switching digit width)."""
    log_n: int
    q: list
    p: list
    c: _CParams = field(init=False, repr=False)

    def __post_init__(self):
        self.q = [int(x) for x in self.q]
        self.p = [int(x) for x in self.p]
        self.c = _CParams()
        self.c.log_n, self.c.n_q, self.c.n_p = self.log_n, len(self.q), len(self.p)
        for i, m in enumerate(self.q + self.p):
            self.c.mod[i] = m

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def n_q(self) -> int:
        return len(self.q)

    @property
    def alpha(self) -> int:
        return len(self.p)

    @property
    def dnum(self) -> int:
        return -(-self.n_q // self.alpha)

    def digits(self, level: int) -> list[range]:
        a = self.alpha
        return [range(j * a, min((j + 1) * a, level)) for j in range(-(-level // a))]

    def mods_qp(self, level: int) -> list[int]:
        """Moduli of the rows q_0..q_{level-1}, p_0..p_{alpha-1}."""
        return self.q[:level] + self.p

    def key_rows(self, level: int) -> list[int]:
        """Rows of a top-level key used at `level` (truncation)."""
        return list(range(level)) + [self.n_q + k for k in range(self.alpha)]

    @property
    def P(self) -> int:
        return math.prod(self.p)

    def ptr(self):
        return ctypes.byref(self.c)


def galois_element(k: int, log_n: int) -> int:
    """g = 5^k mod 2N; HRot by k rotates slots left by k (Sec. 2.2 Eq. 4)."""
    n = 1 << log_n
    return pow(5, k % (n // 2), 2 * n)


# --------------------------------------------------------------------------
# ring operations (C)
# --------------------------------------------------------------------------

def ntt(a, mods, log_n: int) -> np.ndarray:
    x = _u32(a).copy()
    lib().orc_ntt(x, _u64(mods), len(mods), log_n)
    return x


def intt(a, mods, log_n: int) -> np.ndarray:
    x = _u32(a).copy()
    lib().orc_intt(x, _u64(mods), len(mods), log_n)
    return x


def bconv(x, in_mods, out_mods, log_n: int) -> np.ndarray:
    """Fast base conversion (Eq. 2, centred lift), coefficient domain."""
    out = np.zeros((len(out_mods), 1 << log_n), dtype=np.uint32)
    lib().orc_bconv(_u32(x), _u64(in_mods), len(in_mods), out, _u64(out_mods), len(out_mods), log_n)
    return out


def modup(P: Params, d, level: int, j: int) -> np.ndarray:
    out = np.zeros((level + P.alpha, P.n), dtype=np.uint32)
    lib().orc_modup(P.ptr(), _u32(d), level, j, out)
    return out


def moddown(P: Params, x, level: int) -> np.ndarray:
    out = np.zeros((level, P.n), dtype=np.uint32)
    lib().orc_moddown(P.ptr(), _u32(x), level, out)
    return out


def keyswitch(P: Params, d, level: int, evk):
    o0 = np.zeros((level, P.n), dtype=np.uint32)
    o1 = np.zeros((level, P.n), dtype=np.uint32)
    lib().orc_keyswitch(P.ptr(), _u32(d), level, _u32(evk), o0, o1)
    return o0, o1


def rescale(P: Params, ct, level: int) -> np.ndarray:
    out = np.zeros((2, level - 1, P.n), dtype=np.uint32)
    lib().orc_rescale(P.ptr(), _u32(ct), level, out)
    return out


def hmult(P: Params, cta, ctb, rlk, level: int) -> np.ndarray:
    cta, ctb = _u32(cta), _u32(ctb)
    out = np.zeros((2, level, P.n), dtype=np.uint32)
    lib().orc_hmult(P.ptr(), cta, cta.shape[1], ctb, ctb.shape[1], _u32(rlk), level, out)
    return out


def automorph_ntt(a, log_n: int, g: int) -> np.ndarray:
    a = _u32(a)
    out = np.zeros_like(a)
    lib().orc_automorph_ntt(a, out, a.shape[0], log_n, g)
    return out


def automorph_coef(a, mods, log_n: int, g: int) -> np.ndarray:
    a = _u32(a)
    out = np.zeros_like(a)
    lib().orc_automorph_coef(a, out, _u64(mods), a.shape[0], log_n, g)
    return out


def hrot(P: Params, ct, level: int, g: int, rk) -> np.ndarray:
    ct = _u32(ct)
    out = np.zeros((2, level, P.n), dtype=np.uint32)
    lib().orc_hrot(P.ptr(), ct, ct.shape[1], level, g, _u32(rk), out)
    return out


def hrot_hoisted(P: Params, ct, level: int, gs, rks) -> np.ndarray:
    ct = _u32(ct)
    rks = [_u32(r) for r in rks]
    ptrs = (ctypes.c_void_p * len(rks))(*[r.ctypes.data for r in rks])
    out = np.zeros((len(gs), 2, level, P.n), dtype=np.uint32)
    lib().orc_hrot_hoisted(P.ptr(), ct, ct.shape[1], level, len(gs), _u64(gs), ptrs, out)
    return out


# --------------------------------------------------------------------------
# element-wise mechanisms (Sec. 2.1: HAdd, PAdd, PMult) and conjugation
# --------------------------------------------------------------------------

def hadd(P: Params, ct1, ct2, level: int) -> np.ndarray:
    """HAdd: the component-wise sum of two ciphertexts at `level` (Sec. 2.1)."""
    mods = P.q[:level]
    return np.stack([add_mod(_u32(ct1)[h, :level], _u32(ct2)[h, :level], mods) for h in range(2)])


def padd(P: Params, ct, pt, level: int) -> np.ndarray:
    """PAdd: (b + m, a) for a plaintext m in the evaluation domain (Sec. 2.1)."""
    ct = _u32(ct)
    return np.stack([add_mod(ct[0, :level], _u32(pt)[:level], P.q[:level]), ct[1, :level].copy()])


def pmult(P: Params, ct, pt, level: int) -> np.ndarray:
    """PMult: (b * m, a * m) slot-wise in the evaluation domain; the scale
    multiplies (Sec. 2.1)."""
    ct = _u32(ct)
    return np.stack([mul_mod(ct[h, :level], _u32(pt)[:level], P.q[:level]) for h in range(2)])


def conj_galois(log_n: int) -> int:
    """Galois element of complex conjugation of the slots: X -> X^(2N-1)."""
    return (2 << log_n) - 1


def hconj(P: Params, ct, level: int, ck) -> np.ndarray:
    """HConj: the automorphism X -> X^(2N-1) followed by key switching with
    the conjugation key (the HRot sequence with another Galois element)."""
    return hrot(P, ct, level, conj_galois(P.log_n), ck)


def hrot_sum_hoisted(P: Params, ct, level: int, gs, rks, pts) -> np.ndarray:
    """sum_r pts[r] * HRot_{g_r}(ct) with one ModUp of a, the plaintext-weighted
    KeyMult results accumulated over Q_l u P and one ModDown (Sec. 5, Par.4/5,
    Eq. 5).  pts[r]: [n_q + n_p][N] evaluation-domain plaintext over all primes."""
    ct = _u32(ct)
    rks = [_u32(r) for r in rks]
    pts = [_u32(p) for p in pts]
    kp = (ctypes.c_void_p * len(rks))(*[r.ctypes.data for r in rks])
    pp = (ctypes.c_void_p * len(pts))(*[p.ctypes.data for p in pts])
    out = np.zeros((2, level, P.n), dtype=np.uint32)
    lib().orc_hrot_sum_hoisted(P.ptr(), ct, ct.shape[1], level, len(gs), _u64(gs), kp, pp, out)
    return out


# --------------------------------------------------------------------------
# 25-30 prime system and rational rescaling (Sec. 3.2, Table 2, Sec. 5.1)
# --------------------------------------------------------------------------

# (number of 25-bit terminal primes, number of 30-bit main primes) per level
# of the exemplar construction (Table 2): levels 0-4 follow the rescaling
# cycle for a 2^40 scale, levels 5-8 are bootstrapping levels (one tau and
# one q per double rescaling, 2^55).
TABLE2_LEVELS = [(2, 0), (0, 3), (4, 1), (2, 4), (0, 7), (1, 8), (2, 9), (3, 10), (4, 11)]


def _ntt_primes_near(center_bits: int, log_n: int, count: int) -> list:
    """The `count` NTT-friendly primes (1 mod 2N) closest to 2^center_bits
    in log scale, from both sides."""
    step, c = 2 << log_n, 1 << center_bits
    lo, hi, out = (c // step) * step + 1, (c // step + 1) * step + 1, []
    while len(out) < count:
        for cand in (lo, hi):
            if is_prime(cand):
                out.append(cand)
        lo, hi = lo - step, hi + step
    return sorted(out[:count], key=lambda p: abs(math.log2(p) - center_bits))


@functools.lru_cache(maxsize=None)
def prime_system_25_30(log_n: int, levels=tuple(TABLE2_LEVELS), tau_bits: int = 25, q_bits: int = 30,
                       targets=(40, 40, 40, 40, 55, 55, 55, 55)):
    """Fixed lists of terminal primes tau_i (about tau_bits) and main primes
    q_i (the largest NTT-friendly primes below 2^q_bits) for `levels`.  The
    terminal primes are chosen among the NTT-friendly primes nearest to
    2^tau_bits (either side) so that every rescaling ratio Q_l / Q_{l-1}
    stays closest to its target scale (Sec. 3.2: within 0.1 bit)."""
    import itertools
    n_tau = max(t for t, _ in levels)
    n_main = max(m for _, m in levels)
    qs = prime_chain(q_bits, log_n, n_main)
    cands = _ntt_primes_near(tau_bits, log_n, n_tau + 8)
    best, best_err = None, None
    for taus in itertools.permutations(cands, n_tau):
        logq = [sum(math.log2(p) for p in level_primes(taus, qs, lv, levels)) for lv in range(len(levels))]
        err = max(abs(logq[lv] - logq[lv - 1] - targets[lv - 1]) for lv in range(1, len(levels)))
        if best_err is None or err < best_err:
            best, best_err = list(taus), err
    return tuple(best), tuple(qs)


def level_primes(taus, qs, level: int, levels=TABLE2_LEVELS) -> list:
    """The primes of a level in the inverted-terminal order
    [tau_{t-1}, ..., tau_0, q_0, ..., q_{m-1}] (Sec. 3.3): every level is a
    contiguous window of the list taus[::-1] + qs."""
    t, m = levels[level]
    return list(taus[:t][::-1]) + list(qs[:m])


def rescale_rational(ct, in_mods, out_mods, log_n: int) -> np.ndarray:
    """Rational rescaling (Sec. 3.2, the sequence of Sec. 5.1): from the
    modulus Q_in to Q_out = Q_in * Q_A / Q_D, where D = primes dropped and
    A = primes added.  Multiply by Q_A (the A residues of the product are 0),
    convert the D residues to every output prime (INTT, BConv with the
    centred lift, NTT), subtract, multiply by Q_D^-1:
      out_o = (Q_A * x_o - conv_o) * Q_D^-1 mod o    (x_o = 0 for o in A).
    ct: [2][len(in_mods)][N] evaluation domain -> [2][len(out_mods)][N]."""
    ct = _u32(ct)
    in_mods, out_mods = [int(m) for m in in_mods], [int(m) for m in out_mods]
    drop = [m for m in in_mods if m not in out_mods]
    add = [m for m in out_mods if m not in in_mods]
    qa, qd = math.prod(add), math.prod(drop)
    dpos = [in_mods.index(m) for m in drop]
    out = np.zeros((2, len(out_mods), 1 << log_n), dtype=np.uint32)
    for h in range(2):
        y = np.stack([(ct[h, i].astype(np.uint64) * (qa % m) % m).astype(np.uint32) for i, m in zip(dpos, drop)])
        conv = ntt(bconv(intt(y, drop, log_n), drop, out_mods, log_n), out_mods, log_n)
        for o, m in enumerate(out_mods):
            x = ct[h, in_mods.index(m)].astype(np.uint64) if m in in_mods else np.zeros(1 << log_n, np.uint64)
            v = (x * (qa % m) + (m - conv[o].astype(np.uint64))) % m
            out[h, o] = (v * pow(qd % m, -1, m) % m).astype(np.uint32)
    return out


# --------------------------------------------------------------------------
# key switching over a window of the prime list (Sec. 3.2: one evk over
# P * Q_max serves every level; Sec. 3.3: each level is a contiguous window)
# --------------------------------------------------------------------------

def window_digits(alpha: int, start: int, length: int) -> list:
    """The key's digits are runs of alpha primes of the full list (the digit
    partition of a key over P * Q_max, Sec. 2.3).  A ciphertext over the
    window [start, start + length) decomposes into the pieces of those runs
    inside the window: (key digit, first prime index, end prime index)."""
    out = []
    for jk in range(start // alpha, (start + length - 1) // alpha + 1):
        out.append((jk, max(jk * alpha, start), min((jk + 1) * alpha, start + length)))
    return out


def _moddown_window(x, win, p, log_n: int) -> np.ndarray:
    """ModDown (Sec. 2.3): x over win + p -> (x_Q - BConv_{P->Q}(x_P)) * P^-1
    over win, conversion in the coefficient domain with the centred lift."""
    k = len(win)
    conv = ntt(bconv(intt(x[k:], p, log_n), p, win, log_n), win, log_n)
    pinv = np.array([pow(math.prod(p) % q, -1, q) for q in win], dtype=np.uint64)
    return mul_mod(add_mod(x[:k], neg_mod(conv, win), win), np.broadcast_to(pinv[:, None], conv.shape), win)


def keymult_window(full, p, start: int, length: int, d, evk, log_n: int):
    """The KeyMult sums of hybrid key switching of d (evaluation domain over
    the window primes full[start:start+length]) with a key over P * Q_max,
    Q_max the product of the whole list `full` (Sec. 3.2): for each key digit
    meeting the window, ModUp of its in-window residues (INTT, BConv to every
    other row of window + P, NTT; its own rows pass unchanged), times that
    digit's key rows for the window primes and P, summed.
    evk: [dnum][2][len(full) + len(p)][N] -> two [length + len(p)][N]."""
    full, p = [int(m) for m in full], [int(m) for m in p]
    win = full[start:start + length]
    mods = win + p
    rows, n = len(mods), 1 << log_n
    key_rows = list(range(start, start + length)) + [len(full) + k for k in range(len(p))]
    d, evk = _u32(d), _u32(evk)
    ks = [np.zeros((rows, n), dtype=np.uint32), np.zeros((rows, n), dtype=np.uint32)]
    for jk, lo, hi in window_digits(len(p), start, length):
        own = list(range(lo - start, hi - start))
        others = [r for r in range(rows) if r not in own]
        dig = full[lo:hi]
        up = np.zeros((rows, n), dtype=np.uint32)
        up[own] = d[own]
        omods = [mods[r] for r in others]
        up[others] = ntt(bconv(intt(d[own], dig, log_n), dig, omods, log_n), omods, log_n)
        for h in range(2):
            ks[h] = add_mod(ks[h], mul_mod(up, evk[jk, h][key_rows], mods), mods)
    return ks[0], ks[1]


def keyswitch_window(full, p, start: int, length: int, d, evk, log_n: int):
    """Key switching over the window: the KeyMult sums, then ModDown of both
    (Sec. 2.3).  Returns two [length][N]."""
    win = [int(m) for m in full[start:start + length]]
    p = [int(m) for m in p]
    ks0, ks1 = keymult_window(full, p, start, length, d, evk, log_n)
    return _moddown_window(ks0, win, p, log_n), _moddown_window(ks1, win, p, log_n)


def hmult_window(full, p, start: int, length: int, cta, ctb, rlk, log_n: int) -> np.ndarray:
    """HMult with relinearisation (Sec. 2.1) of two ciphertexts over the
    window: d0 = b_a b_b, d1 = b_a a_b + a_a b_b, d2 = a_a a_b, then
    (d0, d1) + KeySwitch(d2) with a relinearisation key over P * Q_max."""
    win = [int(m) for m in full[start:start + length]]
    cta, ctb = _u32(cta), _u32(ctb)
    d0 = mul_mod(cta[0], ctb[0], win)
    d1 = add_mod(mul_mod(cta[0], ctb[1], win), mul_mod(cta[1], ctb[0], win), win)
    d2 = mul_mod(cta[1], ctb[1], win)
    u0, u1 = keyswitch_window(full, p, start, length, d2, rlk, log_n)
    return np.stack([add_mod(d0, u0, win), add_mod(d1, u1, win)])


def hmult_rescale_window(full, p, start: int, length: int, out_start: int, out_length: int, cta, ctb, rlk,
                         log_n: int) -> np.ndarray:
    """HMult followed by rescaling to the window below, with ModDown merged
    into the rational rescaling (the MAD-style merge the paper extends to its
    prime system, Sec. 5 and 6): the KeyMult sums plus P * (d0, d1) over
    window + P are rescaled rationally in one step from window + P to the
    output window (dropping P and the window's primes outside the output,
    adding the output's primes outside the window) -- one rounding of
    Q_A * x / (P * Q_D) instead of ModDown's and then rescaling's."""
    full, p = [int(m) for m in full], [int(m) for m in p]
    win = full[start:start + length]
    cta, ctb = _u32(cta), _u32(ctb)
    d0 = mul_mod(cta[0], ctb[0], win)
    d1 = add_mod(mul_mod(cta[0], ctb[1], win), mul_mod(cta[1], ctb[0], win), win)
    d2 = mul_mod(cta[1], ctb[1], win)
    ks0, ks1 = keymult_window(full, p, start, length, d2, rlk, log_n)
    pq = np.array([math.prod(p) % q for q in win], dtype=np.uint64)[:, None]
    x = np.stack([ks0, ks1])
    for h, dh in ((0, d0), (1, d1)):
        x[h, :length] = add_mod(x[h, :length], mul_mod(dh, np.broadcast_to(pq, dh.shape), win), win)
    return rescale_rational(x, win + p, full[out_start:out_start + out_length], log_n)


def hrot_sum_window(full, p, start: int, length: int, ct, gs, rks, pts, log_n: int) -> np.ndarray:
    """Sum of plaintext-weighted rotations over the window (Sec. 5 Par.4/5,
    Eq. 5, in the fused order of hrot_sum_hoisted): for each rotation, the
    KeyMult sums of phi_g(a) times the plaintext's rows (prime ids: the
    window's, then P's), accumulated over window + P; one ModDown; plus
    sum_i pt_i * phi_i(b).  pts[i]: [len(full) + len(p)][N] by prime id."""
    full, p = [int(m) for m in full], [int(m) for m in p]
    win = full[start:start + length]
    mods = win + p
    rows = list(range(start, start + length)) + [len(full) + k for k in range(len(p))]
    ct = _u32(ct)
    acc = [np.zeros((len(mods), 1 << log_n), dtype=np.uint32) for _ in range(2)]
    tail = np.zeros((length, 1 << log_n), dtype=np.uint32)
    for g, rk, pt in zip(gs, rks, pts):
        pt = _u32(pt)[rows]
        ks = keymult_window(full, p, start, length, automorph_ntt(ct[1], log_n, g), rk, log_n)
        for h in range(2):
            acc[h] = add_mod(acc[h], mul_mod(ks[h], pt, mods), mods)
        tail = add_mod(tail, mul_mod(automorph_ntt(ct[0], log_n, g), pt[:length], win), win)
    return np.stack([add_mod(_moddown_window(acc[0], win, p, log_n), tail, win),
                     _moddown_window(acc[1], win, p, log_n)])


def hrot_window(full, p, start: int, length: int, ct, g: int, rk, log_n: int) -> np.ndarray:
    """HRot (Sec. 2.1, Eq. 4) of a ciphertext over the window:
    (phi_g(b), 0) + KeySwitch(phi_g(a)) with a key over P * Q_max."""
    win = [int(m) for m in full[start:start + length]]
    ct = _u32(ct)
    pb, pa = automorph_ntt(ct[0], log_n, g), automorph_ntt(ct[1], log_n, g)
    u0, u1 = keyswitch_window(full, p, start, length, pa, rk, log_n)
    return np.stack([add_mod(pb, u0, win), u1])


def reduce_signed(coef, mods, log_n: int) -> np.ndarray:
    out = np.zeros((len(mods), 1 << log_n), dtype=np.uint32)
    lib().orc_reduce_signed(np.ascontiguousarray(coef, dtype=np.int64), _u64(mods), len(mods), log_n, out)
    return out


# --------------------------------------------------------------------------
# element-wise helpers (numpy; every operand < 2^32, products < 2^64)
# --------------------------------------------------------------------------

def _col(mods) -> np.ndarray:
    return np.asarray(mods, dtype=np.uint64)[:, None]


def mul_mod(a, b, mods) -> np.ndarray:
    m = _col(mods)
    return ((a.astype(np.uint64) % m) * (b.astype(np.uint64) % m) % m).astype(np.uint32)


def add_mod(a, b, mods) -> np.ndarray:
    m = _col(mods)
    return ((a.astype(np.uint64) + b.astype(np.uint64)) % m).astype(np.uint32)


def neg_mod(a, mods) -> np.ndarray:
    m = _col(mods)
    return ((m - a.astype(np.uint64) % m) % m).astype(np.uint32)


# --------------------------------------------------------------------------
# keys, encoding, encryption (host only)
# --------------------------------------------------------------------------

def to_ntt(coef, mods, log_n: int) -> np.ndarray:
    """Signed integer polynomial -> NTT-domain residues [len(mods)][N]."""
    return ntt(reduce_signed(coef, mods, log_n), mods, log_n)


def make_switch_key(P: Params, s_ntt, sp_ntt, a, e) -> np.ndarray:
    """Key switching sp -> s (hybrid, digit width alpha), top level.

    s_ntt, sp_ntt: [n_q+alpha][N] NTT residues of s and s'.
    a: [dnum][n_q+alpha][N] uniform residues (NTT domain).
    e: [dnum][N] integer errors.
    Returns [dnum][2][n_q+alpha][N]:  half 0 = -a*s + e + g_j*s', half 1 = a,
    where the gadget g_j = P * Dhat_j * [Dhat_j^-1]_{D_j} is P on the rows of
    digit j and 0 on every other row (Sec. 2.1 evk over R_PQ, dnum pairs).
    """
    mods = P.q + P.p
    out = np.zeros((P.dnum, 2, len(mods), P.n), dtype=np.uint32)
    for j in range(P.dnum):
        ej = to_ntt(e[j], mods, P.log_n)
        b = add_mod(neg_mod(mul_mod(a[j], s_ntt, mods), mods), ej, mods)
        for i in P.digits(P.n_q)[j]:
            gsp = (sp_ntt[i].astype(np.uint64) * (P.P % P.q[i]) % P.q[i]).astype(np.uint32)
            b[i] = ((b[i].astype(np.uint64) + gsp) % P.q[i]).astype(np.uint32)
        out[j, 0] = b
        out[j, 1] = a[j]
    return out


def relin_key(P: Params, s, a, e) -> np.ndarray:
    """Relinearisation key: switches s^2 -> s."""
    mods = P.q + P.p
    s_ntt = to_ntt(s, mods, P.log_n)
    return make_switch_key(P, s_ntt, mul_mod(s_ntt, s_ntt, mods), a, e)


def rotation_key(P: Params, s, k: int, a, e) -> np.ndarray:
    """Rotation key for HRot by k: switches phi_{5^k}(s) -> s."""
    mods = P.q + P.p
    s_ntt = to_ntt(s, mods, P.log_n)
    return make_switch_key(P, s_ntt, automorph_ntt(s_ntt, P.log_n, galois_element(k, P.log_n)), a, e)


def conj_key(P: Params, s, a, e) -> np.ndarray:
    """Conjugation key: switches phi_{2N-1}(s) -> s."""
    mods = P.q + P.p
    s_ntt = to_ntt(s, mods, P.log_n)
    return make_switch_key(P, s_ntt, automorph_ntt(s_ntt, P.log_n, conj_galois(P.log_n)), a, e)


def _slot_positions(log_n: int):
    """Evaluation index k (root zeta^(2k+1), zeta = exp(i*pi/N)) of slot j and
    of its conjugate: 2k+1 = 5^j mod 2N and 2k+1 = -5^j mod 2N."""
    n = 1 << log_n
    e = np.array([pow(5, j, 2 * n) for j in range(n // 2)], dtype=np.int64)
    return (e - 1) // 2, (2 * n - e - 1) // 2


def encode(z, log_n: int, scale: float) -> np.ndarray:
    """Canonical embedding (Sec. 2.1): the real integer polynomial m with
    m(zeta^(5^j)) ~= scale * z_j, zeta = exp(i pi / N), rounded to nearest.

    m(zeta^(2k+1)) = sum_n (m_n zeta^n) w^(n k), w = exp(2 pi i / N), so the
    vector of values is N * ifft(m * zeta^n); invert it with a forward FFT."""
    n = 1 << log_n
    pos, conj = _slot_positions(log_n)
    v = np.zeros(n, dtype=np.complex128)
    v[pos] = scale * np.asarray(z)
    v[conj] = scale * np.conj(np.asarray(z))
    twist = np.exp(-1j * np.pi * np.arange(n) / n)
    m = np.fft.fft(v) / n * twist
    return np.rint(m.real).astype(np.int64)


def decode(m, log_n: int, scale: float) -> np.ndarray:
    """Inverse of encode: slot j = m(zeta^(5^j)) / scale (m real, float64)."""
    n = 1 << log_n
    pos, _ = _slot_positions(log_n)
    vals = n * np.fft.ifft(np.asarray(m, dtype=np.float64) * np.exp(1j * np.pi * np.arange(n) / n))
    return vals[pos] / scale


def encrypt(P: Params, m, s, level: int, a, e) -> np.ndarray:
    """Secret-key encryption, Eq. 1: (b, a) = (-a s + m + e, a) at `level`.
    m, e: integer coefficient vectors; a: [level][N] uniform NTT residues."""
    mods = P.q[:level]
    s_ntt = to_ntt(s, mods, P.log_n)
    b = add_mod(neg_mod(mul_mod(a, s_ntt, mods), mods), to_ntt(np.asarray(m) + np.asarray(e), mods, P.log_n), mods)
    return np.stack([b, _u32(a)])


def crt_centered(x, mods) -> list:
    """Exact CRT of residue rows x [L][N] to centred Python integers."""
    Q = math.prod(mods)
    acc = np.zeros(x.shape[1], dtype=object)
    for i, q in enumerate(mods):
        qh = Q // q
        c = qh * pow(qh % q, -1, q)
        acc = acc + x[i].astype(np.int64).astype(object) * c
    acc = acc % Q
    return [int(v) - Q if 2 * int(v) > Q else int(v) for v in acc]


def decrypt_coef(P: Params, ct, s) -> list:
    """b + a s, back to coefficients, as centred integers."""
    level = ct.shape[1]
    mods = P.q[:level]
    s_ntt = to_ntt(s, mods, P.log_n)
    v = add_mod(ct[0], mul_mod(ct[1], s_ntt, mods), mods)
    return crt_centered(intt(v, mods, P.log_n), mods)


def decrypt(P: Params, ct, s, scale: float) -> np.ndarray:
    m = decrypt_coef(P, ct, s)
    return decode(np.array([float(v) for v in m]), P.log_n, scale)
