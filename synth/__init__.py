"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-number generation and sampling only -- none of the
CKKS arithmetic.  Both the GPU path and the CPU oracle receive what it draws
as plain inputs (residue arrays, integer coefficient vectors, complex slots).

Generator: SplitMix64 used as a counter-based generator.  Output i of a
stream with key K is mix(K + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64), where
mix is SplitMix64's finaliser (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  A named sub-stream
(e.g. "secret", "rlk", "msg/0/a") gets the key mix(seed XOR FNV-1a-64(name)),
so sub-streams are independent of the order in which they are drawn.

Not cryptographically secure: a parity and benchmark harness, not a
deployment.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _fnv1a64(name: str) -> int:
    h = 0xCBF29CE484222325
    for b in name.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


class Stream:
    """Counter-based SplitMix64 sub-stream."""

    def __init__(self, seed: int, name: str):
        key = np.array([(seed ^ _fnv1a64(name)) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
        self.key = _mix(key)[0]
        self.counter = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.counter + 1, self.counter + 1 + n, dtype=np.uint64)
        self.counter += n
        with np.errstate(over="ignore"):
            return _mix(self.key + idx * _GAMMA)

    def unit(self, n: int) -> np.ndarray:
        """Doubles uniform in (0, 1]."""
        return ((self.u64(n) >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)

    def uniform_mod(self, q: int, n: int) -> np.ndarray:
        """n residues uniform in [0, q) (64-bit draw reduced mod q; bias < 2^-32)."""
        return (self.u64(n) % np.uint64(q)).astype(np.uint32)

    def residues(self, mods, n: int) -> np.ndarray:
        """[len(mods)][n] uint32, limb i uniform in [0, mods[i])."""
        return np.stack([self.uniform_mod(int(q), n) for q in mods]) if len(mods) else np.zeros((0, n), np.uint32)

    def ternary(self, n: int, h: int) -> np.ndarray:
        """int64 vector with exactly h entries in {-1, +1} at uniform positions."""
        pos = np.argsort(self.u64(n), kind="stable")[:h]
        signs = (self.u64(h) & np.uint64(1)).astype(np.int64) * 2 - 1
        s = np.zeros(n, dtype=np.int64)
        s[pos] = signs
        return s

    def gaussian(self, n: int, sigma: float = 3.2, bound: int = 19) -> np.ndarray:
        """Rounded normal(0, sigma^2) integers, redrawn when |e| > bound."""
        out = np.empty(0, dtype=np.int64)
        while out.size < n:
            m = 2 * (n - out.size) + 16
            u1, u2 = self.unit(m), self.unit(m)
            e = np.rint(sigma * np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).astype(np.int64)
            out = np.concatenate([out, e[np.abs(e) <= bound]])
        return out[:n]

    def complex_slots(self, n: int) -> np.ndarray:
        """n complex numbers, real and imaginary parts independently U[-1, 1]."""
        return (2.0 * self.unit(n) - 1.0) + 1j * (2.0 * self.unit(n) - 1.0)

    def integers(self, lo: int, hi: int, n: int) -> np.ndarray:
        """n integers uniform in [lo, hi] (inclusive)."""
        return (self.u64(n) % np.uint64(hi - lo + 1)).astype(np.int64) + lo

    def distinct(self, lo: int, hi: int, n: int) -> np.ndarray:
        """n distinct integers from [lo, hi], drawn without replacement."""
        out: list[int] = []
        while len(out) < n:
            for v in self.integers(lo, hi, n).tolist():
                if v not in out:
                    out.append(v)
                if len(out) == n:
                    break
        return np.array(out, dtype=np.int64)


def stream(seed: int, name: str) -> Stream:
    return Stream(seed, name)


def device_residues(seed: int, name: str, mods, lead: tuple, n: int, torch, device="cuda"):
    """int32 tensor (uint32 bit patterns) of shape (*lead, len(mods), n), limb i
    uniform in [0, mods[i]) (62-bit draw reduced mod q), drawn on the device by
    torch's generator seeded from this sub-stream: for large resident inputs
    (key sets, ciphertext pools) whose host generation would dominate set-up."""
    g = torch.Generator(device=device)
    g.manual_seed(int(stream(seed, name).u64(1)[0] >> np.uint64(1)))
    m = torch.tensor([int(q) for q in mods], dtype=torch.int64, device=device).view(len(mods), 1)
    x = torch.randint(0, 1 << 62, (*lead, len(mods), n), generator=g, device=device, dtype=torch.int64)
    return (x % m).to(torch.int32)
