"""Host checks of two facts the one-wave-per-row kernels rely on (no GPU).

1. Quotient-only twiddles (KeyMult): a table entry is ws = floor(w 2^32 / q)
   alone, and the kernel takes w = ceil(ws q / 2^32) (mulhi plus a carry
   from the low product).  Checked exhaustively on small primes and on
   random and boundary twiddles of the benchmark's prime chain, with the
   Shoup product x w - floor(x ws / 2^32) q landing in [0, 2q).
2. The quad transpose that replaces the last forward (first inverse)
   row-pass exchange: two exchange stages with the partner lane a^1 / a^2
   (register b^1 / b^2 where lane and register bits differ) turn lane a's
   register b into lane b's register a, and move the points of radix-4
   round 2's layout (16m + a + 4k in lane a of quad m) to radix-4 round 3's
   (16m + 4a + k).
"""
import random

import pytest

import paper_2407_13055_amd as ck


def recover(ws: int, q: int) -> int:
    p = ws * q
    return (p >> 32) + (1 if p & 0xFFFFFFFF else 0)


def shoup(x: int, w: int, ws: int, q: int) -> int:
    return (x * w - ((x * ws) >> 32) * q) % (1 << 32)


@pytest.mark.parametrize("q", [3, 17, 97, 257, 7681, 12289])
def test_quotient_recovers_every_twiddle_of_small_primes(q):
    for w in range(q):
        ws = (w << 32) // q
        assert recover(ws, q) == w


def test_quotient_recovers_twiddles_of_the_benchmark_chain():
    rnd = random.Random(5)
    primes = ck.prime_chain(30, 16, 24) + ck.prime_chain(31, 16, 8)
    for q in primes:
        ws_of = lambda w: (w << 32) // q  # noqa: E731
        ws_set = [0, 1, 2, q - 1, q - 2, q // 2, (q + 1) // 2] + [rnd.randrange(q) for _ in range(2000)]
        for w in ws_set:
            ws = ws_of(w)
            assert recover(ws, q) == w
            for x in (0, 1, q - 1, (1 << 32) - 1, rnd.randrange(1 << 32)):
                t = shoup(x, recover(ws, q), ws, q)
                assert t < 2 * q and t % q == (x * w) % q


def quad_transpose(x):
    """x[lane][reg] for 64 lanes, 4 registers: the kernel's two stages."""
    for bit in (1, 2):
        y = [[x[lane ^ bit][b ^ bit] for b in range(4)] for lane in range(64)]
        x = [[y[lane][b] if ((b ^ lane) & bit) else x[lane][b] for b in range(4)] for lane in range(64)]
    return x


def test_quad_transpose_is_a_transpose_within_each_quad():
    x = [[(lane, b) for b in range(4)] for lane in range(64)]
    out = quad_transpose(x)
    for lane in range(64):
        m, a = lane >> 2, lane & 3
        for b in range(4):
            assert out[lane][b] == (4 * m + b, a)


def test_quad_transpose_moves_round_two_points_to_round_three():
    # forward row pass, 256 points, 4 per lane: round j holds
    # l = blk 2^(sh+2) + (t mod 2^sh) + k 2^sh with sh = 6 - 2j
    def points(t, sh):
        l0 = ((t >> sh) << (sh + 2)) + (t & ((1 << sh) - 1))
        return [l0 + (k << sh) for k in range(4)]

    x = [points(t, 2) for t in range(64)]
    assert quad_transpose(x) == [points(t, 0) for t in range(64)]
    # the inverse pass walks the same units the other way (sh = 0 then 2)
    x = [points(t, 0) for t in range(64)]
    assert quad_transpose(x) == [points(t, 2) for t in range(64)]
