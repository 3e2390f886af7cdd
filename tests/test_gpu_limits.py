"""GPU parity at the library's largest parameter set: 64 primes (48
ciphertext primes of 30 bits, 16 special primes of 31 bits, digit width 16),
where every base conversion accumulates 16 products and takes the lazy
range fixes of Sec. 4.2 inside the accumulation (after 8 products, then
every 4); degenerate levels (1 and 2) and a ragged top digit; parameter sets
beyond the limits are refused."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402

LOG_N, N_Q, N_P = 12, 48, 16
_want = {}  # oracle results shared by the tests (the oracle's transforms are O(N^2) per limb)


def oracle_hmult(P, a, b, key, level, rescale):
    k = ("hmult", level, rescale)
    if k not in _want:
        h = oracle.hmult(P, a, b, key, level)
        _want[k] = oracle.rescale(P, h, level) if rescale else h
    return _want[k]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()
    q = oracle.prime_chain(30, LOG_N, N_Q)
    p = oracle.prime_chain(31, LOG_N, N_P)
    P = oracle.Params(LOG_N, q, p)
    C = ck.Context(LOG_N, q, p)
    st = synth.stream(51, "gpu/limits")
    mods = q + p
    a = np.stack([st.residues(q, P.n), st.residues(q, P.n)])
    b = np.stack([st.residues(q, P.n), st.residues(q, P.n)])
    key = np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
    yield P, C, a, b, key
    C.close()


def test_parameters_at_the_limit(big):
    P, C, a, b, key = big
    assert P.dnum == 3 and P.alpha == 16
    # the ModDown inputs are lifted 31-bit residues: 16 products reach 2^64 without the range fixes
    assert max(P.p) > 1 << 30


@pytest.mark.parametrize("level", [N_Q, 17, 2])
def test_hmult_rescale_at_64_primes(big, level):
    P, C, a, b, key = big
    say("hmult_rescale 64 primes level", level)
    out = torch.zeros((2, level - 1, P.n), dtype=torch.int32, device="cuda")
    C.hmult_rescale(ck.to_device(a), ck.to_device(b), ck.to_device(key), level, out)
    torch.cuda.synchronize()
    assert np.array_equal(ck.to_host(out), oracle_hmult(P, a, b, key, level, True))


@pytest.mark.parametrize("level", [N_Q, 1])
def test_hrot_and_hmult_at_64_primes(big, level):
    P, C, a, b, key = big
    say("hrot / hmult 64 primes level", level)
    out = torch.zeros((2, level, P.n), dtype=torch.int32, device="cuda")
    C.hrot(ck.to_device(a), level, 7, ck.to_device(key), out)
    torch.cuda.synchronize()
    assert np.array_equal(ck.to_host(out), oracle.hrot(P, a, level, oracle.galois_element(7, LOG_N), key))
    C.hmult(ck.to_device(a), ck.to_device(b), ck.to_device(key), level, out)
    torch.cuda.synchronize()
    assert np.array_equal(ck.to_host(out), oracle_hmult(P, a, b, key, level, False))


def test_batch_at_the_limit():
    """Batched launches need each level's ModUp conversion in one launch
    (at most 128 target rows): at 64 primes the top level has 144 and the
    call is refused; 48 primes with digit width 16 (64 target rows) run
    batched, bit-exact per item."""
    ck.lib()
    q = oracle.prime_chain(30, LOG_N, N_Q)
    p = oracle.prime_chain(31, LOG_N, N_P)
    st = synth.stream(52, "gpu/limits/batch")
    for nq, refused in ((N_Q, True), (32, False)):
        P = oracle.Params(LOG_N, q[:nq], p)
        C = ck.Context(LOG_N, q[:nq], p)
        mods = P.q + P.p
        a = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
        b = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
        key = np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
        levels = [nq, 2, 17]
        n = len(levels)
        A = ck.to_device(np.stack([a] * n))
        B = ck.to_device(np.stack([b] * n))
        out = torch.zeros((n, 2, nq - 1, P.n), dtype=torch.int32, device="cuda")
        say("batch", nq, "+", N_P, "primes", levels)
        if refused:
            with pytest.raises(ck.CkksError):
                C.hmult_rescale_batch(A, B, C.batch_items(levels), nq, ck.to_device(key), out)
        else:
            C.hmult_rescale_batch(A, B, C.batch_items(levels), nq, ck.to_device(key), out)
            torch.cuda.synchronize()
            got = ck.to_host(out)
            for i, lv in enumerate(levels):
                want = oracle.rescale(P, oracle.hmult(P, a, b, key, lv), lv)
                assert np.array_equal(got[i, :, :lv - 1], want), lv
        C.close()


def test_limits_are_refused():
    ck.lib()
    q = oracle.prime_chain(30, LOG_N, 49)
    p = oracle.prime_chain(31, LOG_N, 17)
    with pytest.raises(ck.CkksError):
        ck.Context(LOG_N, q[:49], p[:16])   # 65 primes
    with pytest.raises(ck.CkksError):
        ck.Context(LOG_N, q[:8], p[:17])    # 17 special primes
    with pytest.raises(ck.CkksError):
        ck.Context(11, q[:3], p[:1])        # ring degree below 2^12
