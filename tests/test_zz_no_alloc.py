"""The allocation-free HMult + relinearisation + rescale
(ckks_hmult_rescale_noalloc, workspace = the library's per-GPU scratch
array) against the call that takes a caller workspace (ckks_hmult_rescale),
bit for bit, through the C ABI: two calls in a row on one GPU, the second
with a smaller input, on the headline ring (N = 2^16, 24 + 8 primes, dnum 3)
and on the small ring (N = 2^12, 3 + 1 primes); and the size limit (a level
whose workspace exceeds the array is refused, a lower level of the same
context still runs)."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402

SCRATCH = 64 << 20  # CKKS_NOALLOC_SCRATCH_BYTES


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()


def ct_pair(q, n, level, seed_name):
    st = synth.stream(31, seed_name)
    a = np.stack([st.residues(q[:level], n), st.residues(q[:level], n)])
    b = np.stack([st.residues(q[:level], n), st.residues(q[:level], n)])
    return ck.to_device(a), ck.to_device(b)


def key(q, p, n, dnum, seed_name):
    st = synth.stream(31, seed_name)
    return ck.to_device(np.stack([np.stack([st.residues(q + p, n), st.residues(q + p, n)]) for _ in range(dnum)]))


def both(C, a, b, rlk, level):
    """(allocation-free result, workspace-call result) of one HMult+rescale."""
    lo = C.rescaled_level(level)
    got = torch.full((2, lo, C.n), -1, dtype=torch.int32, device="cuda")
    want = torch.full((2, lo, C.n), -2, dtype=torch.int32, device="cuda")
    C.hmult_rescale_noalloc(a, b, rlk, level, got)
    C.hmult_rescale(a, b, rlk, level, want)
    torch.cuda.synchronize()
    return ck.to_host(got), ck.to_host(want)


@pytest.mark.parametrize("log_n,bits_q,n_q,bits_p,n_p,levels", [
    (16, 30, 24, 31, 8, (24, 9)),
    (12, 28, 3, 30, 1, (3, 2)),
])
def test_noalloc_matches_workspace_call(log_n, bits_q, n_q, bits_p, n_p, levels):
    q, p = ck.prime_chain(bits_q, log_n, n_q), ck.prime_chain(bits_p, log_n, n_p)
    C = ck.Context(log_n, q, p)
    assert C.workspace_size(ck.OP_HMULT, n_q) <= SCRATCH
    rlk = key(q, p, C.n, C.dnum, "rlk/%d" % log_n)
    for i, level in enumerate(levels):  # second call: smaller input (fewer limbs)
        say("noalloc: N=2^%d level %d call %d" % (log_n, level, i))
        a, b = ct_pair(q, C.n, level, "ct/%d/%d" % (log_n, i))
        got, want = both(C, a, b, rlk, level)
        bad = np.argwhere(got != want)
        assert bad.size == 0, "level %d: %d mismatches, first at %s" % (level, len(bad), bad[:4].tolist())
    C.close()


def test_noalloc_small_ring_matches_oracle():
    """The small ring's allocation-free result is also the oracle's."""
    P = oracle.Params(12, oracle.prime_chain(28, 12, 3), oracle.prime_chain(30, 12, 1))
    C = ck.Context(P.log_n, P.q, P.p)
    st = synth.stream(31, "oracle")
    a = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    b = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    rlk = np.stack([np.stack([st.residues(P.q + P.p, P.n), st.residues(P.q + P.p, P.n)]) for _ in range(P.dnum)])
    out = torch.empty((2, P.n_q - 1, P.n), dtype=torch.int32, device="cuda")
    C.hmult_rescale_noalloc(ck.to_device(a), ck.to_device(b), ck.to_device(rlk), P.n_q, out)
    torch.cuda.synchronize()
    want = oracle.rescale(P, oracle.hmult(P, a, b, rlk, P.n_q), P.n_q)
    assert np.array_equal(ck.to_host(out), want)
    C.close()


def test_noalloc_refuses_levels_beyond_the_scratch_array():
    q, p = ck.prime_chain(30, 16, 48), ck.prime_chain(31, 16, 8)
    C = ck.Context(16, q, p)
    top = 48
    assert C.workspace_size(ck.OP_HMULT, top) > SCRATCH
    fits = max(lv for lv in range(2, top + 1) if C.workspace_size(ck.OP_HMULT, lv) <= SCRATCH)
    rlk = key(q, p, C.n, C.dnum, "rlk/big")
    a, b = ct_pair(q, C.n, top, "ct/big")
    out = torch.empty((2, top - 1, C.n), dtype=torch.int32, device="cuda")
    say("noalloc: refusal at level %d (fits up to %d)" % (top, fits))
    with pytest.raises(ck.CkksError, match="workspace"):
        C.hmult_rescale_noalloc(a, b, rlk, top, out)
    # a level that fits still runs, and matches the workspace call
    a2, b2 = ct_pair(q, C.n, fits, "ct/big/fits")
    got, want = both(C, a2, b2, rlk, fits)
    assert np.array_equal(got, want)
    C.close()
