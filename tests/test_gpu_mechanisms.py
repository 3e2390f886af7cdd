"""GPU parity of the element-wise mechanisms (HAdd, PAdd, PMult) and of
HConj against the oracle, bit-exact, out of place and in place, at the top
level and below it; argument errors."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()


_ctx = {}


def ctx_for(P):
    key = (P.log_n, tuple(P.q), tuple(P.p))
    if key not in _ctx:
        _ctx[key] = ck.Context(P.log_n, P.q, P.p)
    return _ctx[key]


def operands(P, name):
    st = synth.stream(41, name)
    a = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    b = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    pt = st.residues(P.q, P.n)
    return a, b, pt


@pytest.mark.parametrize("which", ["small", "mid", "full"])
def test_elementwise_match_oracle(which, params_small, params_mid, params_full):
    P = {"small": params_small, "mid": params_mid, "full": params_full}[which]
    C = ctx_for(P)
    a, b, pt = operands(P, "gpu/ew/" + which)
    da, db, dp = ck.to_device(a), ck.to_device(b), ck.to_device(pt)
    for level in (P.n_q, max(1, P.n_q - 2)):
        say("elementwise", which, "level", level)
        for name, fn, want in (("hadd", C.hadd, oracle.hadd(P, a, b, level)),
                               ("padd", C.padd, oracle.padd(P, a, pt, level)),
                               ("pmult", C.pmult, oracle.pmult(P, a, pt, level))):
            out = torch.zeros((2, level, P.n), dtype=torch.int32, device="cuda")
            fn(da, db if name == "hadd" else dp, level, out)
            torch.cuda.synchronize()
            assert np.array_equal(ck.to_host(out), want), (name, level)
    # in place (operand at the operation level)
    L = P.n_q
    x = da.clone()
    C.hadd(x, db, L, x)
    C.pmult(x, dp, L, x)
    C.padd(x, dp, L, x)
    torch.cuda.synchronize()
    want = oracle.padd(P, oracle.pmult(P, oracle.hadd(P, a, b, L), pt, L), pt, L)
    assert np.array_equal(ck.to_host(x), want)
    y = db.clone()
    C.hadd(da, y, L, y)  # in place on the second operand
    torch.cuda.synchronize()
    assert np.array_equal(ck.to_host(y), oracle.hadd(P, a, b, L))


@pytest.mark.parametrize("which", ["small", "mid"])
def test_hconj_matches_oracle(which, params_small, params_mid):
    P = params_small if which == "small" else params_mid
    C = ctx_for(P)
    st = synth.stream(42, "gpu/conj/" + which)
    ct = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    mods = P.q + P.p
    key = np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
    for level in (P.n_q, max(1, P.n_q - 2)):
        say("hconj", which, "level", level)
        out = torch.zeros((2, level, P.n), dtype=torch.int32, device="cuda")
        C.hconj(ck.to_device(ct), level, ck.to_device(key), out)
        torch.cuda.synchronize()
        assert np.array_equal(ck.to_host(out), oracle.hconj(P, ct, level, key))


def test_hconj_of_an_encryption_decrypts_to_the_conjugate(params_small):
    """The GPU result, decrypted by the oracle, is conj(u) within 2^-12."""
    from helpers import Keys
    P = params_small
    C = ctx_for(P)
    K = Keys(P, 0, conj=True)
    u = synth.stream(0, "msg/gpu/conj").complex_slots(P.n // 2)
    ct = K.encrypt(u, 2.0 ** 28, P.n_q, "gpu/conj")
    out = torch.zeros((2, P.n_q, P.n), dtype=torch.int32, device="cuda")
    C.hconj(ck.to_device(ct), P.n_q, ck.to_device(K.conj), out)
    torch.cuda.synchronize()
    got = oracle.decrypt(P, ck.to_host(out), K.s, 2.0 ** 28)
    assert np.max(np.abs(got - np.conj(u))) <= 2.0 ** -12


def test_elementwise_argument_errors(params_small):
    P = params_small
    C = ctx_for(P)
    a, b, pt = operands(P, "gpu/ew/err")
    da, db, dp = ck.to_device(a), ck.to_device(b), ck.to_device(pt)
    L = P.n_q
    out = torch.zeros((2, L, P.n), dtype=torch.int32, device="cuda")
    with pytest.raises(ck.CkksError):
        C.hadd(da, db, L + 1, out)                  # level above the operands
    with pytest.raises(ck.CkksError):
        C.padd(da, dp[:1], L, out)                  # plaintext with too few limbs
    flat = torch.zeros(2 * L * P.n + P.n, dtype=torch.int32, device="cuda")
    x = flat[:2 * L * P.n].view(2, L, P.n)
    x.copy_(da)
    with pytest.raises(ck.CkksError):
        C.hadd(x, db, L, flat[P.n:].view(2, L, P.n))  # out overlaps an input, shifted by one limb
    with pytest.raises(ck.CkksError):
        C.pmult(da, dp, L - 1, da)                  # in place below the operand's level
