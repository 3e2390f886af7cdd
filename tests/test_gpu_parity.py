"""GPU parity: every C-ABI call against the CPU oracle, bit for bit, on the
same seeded inputs.  Sizes span several tiles and ragged tails; the full
N=2^16, 24+8-prime configuration is compared in full."""
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


_ctx_cache = {}


def ctx_for(P):
    key = (P.log_n, tuple(P.q), tuple(P.p))
    if key not in _ctx_cache:
        _ctx_cache[key] = ck.Context(P.log_n, P.q, P.p)
    return _ctx_cache[key]


def dev(a):
    return ck.to_device(a)


def host(t):
    return ck.to_host(t)


def empty(*shape):
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def rand_ct(P, level, name):
    st = synth.stream(7, name)
    return np.stack([st.residues(P.q[:level], P.n), st.residues(P.q[:level], P.n)])


def rand_key(P, name):
    st = synth.stream(7, name)
    mods = P.q + P.p
    return np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])


def assert_same(got, want, what):
    assert got.shape == want.shape, what
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d mismatches, first at %s" % (what, len(bad), bad[:4].tolist())


# ----------------------------------------------------------------------------
# NTT / INTT
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_ntt_intt(log_n):
    q = oracle.prime_chain(30, log_n, 3)
    p = oracle.prime_chain(31, log_n, 2)
    P = oracle.Params(log_n, q, p)
    C = ctx_for(P)
    ids = [0, 3, 1, 4, 2]
    mods = [(q + p)[i] for i in ids]
    x = synth.stream(1, "gpu/ntt/%d" % log_n).residues(mods, P.n)
    say("ntt log_n", log_n)
    t = dev(x)
    C.ntt(t, ids)
    torch.cuda.synchronize()
    want = oracle.ntt(x, mods, log_n)
    assert_same(host(t), want, "ntt")
    C.intt(t, ids)
    torch.cuda.synchronize()
    assert_same(host(t), x, "intt(ntt)")
    t2 = dev(want)
    C.intt(t2, ids)
    torch.cuda.synchronize()
    assert_same(host(t2), oracle.intt(want, mods, log_n), "intt")
    # one limb, and the zero polynomial
    t3 = dev(x[:1])
    C.ntt(t3, ids[:1])
    z = dev(np.zeros((1, P.n), np.uint32))
    C.ntt(z, [4])
    torch.cuda.synchronize()
    assert_same(host(t3), want[:1], "ntt one limb")
    assert not host(z).any()


def test_ntt_many_limbs(params_mid):
    """More limbs than fit one launch map (chunked launches)."""
    P = params_mid
    C = ctx_for(P)
    ids = [i % (P.n_q + P.alpha) for i in range(150)]
    mods = [(P.q + P.p)[i] for i in ids]
    x = synth.stream(2, "gpu/ntt/many").residues(mods, P.n)
    t = dev(x)
    C.ntt(t, ids)
    torch.cuda.synchronize()
    assert_same(host(t), oracle.ntt(x, mods, P.log_n), "ntt 150 limbs")


# ----------------------------------------------------------------------------
# BConv
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["small", "mid", "full"])
def test_bconv(which, params_small, params_mid, params_full):
    P = {"small": params_small, "mid": params_mid, "full": params_full}[which]
    C = ctx_for(P)
    all_ids = list(range(P.n_q + P.alpha))
    mods_all = P.q + P.p
    cases = [(all_ids[:P.alpha], all_ids[P.alpha:]), (all_ids[P.n_q:], all_ids[:P.n_q]), ([0], all_ids[1:])]
    if len(all_ids) > 12:
        cases.append((all_ids[:12], all_ids[12:20]))  # more than 8 inputs: the lazy range fixes
    for ins, outs in cases:
        say("bconv", which, len(ins), "->", len(outs))
        x = synth.stream(3, "gpu/bconv/%s/%d" % (which, len(ins))).residues([mods_all[i] for i in ins], P.n)
        out = empty(len(outs), P.n)
        C.bconv(dev(x), ins, out, outs)
        torch.cuda.synchronize()
        want = oracle.bconv(x, [mods_all[i] for i in ins], [mods_all[i] for i in outs], P.log_n)
        assert_same(host(out), want, "bconv")


# ----------------------------------------------------------------------------
# KeySwitch, HMult, HRot, rescale on random residues
# ----------------------------------------------------------------------------
def _levels(P):
    return sorted({P.n_q, max(P.n_q - 1, 1), 1, min(P.alpha + 1, P.n_q)}, reverse=True)


@pytest.mark.parametrize("which", ["small", "mid"])
def test_keyswitch(which, params_small, params_mid):
    P = params_small if which == "small" else params_mid
    C = ctx_for(P)
    evk = rand_key(P, "gpu/ks/key")
    evk_d = dev(evk)
    for level in _levels(P):
        say("keyswitch", which, "level", level)
        d = synth.stream(4, "gpu/ks/d/%d" % level).residues(P.q[:level], P.n)
        o0, o1 = empty(level, P.n), empty(level, P.n)
        C.keyswitch(dev(d), level, evk_d, o0, o1)
        torch.cuda.synchronize()
        w0, w1 = oracle.keyswitch(P, d, level, evk)
        assert_same(host(o0), w0, "keyswitch out0 level %d" % level)
        assert_same(host(o1), w1, "keyswitch out1 level %d" % level)


@pytest.mark.parametrize("which", ["small", "mid"])
def test_hmult_and_rescale(which, params_small, params_mid):
    P = params_small if which == "small" else params_mid
    C = ctx_for(P)
    rlk = rand_key(P, "gpu/hm/rlk")
    rlk_d = dev(rlk)
    for level in _levels(P):
        say("hmult", which, "level", level)
        la, lb = min(level + 1, P.n_q), level  # first input above the operation level
        a, b = rand_ct(P, la, "gpu/hm/a/%d" % level), rand_ct(P, lb, "gpu/hm/b/%d" % level)
        out = empty(2, level, P.n)
        C.hmult(dev(a), dev(b), rlk_d, level, out)
        torch.cuda.synchronize()
        want = oracle.hmult(P, a, b, rlk, level)
        assert_same(host(out), want, "hmult level %d" % level)
        if level >= 2:
            rs = empty(2, level - 1, P.n)
            C.rescale(out, rs)
            fused = empty(2, level - 1, P.n)
            C.hmult_rescale(dev(a), dev(b), rlk_d, level, fused)
            torch.cuda.synchronize()
            want_rs = oracle.rescale(P, want, level)
            assert_same(host(rs), want_rs, "rescale level %d" % level)
            assert_same(host(fused), want_rs, "fused hmult+rescale level %d" % level)


@pytest.mark.parametrize("which", ["small", "mid"])
def test_hrot(which, params_small, params_mid):
    P = params_small if which == "small" else params_mid
    C = ctx_for(P)
    for k in (1, 5, -1, P.n // 2 - 3):
        rk = rand_key(P, "gpu/hr/rk/%d" % k)
        rk_d = dev(rk)
        for level in _levels(P)[:2]:
            say("hrot", which, "k", k, "level", level)
            ct = rand_ct(P, P.n_q, "gpu/hr/ct/%d" % level)
            out = empty(2, level, P.n)
            C.hrot(dev(ct), level, k, rk_d, out)
            torch.cuda.synchronize()
            want = oracle.hrot(P, ct, level, oracle.galois_element(k % (P.n // 2), P.log_n), rk)
            assert_same(host(out), want, "hrot k %d level %d" % (k, level))


# ----------------------------------------------------------------------------
# full size: N=2^16, 24 ciphertext primes, 8 special primes, dnum 3
# ----------------------------------------------------------------------------
def test_full_size_hmult_rescale_hrot(params_full):
    P = params_full
    C = ctx_for(P)
    level = P.n_q
    rlk = rand_key(P, "gpu/full/rlk")
    a, b = rand_ct(P, level, "gpu/full/a"), rand_ct(P, level, "gpu/full/b")
    say("full hmult")
    out = empty(2, level, P.n)
    C.hmult(dev(a), dev(b), dev(rlk), level, out)
    rs = empty(2, level - 1, P.n)
    C.rescale(out, rs)
    torch.cuda.synchronize()
    want = oracle.hmult(P, a, b, rlk, level)
    fused = empty(2, level - 1, P.n)
    C.hmult_rescale(dev(a), dev(b), dev(rlk), level, fused)
    torch.cuda.synchronize()
    want_rs = oracle.rescale(P, want, level)
    assert_same(host(out), want, "full hmult")
    assert_same(host(rs), want_rs, "full rescale")
    assert_same(host(fused), want_rs, "full fused hmult+rescale")
    say("full hrot")
    rk = rand_key(P, "gpu/full/rk1")
    o2 = empty(2, level, P.n)
    C.hrot(dev(a), level, 1, dev(rk), o2)
    torch.cuda.synchronize()
    assert_same(host(o2), oracle.hrot(P, a, level, oracle.galois_element(1, P.log_n), rk), "full hrot")


# ----------------------------------------------------------------------------
# real keys and encryptions: GPU == oracle, and the oracle's result decrypts
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["small", "mid"])
def test_encrypted_hmult_hrot(which, params_small, params_mid):
    from helpers import Keys
    P = params_small if which == "small" else params_mid
    scale = 2.0 ** 28 if which == "small" else 2.0 ** 30
    K = Keys(P, 0, rot_ks=(1,))
    C = ctx_for(P)
    level = P.n_q
    st = synth.stream(0, "msg")
    u, v = st.complex_slots(P.n // 2), st.complex_slots(P.n // 2)
    ca, cb = K.encrypt(u, scale, level, "a"), K.encrypt(v, scale, level, "b")
    say("encrypted hmult", which)
    rs = empty(2, level - 1, P.n)
    C.hmult_rescale(dev(ca), dev(cb), dev(K.rlk), level, rs)
    ro = empty(2, level, P.n)
    C.hrot(dev(ca), level, 1, dev(K.rot[1]), ro)
    torch.cuda.synchronize()
    want = oracle.rescale(P, oracle.hmult(P, ca, cb, K.rlk, level), level)
    assert_same(host(rs), want, "encrypted hmult+rescale")
    got = oracle.decrypt(P, want, K.s, scale * scale / P.q[level - 1])
    assert np.max(np.abs(got - u * v)) <= 2.0 ** -12
    want_r = oracle.hrot(P, ca, level, oracle.galois_element(1, P.log_n), K.rot[1])
    assert_same(host(ro), want_r, "encrypted hrot")
    assert np.max(np.abs(oracle.decrypt(P, want_r, K.s, scale) - np.roll(u, -1))) <= 2.0 ** -12


# ----------------------------------------------------------------------------
# argument errors are reported, not launched
# ----------------------------------------------------------------------------
def test_argument_errors(params_small):
    P = params_small
    C = ctx_for(P)
    ct = dev(rand_ct(P, 3, "gpu/err"))
    rlk = dev(rand_key(P, "gpu/err/rlk"))
    out = empty(2, 3, P.n)
    with pytest.raises(ck.CkksError, match="level"):
        C.hmult(ct, ct, rlk, 4, out)
    with pytest.raises(ck.CkksError, match="level"):
        C.rescale(ct[:, :1].contiguous(), empty(2, 1, P.n))
    with pytest.raises(ck.CkksError, match="workspace"):
        C.hmult(ct, ct, rlk, 3, out, ws=torch.empty(64, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ck.CkksError, match="overlap"):
        C.hmult(ct, ct, rlk, 3, ct)
    buf = torch.empty(P.n * 3 + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(ck.CkksError, match="misaligned"):
        C.ntt(buf[1:], [0, 1, 2])
    with pytest.raises(ck.CkksError, match="prime id"):
        C.ntt(out, [0, 9])
    with pytest.raises(ck.CkksError, match="1 mod 2N|prime"):
        ck.Context(12, [268369921, 268369923], [1073692673])


# ----------------------------------------------------------------------------
# ciphertexts with their scale (ckks_ct calls): same residues as the raw calls,
# scale tracked as Sec. 2.1 states, and the tracked scale decodes the result
# ----------------------------------------------------------------------------
def test_ct_calls_track_scale(params_mid):
    from helpers import Keys
    P = params_mid
    scale = 2.0 ** 30
    K = Keys(P, 0, rot_ks=(3,))
    C = ctx_for(P)
    L = P.n_q
    st = synth.stream(0, "msg/ct")
    u, v = st.complex_slots(P.n // 2), st.complex_slots(P.n // 2)
    ca, cb = K.encrypt(u, scale, L, "ct/a"), K.encrypt(v, scale, L, "ct/b")
    A, B = ck.Ciphertext(dev(ca), scale), ck.Ciphertext(dev(cb), scale)
    rlk, rk = dev(K.rlk), dev(K.rot[3])
    say("ckks_ct calls")
    hm = C.ct_hmult(A, B, rlk, L, ck.Ciphertext(empty(2, L, P.n), 0.0))
    assert hm.scale == scale * scale and hm.level == L
    rs = C.ct_rescale(hm, ck.Ciphertext(empty(2, L - 1, P.n), 0.0))
    assert rs.scale == scale * scale / P.q[L - 1] and rs.level == L - 1
    fused = C.ct_hmult_rescale(A, B, rlk, L, ck.Ciphertext(empty(2, L - 1, P.n), 0.0))
    assert fused.scale == rs.scale
    rot = C.ct_hrot(A, L, 3, rk, ck.Ciphertext(empty(2, L, P.n), 0.0))
    assert rot.scale == scale
    torch.cuda.synchronize()
    want = oracle.hmult(P, ca, cb, K.rlk, L)
    assert_same(host(hm.data), want, "ct_hmult")
    want_rs = oracle.rescale(P, want, L)
    assert_same(host(rs.data), want_rs, "ct_rescale")
    assert_same(host(fused.data), want_rs, "ct_hmult_rescale")
    assert np.max(np.abs(oracle.decrypt(P, host(fused.data), K.s, fused.scale) - u * v)) <= 2.0 ** -12
    assert np.max(np.abs(oracle.decrypt(P, host(rot.data), K.s, rot.scale) - np.roll(u, -3))) <= 2.0 ** -12
    with pytest.raises(ck.CkksError, match="shape"):
        C.ct_hmult_rescale(A, B, rlk, L, ck.Ciphertext(empty(2, L, P.n), 0.0))
