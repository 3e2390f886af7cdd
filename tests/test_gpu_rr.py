"""GPU parity of rational rescaling in the 25-30 prime system (Sec. 3.2,
Table 2's construction): every level transition of the exemplar cycle and
of the bootstrapping levels, bit-exact against the oracle at N=2^12 and
2^16; an encryption rescaled on the GPU decrypts to its message."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from test_oracle_rr import encrypt_big

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_ctx = {}


def system(log_n):
    """Context whose ciphertext primes are the inverted-terminal list
    [tau_3..tau_0, q_0..q_10] plus one special prime."""
    if log_n not in _ctx:
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
        taus, qs = oracle.prime_system_25_30(log_n)
        full = list(taus[::-1]) + list(qs)
        p = [oracle.prime_chain(31, log_n, 1)[0]]
        _ctx[log_n] = (ck.Context(log_n, full, p), taus, qs, full)
    return _ctx[log_n]


def ids_of(full, mods):
    return [full.index(m) for m in mods]


@pytest.mark.parametrize("log_n,frm", [(12, 1), (12, 2), (12, 3), (12, 4), (12, 5), (12, 8), (16, 4), (16, 2),
                                       (16, 6)])
def test_rescale_rational_matches_oracle(log_n, frm):
    C, taus, qs, full = system(log_n)
    mi, mo = oracle.level_primes(taus, qs, frm), oracle.level_primes(taus, qs, frm - 1)
    st = synth.stream(64, "gpu/rr/%d/%d" % (log_n, frm))
    ct = np.stack([st.residues(mi, 1 << log_n), st.residues(mi, 1 << log_n)])
    out = torch.zeros((2, len(mo), 1 << log_n), dtype=torch.int32, device="cuda")
    say("rescale_rational N=2^%d level %d -> %d" % (log_n, frm, frm - 1))
    C.rescale_rational(ck.to_device(ct), ids_of(full, mi), ids_of(full, mo), out)
    torch.cuda.synchronize()
    assert np.array_equal(ck.to_host(out), oracle.rescale_rational(ct, mi, mo, log_n))


def test_rescaled_encryption_decrypts():
    log_n = 12
    C, taus, qs, full = system(log_n)
    mi, mo = oracle.level_primes(taus, qs, 4), oracle.level_primes(taus, qs, 3)
    s = synth.stream(65, "gpu/rr/secret").ternary(1 << log_n, 64)
    u = synth.stream(65, "gpu/rr/msg").complex_slots(1 << (log_n - 1))
    ct = encrypt_big(mi, log_n, u, 80, s, "gpu")
    out = torch.zeros((2, len(mo), 1 << log_n), dtype=torch.int32, device="cuda")
    C.rescale_rational(ck.to_device(ct), ids_of(full, mi), ids_of(full, mo), out)
    torch.cuda.synchronize()
    Po = oracle.Params(log_n, mo, [oracle.prime_chain(31, log_n, 1)[0]])
    got = oracle.decrypt(Po, ck.to_host(out), s, 2.0 ** 80 * math.prod(mo) / math.prod(mi))
    assert np.max(np.abs(got - u)) <= 2.0 ** -12


def test_rescale_rational_argument_errors():
    C, taus, qs, full = system(12)
    mi = oracle.level_primes(taus, qs, 4)
    ct = torch.zeros((2, len(mi), 1 << 12), dtype=torch.int32, device="cuda")
    out = torch.zeros((2, len(mi), 1 << 12), dtype=torch.int32, device="cuda")
    ids = ids_of(full, mi)
    with pytest.raises(ck.CkksError):
        C.rescale_rational(ct, ids, ids, out)                 # drops nothing
    with pytest.raises(ck.CkksError):
        C.rescale_rational(ct, ids, [ids[0], ids[0]], out[:, :2].contiguous())  # repeated output prime
    with pytest.raises(ck.CkksError):
        C.rescale_rational(ct, ids, [len(full) + 5], out[:, :1].contiguous())   # prime id out of range
