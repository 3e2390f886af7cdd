"""CPU-side checks of the HIP library: it loads, exports every function the
C header declares, and its host-only prime generator agrees with the
oracle's (two independent implementations of the Eq. 3 prime search)."""
import ctypes
import re

import pytest

import oracle
import paper_2407_13055_amd as ck


def declared_functions():
    text = open(ck.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckks_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for n in ["ckks_ntt", "ckks_intt", "ckks_bconv", "ckks_keyswitch", "ckks_hmult", "ckks_hrot", "ckks_rescale",
              "ckks_ctx_create", "ckks_ctx_destroy", "ckks_workspace_size", "ckks_last_error", "ckks_prime_chain"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = ck.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


@pytest.mark.parametrize("bits,log_n,count", [(28, 12, 3), (30, 12, 1), (30, 16, 24), (31, 16, 8), (30, 13, 7)])
def test_prime_chain_matches_oracle(bits, log_n, count):
    assert ck.prime_chain(bits, log_n, count) == oracle.prime_chain(bits, log_n, count)


def test_prime_chain_reports_shortage():
    with pytest.raises(ck.CkksError):
        ck.prime_chain(12, 10, 50)
    assert "enough" in ck.lib().ckks_last_error().decode()
