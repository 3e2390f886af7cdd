"""Host-side argument checks of the Python binding: tensors that are not on
the context's GPU, have the wrong dtype or shape, are strided or too small
are refused before anything reaches the C ABI (no GPU needed: the checks run
on a context object whose device tables are never touched)."""
import pytest

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402


def fake_ctx(log_n=12, n_q=3, n_p=1):
    C = ck.Context.__new__(ck.Context)
    C.log_n, C.q, C.p, C.windows = log_n, list(range(n_q)), list(range(n_p)), None
    C.device, C.h, C._ws, C._ws_sizes = 0, None, {}, {}
    return C


def test_cpu_tensors_are_refused():
    C = fake_ctx()
    with pytest.raises(ck.CkksError, match="cuda:0"):
        C._buf(torch.zeros(16, dtype=torch.int32), "x")


def test_shape_checks_of_ciphertexts():
    C = fake_ctx()
    n = C.n
    for bad in (torch.zeros((3, 2, n), dtype=torch.int32), torch.zeros((2, 2, n // 2), dtype=torch.int32),
                torch.zeros((2 * 2 * n,), dtype=torch.int32)):
        with pytest.raises(ck.CkksError, match="shape"):
            C._ct(bad, "ct", 1)
    with pytest.raises(ck.CkksError, match="below the operation level"):
        C._ct(torch.zeros((2, 2, n), dtype=torch.int32), "ct", 3)
    with pytest.raises(ck.CkksError, match="shape"):
        C._cts(torch.zeros((2, 3, n), dtype=torch.int32), "a", 1)
    with pytest.raises(ck.CkksError, match="shape"):
        C._pt(torch.zeros((2, n + 1), dtype=torch.int32), 2)


def test_rescaled_levels():
    C = fake_ctx()
    assert C.rescaled_level(3) == 2
    C.windows = [(2, 1), (1, 2), (0, 5)]
    assert C.rescaled_level(5) == 2 and C.rescaled_level(2) == 1 and C.rescaled_level(1) == 0


def test_key_size():
    C = fake_ctx(12, 3, 1)
    assert C.dnum == 3 and C.key_residues == 3 * 2 * 4 * 4096


@pytest.mark.gpu
def test_gpu_tensor_checks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    C = fake_ctx()
    n = C.n
    with pytest.raises(ck.CkksError, match="dtype"):
        C._buf(torch.zeros(16, dtype=torch.int64, device="cuda"), "x")
    with pytest.raises(ck.CkksError, match="contiguous"):
        C._buf(torch.zeros((4, 4), dtype=torch.int32, device="cuda").t(), "x")
    with pytest.raises(ck.CkksError, match="needs"):
        C._buf(torch.zeros(16, dtype=torch.int32, device="cuda"), "out", 2 * n)
    with pytest.raises(ck.CkksError, match="dtype"):
        C._buf(torch.zeros(16, dtype=torch.int32, device="cuda"), "ws", dtype="uint8")
