"""Launch-shape knobs change nothing in the results: HMult + rescale, HRot
and the batched calls agree with the oracle under every candidate setting;
the autotuner times, picks, caches and reapplies a setting."""
import json
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402
from paper_2407_13055_amd import tune  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()


def inputs(P, name):
    st = synth.stream(31, name)
    L, mods = P.n_q, P.q + P.p
    a = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    b = np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)])
    key = np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
    return a, b, key


def run_all(C, P, a, b, key, levels):
    L = P.n_q
    out = torch.zeros((2, L - 1, P.n), dtype=torch.int32, device="cuda")
    C.hmult_rescale(ck.to_device(a), ck.to_device(b), ck.to_device(key), L, out)
    rot = torch.zeros((2, L, P.n), dtype=torch.int32, device="cuda")
    C.hrot(ck.to_device(a), L, 3, ck.to_device(key), rot)
    n = len(levels)
    A = ck.to_device(np.stack([a] * n))
    B = ck.to_device(np.stack([b] * n))
    ob = torch.zeros((n, 2, L - 1, P.n), dtype=torch.int32, device="cuda")
    C.hmult_rescale_batch(A, B, C.batch_items(levels), L, ck.to_device(key), ob)
    torch.cuda.synchronize()
    return ck.to_host(out), ck.to_host(rot), ck.to_host(ob)


def test_every_candidate_matches_the_oracle(params_mid):
    P = params_mid
    C = ck.Context(P.log_n, P.q, P.p)
    a, b, key = inputs(P, "gpu/tune/mid")
    L = P.n_q
    levels = [L, 2, 5]
    want_hm = oracle.rescale(P, oracle.hmult(P, a, b, key, L), L)
    want_rot = oracle.hrot(P, a, L, oracle.galois_element(3, P.log_n), key)
    want_b = [oracle.rescale(P, oracle.hmult(P, a, b, key, lv), lv) for lv in levels]
    split = [{**tune.CANDIDATES[0], "rows_per_thread": 16, "rows_per_thread_single": 4},
             {**tune.CANDIDATES[0], "rows_per_thread": 4, "rows_per_thread_single": 16},
             {**tune.CANDIDATES[0], "keymult_rows": 16, "keymult_rows_single": 4},
             {**tune.CANDIDATES[0], "keymult_rows": 4, "keymult_rows_single": 16},
             {**tune.CANDIDATES[0], "cols_per_thread": 16, "cols_per_thread_single": 4},
             {**tune.CANDIDATES[0], "cols_per_thread": 4, "cols_per_thread_single": 16}]
    for cand in tune.CANDIDATES + split:
        say("tuning", cand)
        C.tune(**cand)
        assert C.tuning == {**cand, "rows_per_thread_single": cand["rows_per_thread_single"] or cand["rows_per_thread"],
                            "keymult_rows_single": cand["keymult_rows_single"] or cand["keymult_rows"],
                            "cols_per_thread_single": cand["cols_per_thread_single"] or cand["cols_per_thread"]}
        hm, rot, ob = run_all(C, P, a, b, key, levels)
        assert np.array_equal(hm, want_hm), cand
        assert np.array_equal(rot, want_rot), cand
        for i, lv in enumerate(levels):
            assert np.array_equal(ob[i, :, :lv - 1], want_b[i]), (cand, lv)
    C.close()


def test_full_size_settings_agree(params_full):
    """At N = 2^16 (where the column-tile order changes the launch), a few
    settings against the default one and one oracle HMult + rescale."""
    P = params_full
    C = ck.Context(P.log_n, P.q, P.p)
    a, b, key = inputs(P, "gpu/tune/full")
    ref = run_all(C, P, a, b, key, [P.n_q, 9])
    assert np.array_equal(ref[0], oracle.rescale(P, oracle.hmult(P, a, b, key, P.n_q), P.n_q))
    for cand in ({"bconv_tpw_up": 1, "bconv_tpw_down": 4, "xcd_pair": 0, "rows_per_thread": 4, "col_threads": 256},
                 {"bconv_tpw_up": 4, "bconv_tpw_down": 1, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 512},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 4, "col_threads": 512},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 256,
                  "rows_per_thread_single": 4},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 1, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 128},
                 {"bconv_tpw_up": 4, "bconv_tpw_down": 2, "xcd_pair": 0, "rows_per_thread": 4, "col_threads": 128},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 4, "col_threads": 128,
                  "keymult_rows": 4},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 128,
                  "rows_per_thread_single": 4, "keymult_rows_single": 4},
                 {"bconv_tpw_up": 1, "bconv_tpw_down": 4, "xcd_pair": 1, "rows_per_thread": 4, "col_threads": 256,
                  "cols_per_thread": 4},
                 {"bconv_tpw_up": 4, "bconv_tpw_down": 2, "xcd_pair": 0, "rows_per_thread": 16, "col_threads": 256,
                  "cols_per_thread": 4, "keymult_rows": 4},
                 {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 16, "col_threads": 128,
                  "rows_per_thread_single": 4, "keymult_rows_single": 4, "cols_per_thread_single": 4}):
        say("tuning", cand)
        C.tune(**cand)
        got = run_all(C, P, a, b, key, [P.n_q, 9])
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), cand
    C.close()


def test_bad_tuning_is_rejected(params_small):
    P = params_small
    C = ck.Context(P.log_n, P.q, P.p)
    for bad in ({"bconv_tpw_up": 3}, {"bconv_tpw_down": 0}, {"xcd_pair": 2}, {"rows_per_thread": 8},
                {"col_threads": 64}, {"rows_per_thread_single": 8}, {"keymult_rows": 8},
                {"keymult_rows_single": 2}, {"cols_per_thread": 8}, {"cols_per_thread_single": 1}):
        with pytest.raises(ck.CkksError):
            C.tune(**bad)
    assert C.tuning == {"bconv_tpw_up": 2, "bconv_tpw_down": 2, "xcd_pair": 1, "rows_per_thread": 16,
                        "col_threads": 256, "rows_per_thread_single": 4, "keymult_rows": 4,
                        "keymult_rows_single": 4, "cols_per_thread": 4, "cols_per_thread_single": 4}
    # the binding's defaults are the library's own
    default = C.tuning
    C.tune(bconv_tpw_up=4, rows_per_thread=4, keymult_rows=16, cols_per_thread=16, col_threads=512)
    assert C.tuning != default
    C.tune()
    assert C.tuning == default
    C.close()


def test_autotune_times_caches_and_reapplies(params_mid, tmp_path):
    P = params_mid
    C = ck.Context(P.log_n, P.q, P.p)
    cache = str(tmp_path / "tuning.json")
    cands = tune.CANDIDATES[:4] + tune.CANDIDATES[-2:]
    r1 = tune.autotune(C, batch=4, reps=2, cache=cache, candidates=cands)
    assert r1["source"] == "timed" and len(r1["table"]) == len(cands) + 8  # + the single-launch widths
    assert {**r1["tuning"], "rows_per_thread_single": 0, "keymult_rows_single": 0, "cols_per_thread_single": 0} in cands
    assert C.tuning == r1["tuning"]
    for k in ("rows_per_thread_single", "keymult_rows_single", "cols_per_thread_single"):
        assert r1["tuning"][k] in (4, 16)
    db = json.load(open(cache))
    assert len(db) == 1 and list(db.values())[0]["tuning"] == r1["tuning"]
    C.tune(**tune.CANDIDATES[-1])
    r2 = tune.autotune(C, cache=cache)
    assert r2["source"] == "cache" and C.tuning == r1["tuning"]
    C.close()


@pytest.mark.parametrize("log_n", [12, 13, 14, 15, 16])
def test_narrow_passes_on_every_ring(log_n):
    """The one-wave-per-row KeyMult and the 4-residue column passes (whose
    radix-4 rounds end with a radix-2 round on odd column sizes) on every
    supported ring degree: HMult + rescale, HRot and a batch, against the
    oracle."""
    P = oracle.Params(log_n, oracle.prime_chain(30, log_n, 5), oracle.prime_chain(31, log_n, 2))
    C = ck.Context(P.log_n, P.q, P.p)
    a, b, key = inputs(P, "gpu/tune/narrow/%d" % log_n)
    L = P.n_q
    levels = [L, 2, 3]
    want_hm = oracle.rescale(P, oracle.hmult(P, a, b, key, L), L)
    want_rot = oracle.hrot(P, a, L, oracle.galois_element(3, P.log_n), key)
    want_b = [oracle.rescale(P, oracle.hmult(P, a, b, key, lv), lv) for lv in levels]
    for cand in ({"cols_per_thread": 4, "keymult_rows": 4, "rows_per_thread": 4, "bconv_tpw_up": 1,
                  "bconv_tpw_down": 1},
                 {"cols_per_thread": 4, "bconv_tpw_up": 2, "bconv_tpw_down": 4, "xcd_pair": 0},
                 {"cols_per_thread": 16, "cols_per_thread_single": 4, "keymult_rows_single": 4,
                  "bconv_tpw_up": 4, "bconv_tpw_down": 2}):
        say("N=2^%d" % log_n, cand)
        C.tune(**cand)
        hm, rot, ob = run_all(C, P, a, b, key, levels)
        assert np.array_equal(hm, want_hm), cand
        assert np.array_equal(rot, want_rot), cand
        for i, lv in enumerate(levels):
            assert np.array_equal(ob[i, :, :lv - 1], want_b[i]), (cand, lv)
    C.close()
