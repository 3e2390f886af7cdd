"""GPU tests of the serving loop: every request's result, produced inside
a mix of concurrent batches, equals the same request run alone through the
single-operation calls, bit for bit; a sample also equals the oracle.  A
tight memory budget with held results makes requests wait, and changes
nothing in the results."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2407_13055_amd as ck  # noqa: E402
from paper_2407_13055_amd import serving as sv  # noqa: E402

OFFSETS = [1, 5, 17, 100]
N_SRC = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup(params_small, params_mid):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ck.lib()
    env = {}
    for P in (params_small, params_mid):
        C = ck.Context(P.log_n, P.q, P.p)
        st = synth.stream(21, "gpu/serve/%d" % P.log_n)
        L, mods = P.n_q, P.q + P.p

        def cts():
            return np.stack([np.stack([st.residues(P.q, P.n), st.residues(P.q, P.n)]) for _ in range(N_SRC)])

        def key():
            return np.stack([np.stack([st.residues(mods, P.n), st.residues(mods, P.n)]) for _ in range(P.dnum)])
        A, B = cts(), cts()
        rlk = key()
        rks = np.stack([key() for _ in OFFSETS])
        env[P.log_n] = dict(P=P, C=C, A=A, B=B, rlk=rlk, rks=rks, dA=ck.to_device(A), dB=ck.to_device(B),
                            drlk=ck.to_device(rlk), drks=ck.to_device(rks))
    return env


def serve(env, requests, budget, hold, lanes=3, depth=2, max_batch=8, linger=0.0):
    ex = sv.GpuExecutor(ck, torch, {k: e["C"] for k, e in env.items()},
                        {k: (e["dA"], e["dB"]) for k, e in env.items()},
                        {k: (e["drlk"], e["drks"]) for k, e in env.items()}, budget, lanes=lanes, depth=depth,
                        max_batch=max_batch)
    got = {}

    def on_ready(r, b):
        got[r.rid] = ck.to_host(ex.result(b, r.slot))
    clock = sv.RealClock()
    ex.start(clock)
    rep = sv.Server(ex, budget, max_batch=max_batch, hold=hold, on_ready=on_ready, linger=linger).run(requests, clock)
    torch.cuda.synchronize()
    return rep, got


def alone(env, r):
    e = env[r.log_n]
    C, P = e["C"], e["P"]
    out = torch.zeros((2, r.out_level, P.n), dtype=torch.int32, device="cuda")
    a = e["dA"][r.src]
    if r.kind == sv.K_HROT:
        C.hrot(a, r.level, r.rot, e["drks"][r.key], out)
    elif r.kind == sv.K_HMULT_RS:
        C.hmult_rescale(a, e["dB"][r.src], e["drlk"], r.level, out)
    else:
        C.hmult(a, e["dB"][r.src], e["drlk"], r.level, out)
    torch.cuda.synchronize()
    return ck.to_host(out)


def oracle_of(env, r):
    e = env[r.log_n]
    P = e["P"]
    a = e["A"][r.src]
    if r.kind == sv.K_HROT:
        return oracle.hrot(P, a, r.level, oracle.galois_element(r.rot % (P.n // 2), P.log_n), e["rks"][r.key])
    h = oracle.hmult(P, a, e["B"][r.src], e["rlk"], r.level)
    return oracle.rescale(P, h, r.level) if r.kind == sv.K_HMULT_RS else h


def requests(env, rate, duration, seed=0):
    return sv.poisson_requests(seed, rate, duration, sorted(env), {k: e["P"].n_q for k, e in env.items()},
                               OFFSETS, N_SRC)


def check(env, rep, got, n_oracle):
    done = [r for r in rep.requests if not r.rejected]
    assert len(done) == len(rep.requests)
    assert set(got) == {r.rid for r in done}
    for r in done:
        assert np.array_equal(got[r.rid], alone(env, r)), "request %d (%s, N=2^%d, level %d) differs alone" % (
            r.rid, r.kind, r.log_n, r.level)
    pick = synth.stream(22, "gpu/serve/oracle").distinct(0, len(done) - 1, min(n_oracle, len(done)))
    for i in pick.tolist():
        r = done[i]
        assert np.array_equal(got[r.rid], oracle_of(env, r)), "request %d differs from the oracle" % r.rid


def test_mix_equals_alone(setup):
    env = setup
    reqs = requests(env, 4000, 0.1)
    say("serving", len(reqs), "requests")
    # one lane, one batch in flight: requests arriving during a launch wait
    # and share the next batch, on any device speed
    rep, got = serve(env, reqs, 256 << 20, 0.0, lanes=1, depth=1)
    s = rep.summary()
    say("summary", s)
    assert rep.batches < len(reqs)  # some requests shared a batch
    assert all(r.arrival <= r.launched <= r.ready for r in rep.requests)
    check(env, rep, got, 8)


def test_budget_pressure(setup):
    env = setup
    reqs = requests(env, 8000, 0.05, seed=1)
    e = env[13]
    one = (2 * e["P"].n_q * (4 << 13)) + e["C"].workspace_size(ck.OP_HMULT, e["P"].n_q)
    budget = 3 * one
    say("serving under pressure", len(reqs), "requests, budget", budget)
    rep, got = serve(env, reqs, budget, 2e-3)
    assert rep.peak_bytes <= budget and rep.blocked_polls > 0
    check(env, rep, got, 4)


def test_linger_under_load(setup):
    """Heavy arrival rate with a linger time: batches fill up while others
    run, and every result still equals the operation run alone."""
    env = setup
    reqs = requests(env, 20000, 0.05, seed=2)
    say("serving with linger", len(reqs), "requests")
    rep, got = serve(env, reqs, 256 << 20, 0.0, linger=300e-6)
    say("summary", rep.summary())
    assert rep.batches < len(reqs)
    check(env, rep, got, 4)
