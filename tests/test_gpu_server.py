"""GPU tests of the submit/poll server: results against the oracle, the same
result alone and in a mix (bitwise), memory-based admission, back-pressure,
and continuous batching (a small request that arrives with a large one
finishes first)."""
import json
import os
import time

import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

pytestmark = pytest.mark.gpu

SAMPLES = os.path.join(os.path.dirname(__file__), "golden", "workload_samples.json")


@pytest.fixture(scope="module")
def P():
    import paper_2501_15126_amd.perm as P
    return P


def _tol(n, ref, abs_sum):
    return max(1e-9 * abs(ref), (2 * n + 2) * 2.0 ** -53 * abs_sum)


def _samples():
    with open(SAMPLES) as f:
        data = json.load(f)
    return [v for v in data.values() if v["workload"] == "serving"]


def test_server_results_vs_oracle(P, oracle_mod):
    """Requests of the serving mix with n <= 22 against the oracle run here,
    0/1 counts exactly equal."""
    O = oracle_mod
    reqs = [W.serving_request(3, i) for i in range(40)]
    reqs = [r for r in reqs if r[0] <= 22]
    with P.Server() as srv:
        tickets = [srv.submit(r) for r in reqs]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs)
    for ccs, g in zip(reqs, got):
        n = ccs[0]
        if O.structural_rank(ccs) < n:
            assert g == 0.0
        elif (ccs[3] == 1.0).all():
            assert g == float(O.perm_int(ccs)), (n, g)
        else:
            ref, abs_sum = O.perm_nw(ccs)
            assert abs(g - ref) <= _tol(n, ref, abs_sum)


def test_server_full_size_goldens(P):
    """The serving mix's own requests at n = 23..36 (0/1 and U(0,1)), all in
    flight together, against stored oracle values: 0/1 counts below 2^53
    exactly equal (several with FP64 rounding bounds far above 1/2), larger
    ones within 1e-9 and, on a server that runs all three primes, the exact
    counts rounded to double; real ones within the tolerance."""
    recs = _samples()
    assert len(recs) >= 40
    reqs = [W.serving_request(r["seed"], r["index"]) for r in recs]
    with P.Server() as srv:
        tickets = [srv.submit(q) for q in reqs]
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    big = [i for i, r in enumerate(recs) if r["kind"] == "01" and int(r["perm_exact"]) >= 2 ** 53]
    assert len(big) >= 4
    assert st["completed"] == len(reqs) and st["exact_uncertified"] <= len(big)
    for i, (r, g) in enumerate(zip(recs, got)):
        print("server golden", r["index"], r["n"], r["kind"], g, flush=True)
        if r["kind"] == "01":
            e = int(r["perm_exact"])
            if i in big:
                assert abs(g - e) <= 1e-9 * e, (r["index"], r["n"], g, e)
            else:
                assert g == float(e), (r["index"], r["n"], g, e)
        else:
            ref = r["perm_ld_hi"] + r["perm_ld_lo"]
            assert abs(g - ref) <= _tol(r["n"], ref, r["abs_sum"]), (r["index"], r["n"], g, ref)
    with P.Server(exact_passes=3) as srv:
        got3 = [srv.wait(t) for t in [srv.submit(reqs[i]) for i in big]]
        st3 = srv.stats()
    assert st3["exact_uncertified"] == 0
    assert got3 == [float(int(recs[i]["perm_exact"])) for i in big]


def test_server_exact_extra_passes(P, oracle_mod):
    """A server that runs every exact request with all three primes (forced
    extra passes re-enter the rounds) returns the same exact counts."""
    O = oracle_mod
    reqs = [W.single_01(n, 0.3, 800 + n) for n in range(14, 24)]
    exact = [O.perm_int(c) for c in reqs]
    with P.Server(exact_passes=3) as srv:
        got = [srv.wait(t) for t in [srv.submit(q) for q in reqs]]
        st = srv.stats()
    assert got == [float(e) for e in exact]
    assert st["extra_passes"] == 2 * len(reqs)


def test_server_wait_from_many_threads(P):
    """Submits from one thread while others wait on (and race to collect) the
    same tickets: each result is collected once, the rest see an unknown or
    collected ticket, and nothing else fails."""
    import threading
    reqs = [W.single_01(18, 0.2, 900 + i) for i in range(24)]
    with P.Server() as srv:
        tickets = []
        lock = threading.Lock()
        results, errors = {}, []

        def waiter(k):
            while True:
                with lock:
                    if k >= len(tickets):
                        if len(tickets) == len(reqs):
                            return
                        t = None
                    else:
                        t = tickets[k]
                if t is None:
                    time.sleep(0.0005)
                    continue
                try:
                    v = srv.wait(t)
                    with lock:
                        results.setdefault(k, []).append(v)
                except P.PermError as e:
                    if e.status != P.PERM_EINVAL:
                        errors.append(e)
                return

        ths = [threading.Thread(target=waiter, args=(k % len(reqs),)) for k in range(3 * len(reqs))]
        for th in ths:
            th.start()
        for q in reqs:
            t = srv.submit(q)
            with lock:
                tickets.append(t)
        for th in ths:
            th.join()
    assert not errors
    assert sorted(results) == list(range(len(reqs)))
    assert all(len(v) == 1 for v in results.values())


def test_server_alone_equals_in_mix(P):
    probe = [W.single_real(24, 0.3, 11), W.single_01(26, 0.15, 12), W.random_sparse(20, 0.3, 13, kind="signed")]
    others = [W.serving_request(5, i) for i in range(30)]
    alone = []
    with P.Server() as srv:
        for q in probe:
            alone.append(srv.wait(srv.submit(q)))
    with P.Server() as srv:
        tickets = []
        for i, o in enumerate(others):
            tickets.append(srv.submit(o))
            if i in (3, 11, 20):
                tickets.append(("probe", srv.submit(probe[(3, 11, 20).index(i)])))
            if i % 7 == 0:
                time.sleep(0.002)
        mixed = [srv.wait(t[1]) for t in tickets if isinstance(t, tuple)]
        for t in tickets:
            if not isinstance(t, tuple):
                srv.wait(t)
    assert mixed == alone
    # the server's chunks: batch_kappa_shift lowered by 3
    assert list(P.perm_batch(probe, batch_kappa_shift=-3)) == alone


def test_server_memory_admission_and_backpressure(P):
    reqs = [W.single_01(22, 0.2, 30 + i) for i in range(12)]
    with P.Server(device_mem_budget=64 * 1024, max_inflight=64) as srv:
        tickets = [srv.submit(r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["arena_peak"] <= 64 * 1024
        assert st["completed"] == 12
        big = W.single_real(40, 0.3, 1)
        with pytest.raises(P.PermError) as e:
            srv.submit(big)
        assert e.value.status == P.PERM_ETOOBIG
    assert list(P.perm_batch(reqs, batch_kappa_shift=-3)) == res
    with P.Server(max_inflight=3) as srv:
        t = [srv.submit(reqs[i]) for i in range(3)]
        assert srv.try_submit(reqs[3]) is None  # three outstanding tickets
        srv.wait(t[0])
        t4 = srv.try_submit(reqs[3])
        assert t4 is not None
        for x in t[1:] + [t4]:
            srv.wait(x)


def test_server_continuous_batching(P):
    """A small request submitted right after a large one is admitted with it,
    shares the rounds, and completes while the large one is still running
    (rounds of 1e9 Gray steps: the large request, 2^33 steps, needs at least
    eight more after the small one's)."""
    large = W.single_real(34, 0.3, 2)
    small = W.single_real(14, 0.3, 3)
    with P.Server(round_steps=1e9) as srv:
        tl = srv.submit(large)
        ts = srv.submit(small)
        vs = srv.wait(ts)
        assert srv.poll(tl) is None, "the large request should still be running"
        vl = srv.wait(tl)
        st = srv.stats()
    assert st["rounds"] >= 2
    assert vs == P.perm_batch([small], batch_kappa_shift=-3)[0]
    assert vl == P.perm_batch([large], batch_kappa_shift=-3)[0]


def test_server_errors(P):
    with P.Server() as srv:
        with pytest.raises(P.PermError) as e:
            srv.submit((3, np.array([0, 1, 2, 3]), np.array([0, 3, 1]), np.ones(3)))
        assert e.value.status == P.PERM_EINVAL
        with pytest.raises(P.PermError) as e:
            srv.poll(123456)
        assert e.value.status == P.PERM_EINVAL
        singular = np.ones((4, 4))
        singular[:, 0] = 0
        from oracle import oracle as O
        t = srv.submit(O.dense_to_ccs(singular))
        assert srv.poll(t) == 0.0
