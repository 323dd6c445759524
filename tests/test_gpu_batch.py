"""GPU parity tests of perm_batch (precompiled batch kernels) against the oracle.

Tolerance as in test_gpu_perm.py: max(1e-9 |oracle|, (2n + 2) 2^-53 A) for real
inputs; 0/1 inputs must give exactly the integer number of perfect matchings
(the exact mode), compared with == against the oracle's exact integer form.
Full-size parity for the 2000-matrix workload (n 23..30, the 4-row group
counts 6..8 that carry most of its device time) uses stored oracle values
(tests/golden/workload_samples.json, written by make_workload_golden.py).
"""
import json
import os

import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

pytestmark = pytest.mark.gpu

SAMPLES = os.path.join(os.path.dirname(__file__), "golden", "workload_samples.json")


def _samples(kind):
    with open(SAMPLES) as f:
        data = json.load(f)
    return [v for v in data.values() if v["workload"] == kind]


@pytest.fixture(scope="module")
def P():
    import paper_2501_15126_amd.perm as P
    return P


def _tol(n, ref, abs_sum):
    return max(1e-9 * abs(ref), (2 * n + 2) * 2.0 ** -53 * abs_sum)


def _mixed(seed, count):
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(count):
        n = int(rng.integers(1, 23))
        kind = ("real", "signed", "01")[i % 3]
        mats.append(W.random_sparse(n, float(rng.uniform(0.1, 0.6)), seed=seed * 1000 + i, kind=kind,
                                    diag=bool(i % 4)))
    return mats


def test_batch_vs_oracle_mixed(P, oracle_mod):
    """n 1..22, densities 0.1..0.6 (the dense 0/1 ones have FP64 rounding
    bounds far above 1/2): real and signed values within the tolerance, 0/1
    values exactly equal to the oracle's integer count."""
    O = oracle_mod
    mats = _mixed(1, 90)
    got, st = P.perm_batch_ex(mats)
    assert st["count"] == 90
    assert st["exact_uncertified"] == 0
    n01 = 0
    for i, ccs in enumerate(mats):
        n = ccs[0]
        print("batch case", i, n, flush=True)
        if O.structural_rank(ccs) < n:
            assert got[i] == 0.0
            continue
        if (ccs[3] == 1.0).all():
            assert got[i] == float(O.perm_int(ccs)), (i, n, got[i])
            n01 += 1
        else:
            ref, abs_sum = O.perm_nw(ccs)
            assert abs(got[i] - ref) <= _tol(n, ref, abs_sum), (i, n, got[i], ref)
    assert st["exact_certified"] >= n01


def test_batch_workload_goldens(P):
    """The 2000-matrix workload's own matrices at n = 23..30 (8 of each 4-row
    group count 6, 7, 8; U(-1,1) values, the cancellation-heavy case) against
    stored long double oracle values, in the launch form the benchmark times
    and one matrix per launch."""
    recs = _samples("batch")
    assert len(recs) == 24
    mats = [W.batch_matrix(r["seed"], r["index"]) for r in recs]
    for mode in ("streams", "sequential"):
        got = P.perm_batch(mats, batch_mode=mode)
        for r, g, ccs in zip(recs, got, mats):
            assert ccs[0] == r["n"] and len(ccs[2]) == r["nnz"]
            ref = r["perm_ld_hi"] + r["perm_ld_lo"]
            tol = _tol(r["n"], ref, r["abs_sum"])
            print("batch golden", r["index"], r["n"], g, ref, tol, flush=True)
            assert abs(g - ref) <= tol, (r["index"], r["n"], g, ref)


def test_batch_serving_goldens(P):
    """The serving mix's requests at n = 23..36 run as one batch (the server's
    chunk size): 0/1 counts below 2^53 equal the stored exact counts (several
    with FP64 rounding bounds far above 1/2); larger counts, which a double
    cannot hold in general, are within 1e-9 of them, and with all three primes
    forced they are the exact counts rounded to double; real ones within the
    tolerance."""
    recs = _samples("serving")
    assert len(recs) >= 40
    mats = [W.serving_request(r["seed"], r["index"]) for r in recs]
    got, st = P.perm_batch_ex(mats, batch_kappa_shift=-3)
    big = [i for i, r in enumerate(recs) if r["kind"] == "01" and int(r["perm_exact"]) >= 2 ** 53]
    assert len(big) >= 4
    assert st["exact_uncertified"] <= len(big)
    for i, (r, g) in enumerate(zip(recs, got)):
        print("serving golden", r["index"], r["n"], r["kind"], g, flush=True)
        if r["kind"] == "01":
            e = int(r["perm_exact"])
            if i in big:
                assert abs(g - e) <= 1e-9 * e, (r["index"], r["n"], g, e)
            else:
                assert g == float(e), (r["index"], r["n"], g, e)
        else:
            ref = r["perm_ld_hi"] + r["perm_ld_lo"]
            assert abs(g - ref) <= _tol(r["n"], ref, r["abs_sum"]), (r["index"], r["n"], g, ref)
    got3, st3 = P.perm_batch_ex([mats[i] for i in big], batch_kappa_shift=-3, exact_passes=3)
    assert st3["exact_uncertified"] == 0 and st3["passes"] == 3
    for i, g in zip(big, got3):
        assert g == float(int(recs[i]["perm_exact"])), (recs[i]["index"], g, recs[i]["perm_exact"])


def test_batch_exact_passes(P, oracle_mod):
    """Forcing a second and third pass (the next primes, combined by the
    Chinese remainder theorem) leaves every 0/1 count exact and equal."""
    O = oracle_mod
    mats = [W.single_01(n, 0.3, 700 + n) for n in range(14, 23)]
    exact = [O.perm_int(c) for c in mats]
    for k in (1, 2, 3):
        got, st = P.perm_batch_ex(mats, exact_passes=k)
        assert [g == float(e) for g, e in zip(got, exact)] == [True] * len(mats)
        assert st["passes"] == k


@pytest.mark.skip(reason="the persistent graph form (batch_mode 1) stopped making progress on the GPU in this "
                         "test and is switched off until a cause is shown; see "
                         "test_batch_launch_forms_and_alone_are_bitwise_equal for the other forms")
def test_batch_modes_and_alone_are_bitwise_equal(P):
    """Class streams, the persistent graph (captured once, then relaunched),
    one stream, one matrix per launch, other workgroup sizes, and each matrix
    alone: identical bits (a matrix's work and reduction order depend only on
    it)."""
    mats = _mixed(2, 40)
    a = P.perm_batch(mats)
    b, st1 = P.perm_batch_ex(mats, batch_mode="graph")
    b2, st2 = P.perm_batch_ex(mats, batch_mode="graph")  # same layout: the graph is relaunched
    assert st2["graph_captures"] == st1["graph_captures"]
    c = P.perm_batch(mats, batch_mode="sequential")
    d = P.perm_batch(mats, batch_mode="one_stream")
    assert np.array_equal(a, b) and np.array_equal(a, b2) and np.array_equal(a, c) and np.array_equal(a, d)
    for blk in (64, 128):
        for mode in ("streams", "graph"):
            assert np.array_equal(a, P.perm_batch(mats, batch_mode=mode, block=blk))
    # a different batch after a graph run: captured again, still right
    e = P.perm_batch(mats[:17], batch_mode="graph")
    assert np.array_equal(e, a[:17])
    for i in (0, 7, 19, 33):
        alone = P.perm_batch([mats[i]])
        assert alone[0] == a[i]
    rev = P.perm_batch(mats[::-1])
    assert np.array_equal(rev[::-1], a)


def test_batch_launch_forms_and_alone_are_bitwise_equal(P):
    """Class streams, one stream, one matrix per launch, workgroups of 64 and
    128 threads, and each matrix alone: identical bits (a matrix's work and
    reduction order depend only on it).  The persistent graph form is
    refused while it is switched off."""
    mats = _mixed(2, 40)
    print("launch forms: streams", flush=True)
    a = P.perm_batch(mats)
    print("launch forms: sequential, one_stream", flush=True)
    c = P.perm_batch(mats, batch_mode="sequential")
    d = P.perm_batch(mats, batch_mode="one_stream")
    assert np.array_equal(a, c) and np.array_equal(a, d)
    for blk in (64, 128):
        print("launch forms: block", blk, flush=True)
        assert np.array_equal(a, P.perm_batch(mats, batch_mode="streams", block=blk))
    print("launch forms: alone", flush=True)
    for i in (0, 5, 17, 39):
        assert P.perm_batch([mats[i]])[0] == a[i]
    with pytest.raises(P.PermError) as e:
        P.perm_batch(mats, batch_mode="graph")
    assert e.value.status == P.PERM_EINVAL


def test_batch_workload_sample_vs_oracle(P, oracle_mod):
    """Matrices of the batch workload (n ~ U{16..30}, density ~ U[0.15, 0.40],
    U(-1,1) values, no forced diagonal) with n <= 22 checked against the
    oracle; all of them against the generated single-matrix kernel."""
    O = oracle_mod
    mats = [W.batch_matrix(7, i) for i in range(60)]
    got, st = P.perm_batch_ex(mats)
    for i, ccs in enumerate(mats):
        n = ccs[0]
        single, sst = P.perm_sparse_ex(ccs)
        if sst["singular"]:
            assert got[i] == 0.0
            continue
        if n <= 22:
            ref, abs_sum = O.perm_nw(ccs)
            assert abs(got[i] - ref) <= _tol(n, ref, abs_sum), (i, n, got[i], ref)
        assert abs(got[i] - single) <= 1e-9 * abs(single) + 1e-12, (i, n, got[i], single)


def test_batch_zero_skip_exact_and_chunk_shifts(P, oracle_mod):
    O = oracle_mod
    mats = [W.single_01(n, 0.12, 50 + n) for n in range(10, 27)]
    exact = [O.perm_int(c) for c in mats]
    for zs in ("auto", True, False):
        for shift in (-3, 0, 2):
            got = P.perm_batch(mats, zero_skip=zs, batch_kappa_shift=shift)
            for g, e in zip(got, exact):
                assert g == float(e)
    # exact mode off: the plain FP64 kernels, within the rounding bound
    got = P.perm_batch(mats, exact=False)
    for g, e, c in zip(got, exact, mats):
        _, abs_sum = O.perm_nw(c)
        assert abs(g - e) <= max(1e-9 * e, _tol(c[0], e, abs_sum))


def test_batch_edge_cases(P, oracle_mod):
    O = oracle_mod
    empty = P.perm_batch([])
    assert len(empty) == 0
    ones = [O.dense_to_ccs(np.array([[2.5]])), O.dense_to_ccs(np.array([[1.5, -2.0], [0.25, 4.0]])),
            O.dense_to_ccs(np.eye(33)), O.dense_to_ccs(np.eye(30)[::-1].copy())]
    got = P.perm_batch(ones)
    assert got[0] == 2.5
    assert got[1] == pytest.approx(1.5 * 4.0 - 2.0 * 0.25, rel=1e-15)
    assert got[2] == 1.0 and got[3] == 1.0
    singular = np.ones((5, 5))
    singular[:, 1] = 0
    assert P.perm_batch([O.dense_to_ccs(singular)])[0] == 0.0
    with pytest.raises(P.PermError) as e:
        P.perm_batch([ones[0], (2, np.array([0, 1, 1]), np.array([5]), np.array([1.0]))])
    assert e.value.status == P.PERM_EINVAL and "matrix 1" in str(e.value)


def test_batch_autotune(P, oracle_mod):
    """perm_batch_autotune runs the batch per candidate (workgroup size, chunk
    shift) and returns options whose results agree with the oracle."""
    O = oracle_mod
    mats = _mixed(5, 48)
    opts, st = P.perm_batch_autotune(mats)
    print("batch autotune", opts, st, flush=True)
    assert st["candidates"] == 7 and st["sample_fraction"] == 1.0
    assert 0.0 < st["best_ms"] <= st["default_ms"]
    assert opts["batch_mode"] == "streams" and -2 <= opts["batch_kappa_shift"] <= 2
    assert opts["block"] in (0, 64, 128, 256)
    got = P.perm_batch(mats, **opts)
    for i, ccs in enumerate(mats):
        if O.structural_rank(ccs) < ccs[0]:
            assert got[i] == 0.0
            continue
        ref, abs_sum = O.perm_nw(ccs)
        assert abs(got[i] - ref) <= _tol(ccs[0], ref, abs_sum), (i, got[i], ref)
