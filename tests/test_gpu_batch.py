"""GPU parity tests of perm_batch (precompiled batch kernels) against the oracle.

Tolerance as in test_gpu_perm.py: max(1e-9 |oracle|, (2n + 2) 2^-53 A) for real
inputs, exact integers for 0/1 inputs (which must round to the exact count).
"""
import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


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
    O = oracle_mod
    mats = _mixed(1, 90)
    got, st = P.perm_batch_ex(mats)
    assert st["count"] == 90
    for i, ccs in enumerate(mats):
        n = ccs[0]
        print("batch case", i, n, flush=True)
        if O.structural_rank(ccs) < n:
            assert got[i] == 0.0
            continue
        if (ccs[3] == 1.0).all():
            # exact count; FP64 must round to it unless the rounding bound of
            # this (dense, large) case exceeds 1/2
            exact = O.perm_int(ccs)
            _, abs_sum = O.perm_nw(ccs)
            assert abs(got[i] - exact) <= max(0.49, _tol(n, exact, abs_sum)), (i, got[i], exact)
        else:
            ref, abs_sum = O.perm_nw(ccs)
            assert abs(got[i] - ref) <= _tol(n, ref, abs_sum), (i, n, got[i], ref)


def test_batch_modes_and_alone_are_bitwise_equal(P):
    """Class streams, one graph, one stream, one matrix per launch, and each
    matrix alone: identical bits (a matrix's work and reduction order depend
    only on it)."""
    mats = _mixed(2, 40)
    a = P.perm_batch(mats)
    b = P.perm_batch(mats, batch_mode="graph")
    c = P.perm_batch(mats, batch_mode="sequential")
    d = P.perm_batch(mats, batch_mode="one_stream")
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
    for i in (0, 7, 19, 33):
        alone = P.perm_batch([mats[i]])
        assert alone[0] == a[i]
    rev = P.perm_batch(mats[::-1])
    assert np.array_equal(rev[::-1], a)


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
                assert abs(g - e) < 0.5 and round(g) == e


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
    """perm_batch_autotune runs the batch per candidate (launch form, chunk
    shift) and returns options whose results agree with the oracle."""
    O = oracle_mod
    mats = _mixed(5, 48)
    opts, st = P.perm_batch_autotune(mats)
    print("batch autotune", opts, st, flush=True)
    assert st["candidates"] == 6 and st["sample_fraction"] == 1.0
    assert 0.0 < st["best_ms"] <= st["default_ms"]
    assert opts["batch_mode"] in ("streams", "graph") and -2 <= opts["batch_kappa_shift"] <= 2
    got = P.perm_batch(mats, **opts)
    for i, ccs in enumerate(mats):
        if O.structural_rank(ccs) < ccs[0]:
            assert got[i] == 0.0
            continue
        ref, abs_sum = O.perm_nw(ccs)
        assert abs(got[i] - ref) <= _tol(ccs[0], ref, abs_sum), (i, got[i], ref)
