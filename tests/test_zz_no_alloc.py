"""GPU test of perm_batch_noalloc, the entry point that allocates no device
memory (its buffers live in the library's fixed device region): two calls in
a row, the second with a smaller batch, each bitwise equal to perm_batch_ex
with the same options, 0/1 counts equal to the oracle's exact integers; a
batch beyond the region is refused with PERM_ETOOBIG."""
import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_15126_amd.perm as P
    return P


def _mixed(seed, count, nmax):
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(count):
        n = int(rng.integers(1, nmax + 1))
        kind = ("real", "signed", "01")[i % 3]
        mats.append(W.random_sparse(n, float(rng.uniform(0.1, 0.6)), seed=seed * 1000 + i, kind=kind,
                                    diag=bool(i % 4)))
    return mats


def test_noalloc_matches_batch_twice(P, oracle_mod):
    O = oracle_mod
    first = _mixed(11, 60, 24) + [W.batch_matrix(1, i) for i in range(40)]
    second = _mixed(12, 17, 18)
    for mats in (first, second):
        print("noalloc: %d matrices, n up to %d" % (len(mats), max(m[0] for m in mats)), flush=True)
        got, st = P.perm_batch_noalloc(mats)
        ref, rst = P.perm_batch_ex(mats)
        assert np.array_equal(got, ref)
        assert st["count"] == len(mats) and st["exact_uncertified"] == rst["exact_uncertified"]
        for i, ccs in enumerate(mats):
            if ccs[0] <= 20 and (ccs[3] == 1.0).all():
                assert got[i] == float(O.perm_int(ccs)), (i, ccs[0])


def test_noalloc_options_and_refusal(P):
    mats = _mixed(13, 30, 22)
    for opts in ({"block": 64}, {"batch_kappa_shift": -2}, {"exact_passes": 2}, {"zero_skip": False}):
        print("noalloc options", opts, flush=True)
        got, _ = P.perm_batch_noalloc(mats, **opts)
        assert np.array_equal(got, P.perm_batch_ex(mats, **opts)[0])
    # 2000 matrices at n = 30 need about 78 MiB (32 KiB of wave partials and
    # 7.7 KiB of column data each): beyond the region, refused before any launch
    big = [W.random_sparse(30, 0.3, seed=5000 + i, kind="real", diag=True) for i in range(2000)]
    with pytest.raises(P.PermError) as e:
        P.perm_batch_noalloc(big)
    assert e.value.status == P.PERM_ETOOBIG and "bytes of device scratch" in str(e.value)
    # the region still serves the next call
    got, _ = P.perm_batch_noalloc(mats)
    assert np.array_equal(got, P.perm_batch_ex(mats)[0])
