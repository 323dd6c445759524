"""CPU tests of the exact mode for integer-valued matrices.

The kernels of an integer-valued matrix work on y = 2x, where every term of
Alg. 1 is an integer, and keep (besides the FP64 sum) the term sum modulo a
prime below 2^24 and the sum of |term|.  The integer term sum is
T = sum_g (-1)^g prod_i y_i = (-1)^(n-1) 2^(n-1) perm (Sec. II, Alg. 1 and its
final factor); the oracle's exact integer form of Alg. 1 returns T itself
(mod 2^128), which pins both the kernels' residues and the host's recovery.
"""
import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2501_15126_amd.perm as P
    return P


def _T(O, ccs):
    """Exact integer term sum of a 0/1 pattern (signed), from the oracle."""
    n = ccs[0]
    T, _ = O.nw_int_range(ccs, 0, 1 << (n - 1))
    return T - (1 << 128) if T >= 1 << 127 else T


def _dd(T):
    """(hi, lo) doubles with hi + lo == T exactly (|T| < 2^100)."""
    hi = float(T)
    return hi, float(T - int(hi))


def test_T_is_signed_power_of_two_times_perm(oracle_mod):
    """The identity the recovery rests on, on the oracle's own numbers."""
    O = oracle_mod
    for seed in range(6):
        ccs = W.single_01(10 + 2 * seed, 0.2, seed)
        n = ccs[0]
        assert _T(O, ccs) == (-1) ** (n - 1) * 2 ** (n - 1) * O.perm_int(ccs)


def test_recover_from_oracle_sums(P, oracle_mod):
    """perm_exact_recover on exact oracle sums, and on estimates off by up to
    the stated bound: the integer is recovered exactly whenever the bound is
    below half the modulus, and more primes are asked for otherwise."""
    O = oracle_mod
    primes = P.exact_primes()
    assert primes == sorted(primes, reverse=True) and all(p < 2 ** 24 for p in primes)
    for seed in range(5):
        ccs = W.single_01(14 + seed, 0.25, 40 + seed)
        n = ccs[0]
        T = _T(O, ccs)
        perm = O.perm_int(ccs)
        hi, lo = _dd(T)
        # no error: FP64 alone certifies (no prime needed)
        v, est, bound, cert, more = P.exact_recover(n, hi, lo, 0.0, 10, [])
        assert cert and v == perm and est == perm and bound == 0.0 and not more
        # an estimate off by 1/3 of the modulus (in perm units), within a bound
        # of 0.4 of it: one prime pins the integer
        p = primes[0]
        off = int(p // 3) * 2 ** (n - 1)
        k_bound = 0.4 * p
        # abs_sum giving that bound for chunk 2^10 (the bound is linear in A)
        unit = P.exact_recover(n, 0.0, 0.0, 1.0, 10, [])[2]
        A = k_bound / unit
        res1 = [T % p]
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T + off), A, 10, res1)
        assert cert and v == perm and abs(bound - k_bound) < 1e-6 * k_bound
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T - off), A, 10, res1)
        assert cert and v == perm
        # the same error without a residue: not certified, another pass asked for
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T + off), A, 10, [])
        assert not cert and more and v == est
        # a bound above half of one prime: one residue is not enough, two are
        A2 = 0.7 * p / unit
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T + off), A2, 10, res1)
        assert not cert and more
        res2 = [T % q for q in primes[:2]]
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T + off), A2, 10, res2)
        assert cert and v == perm
        # residues of another integer (perm + 1) with a small bound: rejected,
        # no further pass (the estimate contradicts the residues)
        wrong = [(T + (-1) ** (n - 1) * 2 ** (n - 1)) % q for q in primes[:3]]
        v, est, bound, cert, more = P.exact_recover(n, hi, lo, 1.0, 10, wrong)
        assert not cert and not more and v == est


def test_recover_large_and_negative(P):
    """Beyond 2^53 exactness is not required (no extra pass), but a
    certified result is still the correctly rounded integer; negative
    permanents (integer matrices with negative entries) recover too."""
    primes = P.exact_primes()
    n = 30
    for perm in (2 ** 60 + 12345, -(2 ** 40) - 7, 3):
        T = (-1) ** (n - 1) * 2 ** (n - 1) * perm
        res = [T % p for p in primes]
        v, est, bound, cert, more = P.exact_recover(n, *_dd(T), 0.0, 12, res)
        assert cert and v == float(perm)
    # uncertified above 2^53: no more passes asked for
    perm = 2 ** 70
    T = (-1) ** (n - 1) * 2 ** (n - 1) * perm
    unit = P.exact_recover(n, 0.0, 0.0, 1.0, 12, [])[2]
    v, est, bound, cert, more = P.exact_recover(n, *_dd(T), 1e9 / unit, 12, [T % primes[0]])
    assert not cert and not more and v == float(perm)
    with pytest.raises(P.PermError):
        P.exact_recover(0, 0.0, 0.0, 0.0, 1, [])


def test_error_bound_formula(P):
    """The stated bound: 2^(1-n) A (gamma_{n+1} + N u' (1 + N u')) (1 + 1e-6)
    + 2^(1-n) 1e-24 A, with u = 2^-53, u' = u / (1 - u), N = 2^chunk_log2."""
    u = 2.0 ** -53
    up = u / (1 - u)
    for n, kap, A in ((20, 8, 1e10), (40, 16, 3.7e30), (36, 12, 1.0)):
        g = (n + 1) * u / (1 - (n + 1) * u)
        N = 2.0 ** kap
        want = 2.0 ** (1 - n) * A * ((g + N * up * (1 + N * up)) * (1 + 1e-6) + 1e-24)
        got = P.exact_recover(n, 0.0, 0.0, A, kap, [])[2]
        assert got == pytest.approx(want, rel=1e-12)


def _emulated(P, ccs, **opts):
    from tests.test_host import _emulate
    return _emulate(P, ccs, **opts)


@pytest.mark.parametrize("mode,tier", [("auto", "global"), ("pure", "global"), ("hybrid", "global"),
                                       ("hybrid", "lds")])
def test_generated_exact_residues_match_oracle(P, oracle_mod, mode, tier):
    """The generated kernels in exact mode (emulated on the CPU over every
    chunk): the residue sums equal the oracle's integer term sum modulo each
    prime, the FP64 part is T in y units, and the recovery gives the exact
    count, with and without zero-aware skipping."""
    O = oracle_mod
    primes = P.exact_primes()
    cases = [(W.single_01(16, 0.2, 2), 7, 3), (W.single_01(18, 0.3, 5), 9, 3), (W.single_01(13, 0.45, 8), 6, 2),
             (W.random_sparse(12, 0.4, 3, kind="01"), 5, 1), (W.single_01(15, 0.35, 9), 4, 0)]
    for ccs, kap, u in cases:
        n = ccs[0]
        T = _T(O, ccs)
        perm = O.perm_int(ccs)
        for zs in (True, False):
            res = []
            for p in primes:
                got, info = _emulated(P, ccs, prime=p, mode=mode, cold_tier=tier, chunk_log2=kap, unroll_log2=u,
                                      zero_skip=zs)
                assert info["exact"] == 0  # exact mode chosen automatically
                assert (info["resid"] - T) % p == 0, (n, mode, tier, zs, p)
                res.append(info["resid"])
            assert abs(info["hi"] + info["lo"] - T) <= 1e-12 * info["abs_sum"] + 0.5
            v, est, bound, cert, more = P.exact_recover(n, info["hi"], info["lo"], info["abs_sum"],
                                                        info["exact_bound_log2"], res[:1])
            assert cert and v == perm, (n, mode, tier, zs, v, perm)


def test_generated_exact_integer_values(P, oracle_mod):
    """Integer values other than 0/1 (negative, > 1): exact mode against
    brute force (Eq. (1), exact in long double at these sizes)."""
    O = oracle_mod
    rng = np.random.default_rng(7)
    for t in range(6):
        n = int(rng.integers(4, 10))
        A = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
        A[rng.random((n, n)) < 0.4] = 0.0
        A[np.arange(n), rng.permutation(n)] = rng.choice([-2.0, 1.0, 3.0], size=n)
        ccs = O.dense_to_ccs(A)
        ref = O.perm_brute(A)
        assert ref == round(ref)
        got, info = _emulated(P, ccs, chunk_log2=min(3, n - 1), unroll_log2=1)
        assert info["exact"] == 0
        p = P.exact_primes()[0]
        v, est, bound, cert, more = P.exact_recover(n, info["hi"], info["lo"], info["abs_sum"], info["exact_bound_log2"],
                                                    [info["resid"]])
        assert cert and v == ref, (t, v, ref)


def test_batch_lane_exact_residues_match_oracle(P, oracle_mod):
    """The batch kernels' exact instances (per-lane code on the CPU): residues
    equal the oracle's T modulo the prime, and the recovered count is exact."""
    from tests.test_host import _batch_emulate, _batch_lane_lib
    O = oracle_mod
    lib = _batch_lane_lib()
    primes = P.exact_primes()
    for seed, (n, d) in enumerate([(12, 0.3), (17, 0.25), (19, 0.4), (21, 0.2), (9, 0.6)]):
        ccs = W.single_01(n, d, 300 + seed)
        T = _T(O, ccs)
        perm = O.perm_int(ccs)
        for zs in (True, False):
            for shift in (0, -3):
                got, info = _batch_emulate(P, lib, ccs, prime=primes[1], with_info=True, zero_skip=zs,
                                           batch_kappa_shift=shift)
                assert info["exact"] == 1
                assert (info["resid"] - T) % primes[1] == 0, (n, zs, shift)
                # the residue is modulo the second prime: recover with both
                v, est, bound, cert, more = P.exact_recover(n, info["hi"], info["lo"], info["abs_sum"],
                                                            info["kappa"], [T % primes[0], info["resid"]])
                assert cert and v == perm


def test_exact_option_rules(P):
    """exact = True needs integer values; auto picks it for them only."""
    real = W.single_real(12, 0.3, 1)
    with pytest.raises(P.PermError) as e:
        P.compile_info(real, exact=True)
    assert e.value.status == P.PERM_EINVAL
    assert P.compile_info(real)["exact"] == -1
    assert P.compile_info(W.single_01(12, 0.3, 1))["exact"] == 0
    assert P.compile_info(W.single_01(12, 0.3, 1), exact=False)["exact"] == -1
    info, _, _ = P.batch_describe(W.single_01(12, 0.3, 1))
    assert info["exact"] == 1
    info, _, _ = P.batch_describe(real)
    assert info["exact"] == 0
    with pytest.raises(P.PermError):
        P.batch_describe(real, exact=True)
