"""Pins for the CPU oracle: each test ties an oracle function to something the
paper prints or the mathematics fixes, never to the oracle itself.

The oracle is test infrastructure (see oracle/perm_oracle.c).  Every check here
is chosen so that a plausible mistake (a dropped term, a wrong sign or index, a
transposed operand, an off-by-one in a range) fails at least one of them.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_sequences():
    seqs = {}
    with open(os.path.join(GOLDEN, "paper_gray_sequences.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            seqs[parts[0]] = parts[1:]
    return seqs


def _signed(tok):
    return (1 if tok[0] == "+" else -1, int(tok[1:]))


def _oracle_scbs(O, steps):
    out = []
    for g in range(1, steps + 1):
        j, s = O.changed_bit(g)
        out.append((s, j))
    return out


# ---------------------------------------------------------------------------
# Gray code / signed changed-bit sequence (Sec. II Fig. 1, Sec. IV)
# ---------------------------------------------------------------------------

def test_scbs_matches_printed_sequences(oracle_mod):
    O = oracle_mod
    g = _golden_sequences()
    for name, k in (("SCBS2", 2), ("SCBS3", 3), ("SCBS4", 4)):
        want = [_signed(t) for t in g[name][0].split(",")]
        assert len(want) == 2 ** k - 1
        assert _oracle_scbs(O, 2 ** k - 1) == want, name


def test_fig1_first_iterations(oracle_mod):
    O = oracle_mod
    g = _golden_sequences()
    want = [_signed(t) for t in g["FIG1_FIRST8"][0].split(",")]
    assert _oracle_scbs(O, 8) == want
    s, j = _signed(g["FIG1_STEP16"][0])
    assert O.changed_bit(16) == (j, s)
    # column 4 is used for the first time at iteration 16
    assert all(O.changed_bit(i)[0] != 4 for i in range(1, 16))


def test_unsigned_cbs_5x5(oracle_mod):
    O = oracle_mod
    want = [int(t) for t in _golden_sequences()["CBS_5x5"][0].split(",")]
    assert [O.changed_bit(i)[0] for i in range(1, 16)] == want


def test_chunk_table_5x5(oracle_mod):
    """Sec. IV table: 5 threads, chunks of 3 consecutive iterations."""
    O = oracle_mod
    g = _golden_sequences()
    for loc in range(3):
        toks, distinct = g["TABLE5x5_L%d" % loc]
        want = [_signed(t) for t in toks.split(",")]
        got = []
        for t in range(5):
            j, s = O.changed_bit(3 * t + loc + 1)
            got.append((s, j))
        assert got == want
        assert len(set(got)) == int(distinct)


def test_recursive_scbs_construction(oracle_mod):
    """SCBS(k) = [SCBS(k-1), +(k-1), -SCBS(k-1)^R] (Sec. IV), up to k = 12."""
    O = oracle_mod
    seq = [(1, 0)]  # SCBS(1)
    for k in range(2, 13):
        seq = seq + [(1, k - 1)] + [(-s, j) for (s, j) in reversed(seq)]
        assert _oracle_scbs(O, 2 ** k - 1) == seq


def test_theorem1_closed_form(oracle_mod):
    """Theorem 1: j = largest power of 2 dividing i; sign + iff (i-2^j)/2^(j+1) even."""
    O = oracle_mod
    for i in range(1, 2 ** 14):
        j = (i & -i).bit_length() - 1
        s = 1 if ((i - 2 ** j) // 2 ** (j + 1)) % 2 == 0 else -1
        assert O.changed_bit(i) == (j, s)
    for i in (2 ** 40 + 2 ** 17, 3 * 2 ** 50, 2 ** 62 - 1, 2 ** 63 - 2 ** 5):
        j = (i & -i).bit_length() - 1
        s = 1 if ((i - 2 ** j) // 2 ** (j + 1)) % 2 == 0 else -1
        assert O.changed_bit(i) == (j, s)


def test_lemma1_counts(oracle_mod):
    """Lemma 1: in SCBS(n-1), column j appears exactly 2^(n-j-2) times."""
    O = oracle_mod
    for n in (3, 6, 11, 15):
        counts = [0] * (n - 1)
        for g in range(1, 2 ** (n - 1)):
            counts[O.changed_bit(g)[0]] += 1
        assert counts == [2 ** (n - j - 2) for j in range(n - 1)]


def test_gray_is_reflected_binary(oracle_mod):
    O = oracle_mod
    # consecutive codes differ in one bit; the code is a bijection on [0, 2^k)
    k = 12
    codes = [O.gray(g) for g in range(2 ** k)]
    assert sorted(codes) == list(range(2 ** k))
    for g in range(1, 2 ** k):
        d = codes[g] ^ codes[g - 1]
        assert d & (d - 1) == 0 and d != 0
    # parity of |Gray_g| equals parity of g (the term sign of Alg. 1)
    for g in range(2 ** k):
        assert bin(codes[g]).count("1") % 2 == g % 2


# ---------------------------------------------------------------------------
# Closed forms for the dense definitions (Eq. 1, Eq. 2)
# ---------------------------------------------------------------------------

def _derangements(n):
    d = [1, 0]
    for m in range(2, n + 1):
        d.append((m - 1) * (d[-1] + d[-2]))
    return d[n]


def test_brute_closed_forms(oracle_mod):
    O = oracle_mod
    for n in range(1, 10):
        assert O.perm_brute(np.eye(n)) == 1.0
        assert O.perm_brute(np.ones((n, n))) == math.factorial(n)
        assert O.perm_brute(np.ones((n, n)) - np.eye(n)) == _derangements(n)
    a, b, c, d = 1.5, -2.25, 3.0, 0.5
    assert O.perm_brute(np.array([[a, b], [c, d]])) == a * d + b * c
    # upper triangular: only the identity permutation survives
    rng = np.random.default_rng(0)
    for n in (4, 7, 9):
        U = np.triu(rng.uniform(-2, 2, (n, n)))
        assert O.perm_brute(U) == pytest.approx(float(np.prod(np.diag(U))), rel=1e-15)


def test_ryser_closed_forms(oracle_mod):
    O = oracle_mod
    for n in range(1, 15):
        assert O.perm_ryser(np.ones((n, n))) == math.factorial(n)
        assert O.perm_ryser(np.ones((n, n)) - np.eye(n)) == _derangements(n)
        assert O.perm_ryser(np.eye(n)) == 1.0


def test_ryser_equals_brute_random(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(1)
    for trial in range(60):
        n = int(rng.integers(1, 8))
        A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.6)
        ref = O.perm_brute(A)
        assert O.perm_ryser(A) == pytest.approx(ref, rel=1e-13, abs=1e-13)


# ---------------------------------------------------------------------------
# Alg. 1 (Nijenhuis-Wilf in Gray order) against the definitions
# ---------------------------------------------------------------------------

def test_nw_equals_brute_random_sparse(oracle_mod):
    """200 random sparse matrices, n <= 8, real / signed / 0-1, with and without
    entries in the last column (pins the x-initialisation reading of Alg. 1)."""
    O = oracle_mod
    rng = np.random.default_rng(2)
    no_last = 0
    for trial in range(200):
        n = int(rng.integers(1, 9))
        kind = trial % 3
        mask = rng.random((n, n)) < rng.uniform(0.3, 0.9)
        if trial % 4 == 0:
            mask[:, n - 1] = False  # rows with no entry in column n-1
        if trial % 4 == 1 and n > 1:
            mask[rng.integers(0, n), n - 1] = False
        if kind == 0:
            vals = rng.uniform(0, 1, (n, n))
        elif kind == 1:
            vals = rng.uniform(-1, 1, (n, n))
        else:
            vals = np.ones((n, n))
        A = np.where(mask, vals, 0.0)
        no_last += int(not mask[:, n - 1].all())
        ref = O.perm_brute(A)
        got, abs_sum = O.perm_nw(O.dense_to_ccs(A))
        assert got == pytest.approx(ref, rel=1e-14, abs=1e-14 * max(1.0, abs_sum)), (trial, n)
    assert no_last > 50


def test_nw_closed_forms_large(oracle_mod):
    O = oracle_mod
    for n in (10, 14, 17):
        got, _ = O.perm_nw(O.dense_to_ccs(np.ones((n, n))))
        assert got == pytest.approx(math.factorial(n), rel=1e-15)
        got, _ = O.perm_nw(O.dense_to_ccs(np.ones((n, n)) - np.eye(n)))
        assert got == pytest.approx(_derangements(n), rel=1e-15)
        got, _ = O.perm_nw(O.dense_to_ccs(np.eye(n)))
        assert got == pytest.approx(1.0, rel=0, abs=1e-12)


def test_nw_permuted_triangular(oracle_mod):
    """perm(P U Q) = prod diag(U) for upper-triangular U (n = 20 and 24)."""
    O = oracle_mod
    rng = np.random.default_rng(3)
    for n in (20, 24):
        U = np.triu(rng.uniform(0.5, 1.5, (n, n)) * (rng.random((n, n)) < 0.25))
        U[np.arange(n), np.arange(n)] = rng.uniform(0.5, 2.0, n)
        P, Q = rng.permutation(n), rng.permutation(n)
        A = U[np.ix_(P, Q)]
        got, abs_sum = O.perm_nw(O.dense_to_ccs(A))
        want = float(np.prod(np.diag(U)))
        assert got == pytest.approx(want, rel=1e-12)


def test_nw_block_diagonal(oracle_mod):
    """perm(A (+) B) = perm(A) perm(B), blocks checked by brute force."""
    O = oracle_mod
    rng = np.random.default_rng(4)
    for _ in range(5):
        a, b = int(rng.integers(2, 8)), int(rng.integers(2, 8))
        A = rng.uniform(-1, 1, (a, a)) * (rng.random((a, a)) < 0.7)
        B = rng.uniform(-1, 1, (b, b)) * (rng.random((b, b)) < 0.7)
        M = np.zeros((a + b, a + b))
        M[:a, :a] = A
        M[a:, a:] = B
        perm = rng.permutation(a + b)
        M = M[perm][:, rng.permutation(a + b)]
        got, abs_sum = O.perm_nw(O.dense_to_ccs(M))
        want = O.perm_brute(A) * O.perm_brute(B)
        assert got == pytest.approx(want, rel=1e-12, abs=1e-13 * abs_sum)


def test_nw_invariances(oracle_mod):
    """Row/column permutation (Sec. V), transposition, row scaling."""
    O = oracle_mod
    rng = np.random.default_rng(5)
    for trial in range(10):
        n = int(rng.integers(8, 15))
        ccs = W.random_sparse(n, 0.3, seed=100 + trial, kind="signed")
        A = O.ccs_to_dense(ccs)
        ref, abs_sum = O.perm_nw(ccs)
        tol = 1e-15 * abs_sum * n
        P, Q = rng.permutation(n), rng.permutation(n)
        assert O.perm_nw(O.dense_to_ccs(A[np.ix_(P, Q)]))[0] == pytest.approx(ref, abs=tol)
        assert O.perm_nw(O.dense_to_ccs(A.T))[0] == pytest.approx(ref, abs=tol)
        r = int(rng.integers(0, n))
        A2 = A.copy()
        A2[r] *= 2.0
        assert O.perm_nw(O.dense_to_ccs(A2))[0] == pytest.approx(2.0 * ref, abs=2 * tol)
    # exact invariance for 0/1 matrices (all quantities are small dyadic numbers)
    for trial in range(5):
        ccs = W.single_01(16, 0.2, seed=trial)
        A = O.ccs_to_dense(ccs)
        ref = O.perm_nw(ccs)[0]
        P, Q = rng.permutation(16), rng.permutation(16)
        assert O.perm_nw(O.dense_to_ccs(A[np.ix_(P, Q)]))[0] == ref


def test_nw_range_additivity_and_threads(oracle_mod):
    """Splitting [0, 2^(n-1)) into ranges, or over threads, gives the same sum."""
    O = oracle_mod
    ccs = W.random_sparse(14, 0.35, seed=7, kind="signed")
    N = 1 << 13
    (h, l), _ = O.nw_range(ccs, 0, N, threads=1)
    full = Fraction(h) + Fraction(l)
    parts = Fraction(0)
    cuts = [0, 1, 77, 1024, 4095, 6000, N]
    for a, b in zip(cuts[:-1], cuts[1:]):
        (h, l), _ = O.nw_range(ccs, a, b, threads=1)
        parts += Fraction(h) + Fraction(l)
    assert float(abs(parts - full)) <= 1e-15 * float(abs(full)) + 1e-18
    for t in (2, 3, 8):
        (h, l), _ = O.nw_range(ccs, 0, N, threads=t)
        assert float(abs(Fraction(h) + Fraction(l) - full)) <= 1e-15 * float(abs(full)) + 1e-18
    # the empty range sums to zero; a one-term range is the term itself
    (h, l), _ = O.nw_range(ccs, 5, 5)
    assert h == 0 and l == 0


def test_nw_single_term_is_signed_product(oracle_mod):
    """Term g = (-1)^g prod_i x_i(Gray_g), x(S) = a_{.,n-1} - rowsum/2 + sum_{j in S} a_{.,j}."""
    O = oracle_mod
    rng = np.random.default_rng(8)
    n = 6
    A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.7)
    ccs = O.dense_to_ccs(A)
    for g in (0, 1, 5, 22, 31):
        S = [j for j in range(n - 1) if (g ^ (g >> 1)) >> j & 1]
        x = A[:, n - 1] - A.sum(1) / 2 + A[:, S].sum(1)
        want = (-1) ** g * np.prod(x)
        (h, l), _ = O.nw_range(ccs, g, g + 1, threads=1)
        assert h + l == pytest.approx(want, rel=1e-14, abs=1e-16)


def test_nw_n1_n2(oracle_mod):
    O = oracle_mod
    assert O.perm_nw(O.dense_to_ccs(np.array([[3.5]])))[0] == 3.5
    assert O.perm_nw(O.dense_to_ccs(np.array([[-2.0]])))[0] == -2.0
    A = np.array([[1.25, -3.0], [0.5, 4.0]])
    assert O.perm_nw(O.dense_to_ccs(A))[0] == 1.25 * 4.0 + (-3.0) * 0.5


# ---------------------------------------------------------------------------
# Exact integer permanent of 0/1 patterns
# ---------------------------------------------------------------------------

def _count_perfect_matchings(mask):
    """Independent DP over column subsets: rows matched in order."""
    n = mask.shape[0]
    dp = np.zeros(1 << n, dtype=object)
    dp[0] = 1
    for S in range(1 << n):
        if dp[S] == 0:
            continue
        i = bin(S).count("1")
        if i == n:
            continue
        for j in range(n):
            if mask[i, j] and not (S >> j) & 1:
                dp[S | (1 << j)] += dp[S]
    return int(dp[(1 << n) - 1])


def test_int_equals_matching_count(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(9)
    for trial in range(30):
        n = int(rng.integers(1, 12))
        mask = rng.random((n, n)) < rng.uniform(0.2, 0.8)
        ccs = O.dense_to_ccs(mask.astype(float))
        want = _count_perfect_matchings(mask)
        if ccs[2].size == 0:
            continue
        assert O.perm_int(ccs) == want, trial


def test_int_closed_forms(oracle_mod):
    O = oracle_mod
    for n in (5, 12, 18, 20):
        assert O.perm_int(O.dense_to_ccs(np.ones((n, n)))) == math.factorial(n)
        assert O.perm_int(O.dense_to_ccs(np.ones((n, n)) - np.eye(n))) == _derangements(n)
        assert O.perm_int(O.dense_to_ccs(np.eye(n))) == 1


def test_int_agrees_with_long_double(oracle_mod):
    O = oracle_mod
    for seed in range(3):
        ccs = W.single_01(22, 0.15, seed)
        exact = O.perm_int(ccs)
        approx, _ = O.perm_nw(ccs)
        assert round(approx) == exact
        assert abs(approx - exact) < 1e-6 * max(1, exact)


# ---------------------------------------------------------------------------
# Alg. 4 (PermanentOrdering)
# ---------------------------------------------------------------------------

def test_ordering_is_greedy_min_unordered_degree(oracle_mod):
    """Each chosen column has the fewest nonzeros in not-yet-ordered rows among
    the columns not chosen yet (ties: lowest index); the rows of the chosen
    column that were not ordered yet follow, in ascending row order."""
    O = oracle_mod
    for seed in range(12):
        n = 10 + seed
        ccs = W.random_sparse(n, 0.12 + 0.02 * (seed % 5), seed=seed, kind="01")
        A = O.ccs_to_dense(ccs) != 0
        rowPerm, colPerm = O.permanent_ordering(ccs)
        assert sorted(rowPerm) == list(range(n)) and sorted(colPerm) == list(range(n))
        ordered_rows, chosen = [], []
        for cidx in range(n):
            remaining = [j for j in range(n) if j not in chosen]
            counts = {j: sum(1 for i in range(n) if A[i, j] and i not in ordered_rows) for j in remaining}
            best = min(counts.values())
            assert colPerm[cidx] == min(j for j in remaining if counts[j] == best)
            col = colPerm[cidx]
            chosen.append(col)
            ordered_rows += [i for i in range(n) if A[i, col] and i not in ordered_rows]
        ordered_rows += [i for i in range(n) if i not in ordered_rows]
        assert rowPerm == ordered_rows


def test_ordering_hand_worked_instance(oracle_mod):
    """Alg. 4 on a 5x5 pattern worked by hand (Sec. V): columns hold rows
    c0 = {0,1,2,3}, c1 = {2}, c2 = {1,4}, c3 = {0,3,4}, c4 = {0,...,4}.
    Step 1: counts over unordered rows 4,1,2,3,5 -> column 1; rows [2].
    Step 2: rows other than 2: c0 3, c2 2, c3 3, c4 4 -> column 2; rows [1, 4].
    Step 3: unordered rows {0, 3}: c0 2, c3 2, c4 2 -> the lowest, column 0;
    rows [0, 3].  (By total degree, 4, 3, 5, column 3 would win here.)
    Steps 4-5: no rows left; columns 3, then 4.  A rule taking the largest
    count (column 4 first), the highest index on ties, or rows in descending
    order gives another result."""
    O = oracle_mod
    A = np.zeros((5, 5))
    for j, rows in enumerate(([0, 1, 2, 3], [2], [1, 4], [0, 3, 4], [0, 1, 2, 3, 4])):
        A[rows, j] = 1.0
    rowPerm, colPerm = O.permanent_ordering(O.dense_to_ccs(A))
    assert list(colPerm) == [1, 2, 0, 3, 4]
    assert list(rowPerm) == [2, 1, 4, 0, 3]


def test_ordering_gives_staircase_pattern(oracle_mod):
    """After ordering, the rows touched by the first c columns are the first
    |I_c| rows, for every c (the pattern of Fig. 4a)."""
    O = oracle_mod
    for seed in range(8):
        ccs = W.single_01(30, 0.1, seed)
        A = O.ccs_to_dense(ccs) != 0
        rp, cp = O.permanent_ordering(ccs)
        B = A[np.ix_(rp, cp)]
        for c in range(1, 31):
            touched = np.nonzero(B[:, :c].any(axis=1))[0]
            assert list(touched) == list(range(len(touched)))


def test_ordering_preserves_permanent(oracle_mod):
    O = oracle_mod
    for seed in range(4):
        ccs = W.single_01(18, 0.15, seed)
        A = O.ccs_to_dense(ccs)
        rp, cp = O.permanent_ordering(ccs)
        assert O.perm_int(O.dense_to_ccs(A[np.ix_(rp, cp)])) == O.perm_int(ccs)


# ---------------------------------------------------------------------------
# Alg. 5 (Partitioning)
# ---------------------------------------------------------------------------

def test_partitioning_worked_example(oracle_mod):
    """Hand-worked instance of Alg. 5 on an ordered 6x6 pattern.

    Columns (ordered) touch rows: c0 {0,1}, c1 {1,2}, c2 {0,3}, c3 {2,4},
    c4 {3,5}, c5 {4,5}; tau[r] = 1200 / (r + 8) threads; GRratio = 16.

      j  nrows nreg  regCost            globCost              score
      0    2    4   4*(1/2)   = 2      4*(1/2)*16   = 32     (1200/12)/34     = 2.9412
      1    3    6   6*(3/4)   = 4.5    3*(1/4)*16   = 12     (1200/14)/16.5   = 5.1948
      2    4    8   8*(7/8)   = 7      2*(1/8)*16   = 4      (1200/16)/11     = 6.8182
      3    5   10  10*(15/16) = 9.375  1*(1/16)*16  = 1      (1200/18)/10.375 = 6.4257
      4    6   12  12*(31/32) = 11.625 0                     (1200/20)/11.625 = 5.1613
      5    6   12  12*(63/64) = 11.8125 0                    (1200/20)/11.8125= 5.0794
    Best strictly increasing score is at j = 2 (k = 4, c = 3).  At j = 5 nrows
    (6) differs from k (4), so the "nrows = k" clause does not fire.
    """
    O = oracle_mod
    cols = [[0, 1], [1, 2], [0, 3], [2, 4], [3, 5], [4, 5]]
    colptr = np.cumsum([0] + [len(c) for c in cols]).astype(np.int32)
    rowidx = np.array(sum(cols, []), np.int32)
    ccs = (6, colptr, rowidx, np.ones(len(rowidx)))
    tau = [1200.0 / (r + 8) for r in range(13)]
    k, c, best = O.partitioning(ccs, tau, 16.0)
    assert (k, c) == (4, 3)
    assert best == pytest.approx((1200 / 16) / 11, rel=1e-12)


def test_partitioning_nrows_equal_k_clause(oracle_mod):
    """A column that adds no new row extends c even when its score is lower.

    Columns: c0 {0,1,2,3}, c1 {0,1}, c2 {2}, c3 {3}; tau constant 100; GRratio 16.
    nrows = 4 = n from j = 0 on, so globCost = 0 throughout:
      j=0: regCost 8*(1/2)   = 4   -> 25.0   > 0        -> (k, c) = (4, 1)
      j=1: regCost 8*(3/4)   = 6   -> 16.667 (lower), nrows = k -> (4, 2)
      j=2: regCost 8*(7/8)   = 7   -> 14.286 (lower), nrows = k -> (4, 3)
      j=3: regCost 8*(15/16) = 7.5 -> 13.333 (lower), nrows = k -> (4, 4)
    Without the clause the result would be (4, 1).
    """
    O = oracle_mod
    cols = [[0, 1, 2, 3], [0, 1], [2], [3]]
    colptr = np.cumsum([0] + [len(c) for c in cols]).astype(np.int32)
    rowidx = np.array(sum(cols, []), np.int32)
    k, c, best = O.partitioning((4, colptr, rowidx, np.ones(len(rowidx))), [100.0] * 9, 16.0)
    assert (k, c) == (4, 4)
    assert best == pytest.approx(100 / 7.5, rel=1e-12)
    # the mixed case: c0 {0,1}, c1 {0,1}, c2 {2}, c3 {3}
    #   j=0: 100/(2 + 16) = 5.556 -> (2,1); j=1: 100/(3 + 8) = 9.091 -> (2,2)
    #   j=2: 100/(5.25 + 2) = 13.793 -> (3,3); j=3: 100/7.5 = 13.333, nrows 4 != 3 -> keep
    cols = [[0, 1], [0, 1], [2], [3]]
    colptr = np.cumsum([0] + [len(c) for c in cols]).astype(np.int32)
    rowidx = np.array(sum(cols, []), np.int32)
    k, c, best = O.partitioning((4, colptr, rowidx, np.ones(len(rowidx))), [100.0] * 9, 16.0)
    assert (k, c) == (3, 3)
    assert best == pytest.approx(100 / 7.25, rel=1e-12)


def test_partitioning_register_columns_touch_register_rows(oracle_mod):
    O = oracle_mod
    for seed in range(6):
        ccs = W.single_01(36, 0.12, seed)
        A = O.ccs_to_dense(ccs) != 0
        rp, cp = O.permanent_ordering(ccs)
        B = A[np.ix_(rp, cp)]
        occ = O.dense_to_ccs(B.astype(float))
        tau = [65536.0 / max(1, (r + 40 + 7) // 8 * 8) for r in range(73)]
        k, c, _ = O.partitioning(occ, tau, 16.0)
        assert 1 <= c <= 36 and 1 <= k <= 36
        assert not B[k:, :c].any()
        assert B[k - 1, :c].any()


# ---------------------------------------------------------------------------
# Structural rank
# ---------------------------------------------------------------------------

def test_structural_rank(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(10)
    for trial in range(60):
        n = int(rng.integers(1, 9))
        mask = rng.random((n, n)) < rng.uniform(0.1, 0.6)
        if not mask.any():
            continue
        ccs = O.dense_to_ccs(mask.astype(float))
        has_pm = _count_perfect_matchings(mask) > 0
        assert (O.structural_rank(ccs) == n) == has_pm
    assert O.structural_rank(O.dense_to_ccs(np.eye(7))) == 7
    A = np.ones((5, 5))
    A[2] = 0
    assert O.structural_rank(O.dense_to_ccs(A)) == 4
    # rank of a matrix with two identical single-entry columns
    A = np.eye(4)
    A[:, 1] = 0
    A[0, 1] = 1
    assert O.structural_rank(O.dense_to_ccs(A)) == 3


def _tridiagonal(n, rng, real):
    """Tridiagonal matrix: values U(0.5, 1.5) when real, else all 1."""
    A = np.zeros((n, n))
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                A[i, j] = rng.uniform(0.5, 1.5) if real else 1.0
    return A


def _continuant(A):
    """perm of a tridiagonal matrix, exactly: expanding along the last row,
    perm(T_k) = a_kk perm(T_{k-1}) + a_{k-1,k} a_{k,k-1} perm(T_{k-2})."""
    from fractions import Fraction
    n = A.shape[0]
    f2, f1 = Fraction(1), Fraction(A[0, 0])
    for k in range(1, n):
        f2, f1 = f1, Fraction(A[k, k]) * f1 + Fraction(A[k - 1, k]) * Fraction(A[k, k - 1]) * f2
    return f1


def test_nw_tridiagonal_closed_forms(oracle_mod):
    """Structured sparse matrices with closed-form permanents, rows and columns
    shuffled: tridiagonal (Fibonacci F(n+1) for all ones, the continuant for
    real values), I + cyclic shift (2), 2x2 blocks of ones (2^(n/2))."""
    O = oracle_mod
    rng = np.random.default_rng(11)
    fib = [0, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    for n in (5, 12, 21):
        P_r, P_c = rng.permutation(n), rng.permutation(n)
        A = _tridiagonal(n, rng, real=False)[np.ix_(P_r, P_c)]
        assert O.perm_int(O.dense_to_ccs(A)) == fib[n + 1]
        R = _tridiagonal(n, rng, real=True)
        exact = float(_continuant(R))
        got, abs_sum = O.perm_nw(O.dense_to_ccs(R[np.ix_(P_r, P_c)]))
        assert got == pytest.approx(exact, rel=1e-14)
        C = np.eye(n) + np.roll(np.eye(n), 1, axis=1)
        assert O.perm_int(O.dense_to_ccs(C[np.ix_(P_r, P_c)])) == 2
    n = 16
    B = np.kron(np.eye(n // 2), np.ones((2, 2)))
    assert O.perm_int(O.dense_to_ccs(B[np.ix_(rng.permutation(n), rng.permutation(n))])) == 2 ** (n // 2)
