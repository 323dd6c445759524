"""CPU-only tests of the C-ABI library: exported symbols, input validation,
the host-side steps (structural check, Alg. 4 ordering, Alg. 5 partition)
against the oracle bit for bit, the chunk schedule, the code generator (hex
literals, hipRTC resources) and the generated per-lane code run on the CPU.
None of these launch a GPU kernel.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2501_15126_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIM = os.path.join(os.path.dirname(os.path.abspath(__file__)), "support", "cpu_shim.h")


@pytest.fixture(scope="module")
def P():
    import paper_2501_15126_amd.perm as P
    return P


def test_exports_every_declared_symbol(P):
    with open(os.path.join(ROOT, "include", "perm.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(perm_\w+)\s*\(", hdr, re.M))
    assert {"perm_sparse", "perm_sparse_ex", "perm_batch", "perm_plan", "perm_codegen"} <= declared
    lib = ctypes.CDLL(P.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(P.EXPORTED) == declared
    assert "gfx950" in P.version()


def test_no_oracle_in_product_library(P):
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out
    for f in os.listdir(os.path.join(ROOT, "paper_2501_15126_amd", "csrc")):
        with open(os.path.join(ROOT, "paper_2501_15126_amd", "csrc", f)) as fh:
            assert "oracle" not in fh.read().lower(), f


@pytest.mark.parametrize("bad,status", [
    ((3, [1, 1, 2, 3], [0, 1, 2], [1.0, 1.0, 1.0]), "PERM_EINVAL"),        # colptr[0] != 0
    ((3, [0, 2, 1, 3], [0, 1, 2], [1.0, 1.0, 1.0]), "PERM_EINVAL"),        # decreasing colptr
    ((3, [0, 1, 2, 3], [0, 3, 2], [1.0, 1.0, 1.0]), "PERM_EINVAL"),        # row out of range
    ((3, [0, 2, 3, 4], [1, 0, 1, 2], [1.0, 1.0, 1.0, 1.0]), "PERM_EINVAL"),  # unsorted rows
    ((3, [0, 2, 3, 4], [1, 1, 1, 2], [1.0, 1.0, 1.0, 1.0]), "PERM_EINVAL"),  # duplicate row
    ((3, [0, 1, 2, 3], [0, 1, 2], [1.0, np.nan, 1.0]), "PERM_EINVAL"),     # non-finite
    ((3, [0, 1, 2, 3], [0, 1, 2], [1.0, np.inf, 1.0]), "PERM_EINVAL"),
    ((0, [0], [], []), "PERM_EINVAL"),
    ((65, list(range(66)), list(range(65)), [1.0] * 65), "PERM_ETOOBIG"),
])
def test_validation(P, bad, status):
    n, cp, ri, v = bad
    with pytest.raises(P.PermError) as e:
        P.perm_plan((n, np.array(cp), np.array(ri), np.array(v)))
    assert P.STATUS_NAMES[e.value.status] == status
    assert P.last_error()


def test_structural_rank_matches_oracle(P, oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    for t in range(80):
        n = int(rng.integers(1, 40))
        ccs = W.random_sparse(n, float(rng.uniform(0.02, 0.3)), seed=t, kind="01", diag=bool(t % 2))
        if len(ccs[1]) and ccs[1][-1] == 0:
            continue
        assert P.perm_plan(ccs)["structural_rank"] == O.structural_rank(ccs)


def test_explicit_zeros_are_dropped(P, oracle_mod):
    O = oracle_mod
    A = np.eye(5)
    A[0, 1] = 1.0
    ccs = O.dense_to_ccs(A)
    n, cp, ri, v = ccs
    # same pattern plus explicit zeros in every column
    Az = O.ccs_to_dense(ccs)
    cols, rows, vals, ptr = [], [], [], [0]
    for j in range(5):
        for i in range(5):
            if Az[i, j] != 0 or (i + j) % 2 == 0:
                rows.append(i)
                vals.append(Az[i, j])
        ptr.append(len(rows))
    z = (5, np.array(ptr), np.array(rows), np.array(vals))
    pz, pc = P.perm_plan(z), P.perm_plan(ccs)
    assert pz["row_perm"] == pc["row_perm"] and pz["col_perm"] == pc["col_perm"]
    assert (pz["k"], pz["c"], pz["structural_rank"]) == (pc["k"], pc["c"], pc["structural_rank"])
    assert P.perm_codegen(z) == P.perm_codegen(ccs)


def test_ordering_matches_oracle_alg4(P, oracle_mod):
    O = oracle_mod
    for seed in range(40):
        n = 8 + seed % 33
        ccs = W.random_sparse(n, 0.05 + 0.01 * (seed % 20), seed=seed, kind="01")
        if P.perm_plan(ccs)["structural_rank"] < n:
            continue
        plan = P.perm_plan(ccs, mode="auto")
        rp, cp = O.permanent_ordering(ccs)
        assert plan["row_perm"] == rp and plan["col_perm"] == cp, seed
    # the hand-worked instance of the oracle's tests (Sec. V, Alg. 4)
    A = np.zeros((5, 5))
    for j, rows in enumerate(([0, 1, 2, 3], [2], [1, 4], [0, 3, 4], [0, 1, 2, 3, 4])):
        A[rows, j] = 1.0
    plan = P.perm_plan(O.dense_to_ccs(A))
    assert plan["col_perm"] == [1, 2, 0, 3, 4] and plan["row_perm"] == [2, 1, 4, 0, 3]


def test_partition_matches_oracle_alg5(P, oracle_mod):
    """Alg. 5 of the library (with its gfx950 tau table) against the oracle's
    Alg. 5 given the same table, on Alg. 4-ordered matrices."""
    O = oracle_mod
    for seed in range(30):
        n = 10 + seed
        ccs = W.single_01(n, 0.08 + 0.01 * (seed % 10), seed)
        plan = P.perm_plan(ccs, mode="hybrid")
        A = O.ccs_to_dense(ccs)
        B = O.dense_to_ccs(A[np.ix_(plan["row_perm"], plan["col_perm"])])
        for gr in (16.0, 4.0, 64.0):
            k, c, _ = O.partitioning(B, plan["tau"], gr)
            assert P.perm_partition(B, plan["tau"], gr) == (k, c)
        k, c, _ = O.partitioning(B, plan["tau"], 16.0)
        assert (plan["k"], plan["c"]) == (k, min(c, n - 1))


def test_partition_paper_worked_example(P):
    """The hand-worked 6x6 instance of Alg. 5 (see the oracle pins) through
    the library's partition step."""
    cols = [[0, 1], [1, 2], [0, 3], [2, 4], [3, 5], [4, 5]]
    colptr = np.cumsum([0] + [len(c) for c in cols]).astype(np.int32)
    rowidx = np.array(sum(cols, []), np.int32)
    tau = [1200.0 / (r + 8) for r in range(13)]
    assert P.perm_partition((6, colptr, rowidx, np.ones(len(rowidx))), tau, 16.0) == (4, 3)


def test_tau_model_gfx950(P):
    plan = P.perm_plan(W.single_01(40, 0.1, 1))
    tau = plan["tau"]
    # 256 CUs x 4 SIMDs x 64 lanes x waves; waves = min(8, 512 // vgprs)
    assert tau[0] == 256 * 4 * 64 * 8
    assert all(tau[i] >= tau[i + 1] for i in range(len(tau) - 1))
    assert set(np.unique(tau)) <= {256 * 4 * 64 * w for w in range(1, 9)}


def test_schedule_covers_range(P):
    for n in (1, 2, 3, 9, 24, 36, 40, 52):
        info = P.compile_info(W.single_01(n, 0.3, 2))
        if info["singular"]:
            continue
        assert info["nchunks"] << info["chunk_log2"] == 1 << (n - 1)
        assert info["nblocks"] * info["block"] >= info["nchunks"] > (info["nblocks"] - 1) * info["block"]
        assert 0 <= info["unroll_log2"] <= max(0, info["chunk_log2"] - 1)


def test_aligned_chunks_are_wave_uniform(oracle_mod):
    """Lemma 2 on aligned power-of-two chunks: for 64 consecutive chunks (one
    wave), local step l flips the same column in every lane; the direction is
    the same except at l = 2^(kappa-1), where it is the chunk parity.  The
    step l = 2^kappa (which would differ in column) belongs to the next chunk."""
    O = oracle_mod
    for kappa in (1, 3, 6):
        D = 1 << kappa
        for w in (0, 3):
            for l in range(1, D):
                js = set()
                ss = set()
                for lane in range(64):
                    m = 64 * w + lane
                    j, s = O.changed_bit(m * D + l)
                    js.add(j)
                    ss.add(s)
                    if l == D // 2:
                        assert s == (1 if m % 2 == 0 else -1)
                assert js == {(l & -l).bit_length() - 1}
                assert len(ss) == (2 if l == D // 2 else 1)


def test_codegen_hex_literals_exact(P):
    ccs = W.single_real(12, 0.4, 3)
    src = P.perm_codegen(ccs)
    lits = re.findall(r"-?0x[0-9a-f]\.?[0-9a-f]*p[+-]\d+", src)
    vals = {float.fromhex(s) for s in lits}
    fixed = P.perm_plan(ccs)["col_perm"][-1]  # the fixed column only enters the start values
    n, cp, ri, v = ccs
    for j in range(n):
        if j == fixed:
            continue
        for q in range(cp[j], cp[j + 1]):
            assert float(v[q]) in vals or -float(v[q]) in vals


def test_codegen_resources(P):
    """hipRTC (gfx950) compiles without a GPU.  At the compiler's own occupancy
    x stays in VGPRs (no scratch; nested kernels with copies of rows may use
    up to all 512 VGPRs of one wave per SIMD, the others at most 256); the
    automatic occupancy choice recompiles a 4-wave kernel (97..128 VGPRs) for
    5 waves and a 3-wave one (129..168) for 4, and keeps that build only if it
    spills at most 128 bytes per lane."""
    for ccs in (W.single_01(40, 0.10, 1), W.single_real(36, 0.30, 1), W.single_01(24, 0.15, 1)):
        for mode in ("auto", "pure", "hybrid"):
            plain = P.compile_info(ccs, mode=mode, waves_per_simd=-1)
            assert plain["scratch_bytes"] == 0 and plain["waves_hint"] == 0, (ccs[0], mode)
            copies = " copies=" in P.perm_codegen(ccs, mode=mode, waves_per_simd=-1).splitlines()[0]
            assert plain["vgprs"] <= (512 if copies else 256), (ccs[0], mode, plain["vgprs"])
            auto = P.compile_info(ccs, mode=mode)
            want = 5 if 96 < plain["vgprs"] <= 128 else 4 if 128 < plain["vgprs"] <= 168 else 0
            if auto["waves_hint"] == 0:
                assert auto["vgprs"] == plain["vgprs"] and auto["scratch_bytes"] == 0
                if want:  # the higher-occupancy build was rejected
                    assert P.compile_info(ccs, mode=mode, waves_per_simd=want)["scratch_bytes"] > 128
            else:
                assert auto["waves_hint"] == want, (ccs[0], mode, plain["vgprs"])
                assert auto["vgprs"] <= 512 // want and auto["scratch_bytes"] <= 128
        # x in VGPRs at 4 waves (exact mode, with its residue per level: 3;
        # nested kernels with copies: whatever the copies take)
        own = P.compile_info(ccs, waves_per_simd=-1)
        copies = " copies=" in P.perm_codegen(ccs, waves_per_simd=-1).splitlines()[0]
        assert own["vgprs"] <= (512 if copies else 168 if own["exact"] >= 0 else 128)
        # the LDS tier: cold rows in LDS ([row][lane]), at most 40 KiB per workgroup
        # (k as compiled: Alg. 5 runs again with the compiled kernel's register model)
        lds = P.compile_info(ccs, mode="hybrid", cold_tier="lds")
        assert lds["scratch_bytes"] == 0
        assert lds["lds_bytes"] >= 8 * (ccs[0] - lds["k"]) * lds["block"]
        assert lds["lds_bytes"] <= 40960 + 1024


def _emulate(P, ccs, chunks=None, prime=None, **opts):
    """Run the generated perm_lane() of every chunk (or of the chunks listed)
    on the CPU (g++); the listed chunks' sums are returned in info["sums"].
    Exact mode (integer values): the kernel works on y = 2x; the value is
    scaled back, and info holds the term sum (hi, lo), the residue sum modulo
    `prime` (default: the first of the library's) and the sum of |term|."""
    src = P.perm_codegen(ccs, **opts)
    info = P.compile_info(ccs, **opts)
    exact = info["exact"] >= 0
    pm = float(prime if prime is not None else P.exact_primes()[0]) if exact else 0.0
    d = tempfile.mkdtemp(prefix="permemu")
    f = os.path.join(d, "g.cpp")
    with open(f, "w") as fh:
        # one lane: its own queued blocks (if any) are evaluated after its walk
        fh.write(src + '\nextern "C" void cpu_lane(u64 m, double* xg, u64 xs, u64 lid, double* o, double pm) {'
                 ' static double q[kBlockQueueWords]; u32 ev = 0, qc = 0; double xo[2] = {0.0, 0.0};'
                 ' const double pi = pm > 0.0 ? 1.0 / pm : 0.0;'
                 ' dd r = perm_lane(m, xg, xs, lid, true, q, qc, ev, xo, pm, pi);'
                 ' for (u32 s = 0; s < qc; ++s) r = dd_add(r, block_eval(q + s, ev, xo, pm, pi));'
                 ' o[0] = r.h; o[1] = r.l; o[2] = ev; o[3] = qc; o[4] = xo[0]; o[5] = xo[1]; }\n')
    so = os.path.join(d, "g.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-include", SHIM,
                    "-o", so, f], check=True)
    lib = ctypes.CDLL(so)
    lib.cpu_lane.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                             ctypes.c_double]
    n = ccs[0]
    xg = np.zeros(max(1, n), np.float64)
    o = np.zeros(6)
    tot = 0.0
    hi, lo = 0.0, 0.0
    info["evaluated"] = 0
    info["queued"] = 0
    info["sums"] = []
    info["resid"] = 0
    info["abs_sum"] = 0.0
    for m in range(info["nchunks"]) if chunks is None else chunks:
        lib.cpu_lane(m, xg.ctypes.data, 1, 0, o.ctypes.data, pm)
        tot += o[0] + o[1]
        hi, lo = _dd_add(hi, lo, o[0], o[1])
        if chunks is not None:
            info["sums"].append((o[0] + o[1]) * (2.0 ** -n if exact else 1.0))
        info["evaluated"] += int(o[2])
        info["queued"] += int(o[3])
        info["resid"] += int(o[4])
        info["abs_sum"] += o[5]
    info["hi"], info["lo"] = hi, lo
    scale = 2.0 ** -n if exact else 1.0
    return tot * scale * (2.0 if n % 2 else -2.0), info


def _dd_add(h1, l1, h2, l2):
    """Double-double sum (Knuth's two-sum of the high parts, then the low parts)."""
    s = h1 + h2
    bb = s - h1
    e = (h1 - (s - bb)) + (h2 - bb) + (l1 + l2)
    h = s + e
    return h, e - (h - s)


def test_generated_code_on_cpu_matches_oracle(P, oracle_mod):
    """The generator's per-lane code (all three kernel families, several chunk
    and unroll sizes) compiled for the host and summed over all chunks."""
    O = oracle_mod
    cases = [(W.random_sparse(10, 0.3, 0, kind="real"), 3, 1), (W.random_sparse(13, 0.25, 1, kind="signed"), 5, 2),
             (W.single_01(16, 0.2, 2), 7, 3), (W.random_sparse(9, 0.5, 3, kind="real"), 8, 6),
             (W.random_sparse(5, 0.6, 4, kind="signed"), 1, 1)]
    cases += [(W.single_01(18, 0.12, 5), 9, 3), (W.single_01(20, 0.1, 6), 12, 4)]
    for ccs, kappa, u in cases:
        ref, abs_sum = O.perm_nw(ccs)
        for mode, tier in (("auto", "global"), ("pure", "global"), ("hybrid", "global"), ("hybrid", "lds")):
            for zs in (True, False):
                got, info = _emulate(P, ccs, mode=mode, chunk_log2=kappa, unroll_log2=u, zero_skip=zs, cold_tier=tier)
                assert abs(got - ref) <= 1e-12 * abs_sum + 1e-12, (ccs[0], mode, tier, kappa, u, zs, got, ref)


def _nonzero_terms(ccs, fixed):
    """Number of subsets S of the columns other than `fixed` whose Ryser/NW
    product prod_i (a_i,fixed - rowsum_i / 2 + sum_{j in S} a_ij) is nonzero
    (brute force; exact for 0/1 entries)."""
    n, cp, ri, v = ccs
    A = np.zeros((n, n))
    for j in range(n):
        A[ri[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    others = [j for j in range(n) if j != fixed]
    x0 = A[:, fixed] - A.sum(axis=1) / 2
    bits = (np.arange(1 << (n - 1))[:, None] >> np.arange(n - 1)[None, :]) & 1
    X = x0[None, :] + bits @ A[:, others].T
    return int((X != 0).all(axis=1).sum())


def test_zero_skip_prunes_only_zero_terms(P):
    """With zero-aware skipping the generated code evaluates every nonzero term
    (the count of evaluated terms is at least the brute-force count of nonzero
    ones) and prunes whole intervals (far fewer than 2^(n-1) evaluated)."""
    for ccs, kappa, u in ((W.single_01(18, 0.12, 5), 9, 3), (W.single_01(20, 0.1, 6), 12, 4),
                          (W.single_01(16, 0.2, 2), 11, 2)):
        n = ccs[0]
        fixed = int(P.perm_plan(ccs)["col_perm"][-1])
        nz = _nonzero_terms(ccs, fixed)
        _, on = _emulate(P, ccs, chunk_log2=kappa, unroll_log2=u, zero_skip=True)
        _, off = _emulate(P, ccs, chunk_log2=kappa, unroll_log2=u, zero_skip=False)
        assert off["evaluated"] == 1 << (n - 1)
        assert nz <= on["evaluated"] < (1 << (n - 1)) // 4, (n, nz, on["evaluated"])


def test_generated_chunk_start_at_high_indices(P, oracle_mod):
    """Single chunks of the n=40 workload far into the Gray-index space (the
    chunk start reads bits up to 38 of the Gray code, those from chunk_log2 + 6
    on once per wave), emulated on the CPU, against the oracle over the same
    index range of the plan's ordered matrix.  Most chunks of this matrix sum
    to zero, so the chunks tested are drawn (seeded) among those whose Gray
    start has bit 31 set and whose terms the oracle finds nonzero."""
    O = oracle_mod
    ccs = W.single_01(40, 0.10, 1)
    plan = P.perm_plan(ccs)
    A = O.ccs_to_dense(ccs)
    B = O.dense_to_ccs(A[np.ix_(plan["row_perm"], plan["col_perm"])])
    rng = np.random.default_rng(11)
    for zs in (True, False):  # chunk 2^16 pruned, 2^14 not
        kappa = P.compile_info(ccs, zero_skip=zs)["chunk_log2"]
        top = 1 << (39 - kappa)
        ms, refs = [top - 1], [O.nw_range(B, (top - 1) << kappa, top << kappa)]
        for _ in range(20000):
            m = int(rng.integers(0, top))
            g = (m << kappa) ^ (m << kappa >> 1)
            if g >> 31 & 1:
                r = O.nw_range(B, m << kappa, (m + 1) << kappa)
                if r[1][0] + r[1][1] > 0:
                    ms.append(m)
                    refs.append(r)
                    if len(ms) == 5:
                        break
        assert len(ms) == 5
        _, info = _emulate(P, ccs, chunks=ms, zero_skip=zs)
        for m, got, ((h, l), (ah, al)) in zip(ms, info["sums"], refs):
            assert abs(got - (h + l)) <= 1e-12 * (ah + al), (zs, m, got, h + l)


def test_wave_shares_high_gray_bits_of_chunk_starts(P):
    """The generated chunk start reads the Gray bits from chunk_log2 + 6 up
    once per wave.  That is exact because a wave's 64 chunks are consecutive
    and 64-aligned: workgroups are whole multiples of 64 lanes (other sizes
    are refused) and every launch starts at a multiple of the workgroup."""
    rng = np.random.default_rng(3)
    for kappa in (0, 1, 5, 14, 16, 20):
        for _ in range(50):
            c0 = int(rng.integers(0, 1 << (39 - kappa - 6))) * 64
            high = {((m << kappa) ^ ((m << kappa) >> 1)) >> (kappa + 6) for m in range(c0, c0 + 64)}
            assert len(high) == 1, (kappa, c0)
    # the generator reads per wave exactly the bits from chunk_log2 + 6 up
    for ccs in (W.single_01(40, 0.10, 1), W.single_real(36, 0.30, 1)):
        kappa = P.compile_info(ccs)["chunk_log2"]
        src = P.perm_codegen(ccs)
        wave = [int(j) for j in re.findall(r"\(Gw >> (\d+)\)", src)]
        lane = [int(j) for j in re.findall(r"\(double\)\(\(G >> (\d+)\)", src)]
        assert wave and min(wave) >= kappa + 6 and max(lane) < kappa + 6, (kappa, wave, lane)
    ccs = W.single_01(20, 0.2, 1)
    for b in (32, 96, 100):
        with pytest.raises(P.PermError) as e:
            P.compile_info(ccs, block=b)
        assert e.value.status == P.PERM_EINVAL, b


def test_generated_code_tiny_n_on_cpu(P, oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(6)
    for n in range(1, 7):
        A = rng.uniform(-1, 1, (n, n)) * (rng.random((n, n)) < 0.8)
        A[np.arange(n), rng.permutation(n)] = rng.uniform(0.5, 1, n)
        ref = O.perm_brute(A)
        for kappa in sorted({1, n - 1}):
            if n == 1:
                kappa = 0
            got, _ = _emulate(P, O.dense_to_ccs(A), chunk_log2=kappa)
            assert got == pytest.approx(ref, rel=1e-12, abs=1e-14)


def _batch_lane_lib():
    d = tempfile.mkdtemp(prefix="permbatch")
    so = os.path.join(d, "bl.so")
    csrc = os.path.join(ROOT, "paper_2501_15126_amd", "csrc")
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-include", SHIM,
                    "-I", csrc, "-o", so, os.path.join(os.path.dirname(SHIM), "batch_lane_cpu.cpp")], check=True)
    lib = ctypes.CDLL(so)
    lib.cpu_batch_lane.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                   ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p]
    return lib


def _batch_emulate(P, lib, ccs, prime=None, with_info=False, **opts):
    info, vals, tops = P.batch_describe(ccs, **opts)
    if info["singular"]:
        return (0.0, info) if with_info else 0.0
    desc = np.array([info[k] for k in ("n", "ng", "kappa", "zero_skip", "chunk_top", "singular", "exact")] + [0],
                    np.int32)
    pm = float(prime if prime is not None else P.exact_primes()[0]) if info["exact"] else 0.0
    o = np.zeros(4)
    tot = 0.0
    hi, lo = 0.0, 0.0
    info["resid"], info["abs_sum"] = 0, 0.0
    for m in range(1 << (info["n"] - 1 - info["kappa"])):
        assert lib.cpu_batch_lane(desc.ctypes.data, vals.ctypes.data, vals.size, tops.ctypes.data, m, pm,
                                  o.ctypes.data) == 0
        tot += o[0] + o[1]
        hi, lo = _dd_add(hi, lo, o[0], o[1])
        info["resid"] += int(o[2])
        info["abs_sum"] += o[3]
    info["hi"], info["lo"] = hi, lo
    n = info["n"]
    v = tot * (2.0 ** -n if info["exact"] else 1.0) * (2.0 if n % 2 else -2.0)
    return (v, info) if with_info else v


def test_batch_lane_code_on_cpu_matches_oracle(P, oracle_mod):
    """The batch kernels' per-lane code (compiled for the host) summed over all
    chunks, for many sizes, groups, chunk sizes and zero-skip settings."""
    O = oracle_mod
    lib = _batch_lane_lib()
    rng = np.random.default_rng(21)
    for t in range(40):
        n = int(rng.integers(1, 19))
        kind = ("real", "signed", "01")[t % 3]
        ccs = W.random_sparse(n, float(rng.uniform(0.15, 0.6)), seed=500 + t, kind=kind)
        for shift in (0, -3):
            got = _batch_emulate(P, lib, ccs, batch_kappa_shift=shift)
            if O.structural_rank(ccs) < n:
                assert got == 0.0
                continue
            ref, abs_sum = O.perm_nw(ccs)
            assert abs(got - ref) <= 1e-12 * abs_sum + 1e-12, (t, n, kind, shift, got, ref)
    for seed in range(3):
        ccs = W.single_01(20, 0.12, 900 + seed)
        exact = O.perm_int(ccs)
        for zs in (True, False):
            assert _batch_emulate(P, lib, ccs, zero_skip=zs) == exact


def test_plans_on_random_matrices(P):
    """Planning invariants over many random sparse matrices (n 1..64, all
    modes): the orderings are permutations, HYBRID's register-only columns
    touch register rows only, levels and partition stay in range, and every
    plan is accepted by the code generator."""
    rng = np.random.default_rng(2024)
    for t in range(120):
        n = int(rng.integers(1, 65))
        d = float(rng.uniform(0.02, 0.6))
        ccs = W.random_sparse(n, d, seed=5000 + t, kind=("01", "real", "signed")[t % 3], diag=True)
        for mode in ("auto", "pure", "hybrid"):
            pl = P.perm_plan(ccs, mode=mode)
            assert sorted(pl["row_perm"]) == list(range(n)) and sorted(pl["col_perm"]) == list(range(n))
            assert pl["structural_rank"] == n  # a forced diagonal
            k, c = pl["k"], pl["c"]
            assert 1 <= k <= n and 0 <= c <= n
            assert pl["levels"] >= 1
            if mode == "hybrid" and k < n:
                nn, cp, ri, v = ccs
                rpos = np.empty(n, int)
                rpos[np.asarray(pl["row_perm"])] = np.arange(n)
                for j in range(min(c, n - 1)):
                    col = pl["col_perm"][j]
                    assert all(rpos[r] < k for r in ri[cp[col]:cp[col + 1]]), (t, j)
            if n <= 40 and t % 6 == 0:
                src = P.perm_codegen(ccs, mode=mode)
                assert "perm_gray" in src


def test_batch_limits(P):
    """The batch path bounds its work items per matrix (chunks grow with n)
    and refuses n above 44, where a matrix would need one very long launch."""
    for n, want_kappa in ((30, 13), (42, 13), (43, 14), (44, 15)):
        ccs = W.random_sparse(n, 0.2, seed=n, kind="real", diag=True)
        info, _, _ = P.batch_describe(ccs)
        assert info["kappa"] == want_kappa, (n, info["kappa"])
        assert (n - 1 - info["kappa"]) - 6 <= 22
    with pytest.raises(P.PermError) as e:
        P.batch_describe(W.random_sparse(45, 0.2, seed=45, kind="real", diag=True))
    assert e.value.status == P.PERM_ETOOBIG


def test_tuned_options_round_trip(P):
    """The autotuners return a perm_opts; the binding turns it into keyword
    options that rebuild every tuning field exactly."""
    o = P.make_opts(mode="hybrid", chunk_log2=15, unroll_log2=5, block=128, vgpr_budget=112, force_k=30,
                    force_c=20, max_levels=9, gr_ratio=12.5, zero_skip=False, batch_mode="graph",
                    batch_kappa_shift=-2, cold_tier="lds", waves_per_simd=5)
    back = P.make_opts(**P._opts_kwargs(o))
    for name, _ in P.PermOpts._fields_:
        if name in ("hip_stream", "block_partials", "block_partials_cap", "progress"):
            continue
        assert getattr(back, name) == getattr(o, name), name


def test_autotune_argument_errors(P):
    """Argument checks of the tuning entry points run before any device use."""
    import ctypes
    lib = P.library()
    ccs = W.single_01(12, 0.3, 0)
    m = P._Csc(ccs)
    st = P.PermTuneStats()
    assert lib.perm_autotune(ctypes.byref(m.c), None, None, ctypes.byref(st)) == P.PERM_EINVAL
    assert "null output" in P.last_error()
    best = P.PermOpts()
    assert lib.perm_batch_autotune(0, None, None, ctypes.byref(best), ctypes.byref(st)) == P.PERM_EINVAL
    with pytest.raises(P.PermError):
        P.compile_info(ccs, waves_per_simd=9)


def test_block_queue_on_cpu(P, oracle_mod):
    """Queued blocks (start state saved, evaluated after the walk) give the
    exact result and evaluate exactly the terms the in-place path evaluates;
    a one-lane wave fills an 8-slot queue often, exercising the in-place
    fallback of a full queue as well."""
    O = oracle_mod
    queued_any = False
    for ccs, kappa, u in ((W.single_01(18, 0.12, 5), 9, 3), (W.single_01(20, 0.1, 6), 12, 4),
                          (W.single_01(16, 0.2, 2), 11, 2), (W.single_01(22, 0.1, 7), 14, 2)):
        exact = float(O.perm_int(ccs))
        base, ib = _emulate(P, ccs, chunk_log2=kappa, unroll_log2=u, zero_skip=True, block_queue=False)
        assert ib["queued"] == 0 and base == exact
        for slots in (8, 32):
            got, iq = _emulate(P, ccs, chunk_log2=kappa, unroll_log2=u, zero_skip=True, block_queue=slots)
            assert got == exact, (ccs[0], slots, got, exact)
            assert iq["evaluated"] == ib["evaluated"]
            queued_any |= iq["queued"] > 0
    assert queued_any
    # random 0/1 matrices, chunk and unroll sizes, queue sizes
    rng = np.random.default_rng(77)
    for t in range(8):
        n = int(rng.integers(12, 21))
        ccs = W.single_01(n, float(rng.uniform(0.08, 0.25)), 700 + t)
        kappa = int(rng.integers(4, n - 2))
        u = int(rng.integers(1, min(kappa, 9)))
        slots = (8, 16, 32, 64)[t % 4]
        got, _ = _emulate(P, ccs, chunk_log2=kappa, unroll_log2=u, zero_skip=True, block_queue=slots)
        assert got == float(O.perm_int(ccs)), (n, kappa, u, slots)
    # integer values other than 0/1 through the queue
    A = np.where(np.random.default_rng(3).random((16, 16)) < 0.25, 2.0, 0.0) + np.eye(16) * 3.0
    ccs = O.dense_to_ccs(A)
    ref, abs_sum = O.perm_nw(ccs)
    got, iq = _emulate(P, ccs, chunk_log2=10, unroll_log2=3, zero_skip=True, block_queue=16)
    assert abs(got - ref) <= 1e-12 * abs_sum + 1e-12


def test_paired_block_length_follows_density(P, oracle_mod):
    """Paired FP64 kernels take a chunk-long static block (2^13 paired steps,
    chunks of 2^15 at n >= 37) only where copies leave few operations per
    term; a pair in a denser matrix keeps 2^9-step blocks and fewer copies
    (its chunk-long block compiles for minutes and spills)."""
    O = oracle_mod
    head = lambda ccs: P.perm_codegen(ccs, zero_skip=False, exact=False).splitlines()[0]
    sparse = head(W.er_grid_matrix(40, 0.1, 1))
    assert "pair0" in sparse and "kappa=15 u=13" in sparse, sparse
    A = O.ccs_to_dense(W.er_grid_matrix(40, 0.3, 1))
    A[np.nonzero(A[:, 0])[0][2:], 0] = 0.0  # a first column of two entries
    dense = head(O.dense_to_ccs(A))
    assert "pair0" in dense and " u=9 " in dense, dense
    assert int(re.search(r"copies=(\d+)", dense).group(1)) <= 6, dense
    # a block asked for is taken as given
    assert " u=12 " in P.perm_codegen(O.dense_to_ccs(A), zero_skip=False, exact=False, unroll_log2=12,
                                      copy_cols=-1).splitlines()[0]


def test_spilling_paired_build_takes_fewer_copies(P):
    """A paired FP64 build whose automatically chosen copies spill (ER n = 48,
    p = 0.1: chunks of 2^16 with 2^13-step blocks and copies of 13 columns) is
    compiled again with one copied column fewer; the statistics name the
    copies that ran, and the generated text for them is the compiled one."""
    ccs = W.er_grid_matrix(48, 0.1, 1)
    first = P.perm_codegen(ccs).splitlines()[0]
    assert "copies=13" in first, first
    info = P.compile_info(ccs)
    assert info["scratch_bytes"] == 0 and info["copy_cols"] == 12, (info["scratch_bytes"], info["copy_cols"])
    assert "copies=12" in P.perm_codegen(ccs, copy_cols=info["copy_cols"]).splitlines()[0]
    # copies asked for are kept as asked, spill or not
    assert P.compile_info(ccs, copy_cols=13)["copy_cols"] == 13


def test_nested_without_pairing_on_cpu(P, oracle_mod):
    """FP64 AUTO kernels whose first column has three or more entries (no
    pairing) sum the terms through per-level accumulators, level 0's own
    product starting the lowest, with copies of the rows of the walk's first
    m columns (m = none, 1, 2, 3 and the automatic choice); emulated on the
    CPU over every chunk, against the oracle."""
    O = oracle_mod
    cases = [(W.random_sparse(12, 0.4, 0, kind="real"), 8, 4), (W.random_sparse(14, 0.35, 2, kind="signed"), 9, 5),
             (W.random_sparse(16, 0.4, 7, kind="real"), 10, 4), (W.random_sparse(11, 0.45, 5, kind="real"), 6, 3)]
    nested = 0
    for ccs, kappa, u in cases:
        ref, abs_sum = O.perm_nw(ccs)
        for m in (-1, 1, 2, 3, 0):
            opts = dict(chunk_log2=kappa, unroll_log2=u, zero_skip=False, exact=False, copy_cols=m)
            head = P.perm_codegen(ccs, **opts).splitlines()[0]
            assert "pair0" not in head, (ccs[0], head)
            if " nested" not in head:
                continue  # the cached products were cheaper for this matrix
            nested += 1
            if m > 0:
                assert (" copies=%d" % m) in head, (ccs[0], m, head)
            got, info = _emulate(P, ccs, **opts)
            assert info["evaluated"] == 1 << (ccs[0] - 1)
            assert abs(got - ref) <= 1e-13 * abs_sum + 1e-15, (ccs[0], kappa, u, m, got, ref)
    assert nested >= 12


def _fp64_instructions(src):
    """FP64 VALU instructions (add, mul, fma) of the generated kernel in
    hipcc's gfx950 assembly of the source, built with the flags the library's
    hipRTC compile uses: (those of its step loop, the innermost loop with the
    most of them; those of the whole kernel)."""
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "k.hip")
        with open(f, "w") as fh:
            fh.write("#include <hip/hip_runtime.h>\n" + src)
        subprocess.run([os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                        "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", f,
                        "-o", f + ".s"], check=True, capture_output=True)
        with open(f + ".s") as fh:
            asm = fh.read().splitlines()
    fp = [bool(re.match(r"\s+v_(add|mul|fma|fmac)_f64", x)) for x in asm]
    labels = {m.group(1): i for i, line in enumerate(asm) if (m := re.match(r"^(\.LBB\d+_\d+):", line))}
    loops = []
    far = None  # a long branch's target: s_getpc_b64, s_add_u32 ... (label - pc), s_setpc_b64
    for i, line in enumerate(asm):
        m = re.search(r"s_c?branch\w*\s+(\.LBB\d+_\d+)", line)
        if m and labels.get(m.group(1), i) < i:
            loops.append((labels[m.group(1)], i))
        m = re.search(r"s_add_u32\s+s\d+,\s*s\d+,\s*\((\.LBB\d+_\d+)-\.Lpost_getpc", line)
        if m:
            far = m.group(1)
        if "s_setpc_b64" in line and far is not None:
            if labels.get(far, i) < i:
                loops.append((labels[far], i))
            far = None
    best = 0
    for a, b in loops:
        inner = not any(a <= a2 and b2 <= b and (a2, b2) != (a, b) and any(fp[a2:b2]) for a2, b2 in loops)
        if inner:
            best = max(best, sum(fp[a:b]))
    return best, sum(fp)


def test_loop_operation_count_matches_isa(P):
    """FP64 nested kernels: ops_per_step is the compiled kernel's FP64
    instructions per Gray term of a chunk (the step loop's times its
    iterations, the rest once), read by the library from the code object's
    machine code; hipcc's gfx950 assembly of the same source, an independent
    reading, gives exactly the same, with and without copies of the most
    frequent columns' rows."""
    for ccs, ms, u in ((W.single_01(40, 0.10, 1), (-1, 1, 3, 8), 9), (W.single_01(40, 0.10, 1), (0,), 0),
                       (W.single_01(36, 0.15, 1), (-1, 3, 0), 9), (W.single_real(36, 0.30, 1), (0,), 0),
                       (W.single_real(36, 0.30, 1), (0,), 10)):
        # (the last two without pairing, the last with a loop body beyond a
        # branch's reach; u = 0: the default static block, for n = 40 the whole chunk)
        for m in ms:
            opts = dict(zero_skip=False, exact=False, copy_cols=m, waves_per_simd=-1, unroll_log2=u)
            src = P.perm_codegen(ccs, **opts)
            head = src.splitlines()[0]
            assert " nested" in head
            info = P.compile_info(ccs, **opts)
            pair = 1 if "pair0" in head else 0
            # static blocks of 2^(u+1) steps; with pairing a step covers two terms
            iters = 2 ** (info["chunk_log2"] - pair - info["unroll_log2"] - 1)
            loop, total = _fp64_instructions(src)
            if iters >= 2:
                want = (loop * iters + total - loop) / 2.0 ** info["chunk_log2"]
                assert loop > 0
            else:  # one pass over the chunk: straight-line code
                want = total / 2.0 ** info["chunk_log2"]
            assert info["ops_per_step"] == want, (ccs[0], m, loop, total, info)
            assert info["ops_per_step"] <= info["flops_per_step"] <= 2 * info["ops_per_step"]


def test_autotune_singular_needs_no_device(P):
    """A structurally singular matrix has nothing to tune: perm_autotune
    answers with the options it was given and times no candidate (no device
    is touched, so this runs on the CPU)."""
    ccs = W.random_sparse(9, 0.3, seed=3, kind="real")
    n, cp, ri, v = ccs
    keep = ri != 0  # row 0 left empty: structurally singular
    cp2 = np.concatenate([[0], np.cumsum([keep[cp[j]:cp[j + 1]].sum() for j in range(n)])]).astype(np.int32)
    sing = (n, cp2, ri[keep].astype(np.int32), v[keep])
    opts, st = P.perm_autotune(sing, unroll_log2=3)
    assert st["candidates"] == 0 and opts["unroll_log2"] == 3 and opts["mode"] == "auto"


def test_column0_pairing_on_cpu(P, oracle_mod):
    """All-terms FP64 kernels whose first ordered column has one or two entries
    sum each pair of Gray terms that differ in column 0 by one expression
    (the walk flips columns 1..n-2 only, over half the steps); emulated on the
    CPU over every chunk, against the oracle, with every term accounted for."""
    O = oracle_mod
    cases = [(W.random_sparse(10, 0.3, 0, kind="real"), 3, 1), (W.random_sparse(13, 0.25, 1, kind="signed"), 5, 2),
             (W.random_sparse(14, 0.3, 7, kind="real"), 6, 0), (W.single_01(16, 0.2, 2), 7, 3),
             (W.single_01(20, 0.1, 6), 12, 4), (W.random_sparse(12, 0.2, 9, kind="signed"), 8, 5)]
    # a batch-workload matrix whose column 0 holds one negative entry (the
    # pair's bracket is then that literal, negated)
    cases += [(W.batch_matrix(7, 16), 8, 6)]
    # real and signed entries where column 0 has two: the bracket is kept
    # and moved by constants, in the static steps and through the table
    cases += [(W.random_sparse(13, 0.25, 0, kind="real"), 9, 2), (W.random_sparse(15, 0.2, 0, kind="signed"), 11, 2)]
    # static blocks of two paired steps, with the step loop
    cases += [(W.random_sparse(12, 0.3, 4, kind="real"), 6, 1)]
    twins = 0
    for ccs, kappa, u in cases:
        ref, abs_sum = O.perm_nw(ccs)
        opts = dict(chunk_log2=kappa, unroll_log2=u, zero_skip=False, exact=False)
        src = P.perm_codegen(ccs, **opts)
        assert "pair0" in src.splitlines()[0], (ccs[0], kappa, u)
        # with two levels or more the terms go through per-level accumulators
        # (c_{L-1}, the top one, holds the chunk's sum)
        L = P.compile_info(ccs, **opts)["levels"]
        if L >= 2:
            assert "double c0 = 0.0" in src and f"acc0 = c{L - 1};" in src
        if (kappa, u) in ((9, 2), (11, 2)):
            assert "double dp = " in src and "dp = fma(sg, " in src
        # copies of the rows of the walk's most frequent columns
        twins += " copies=" in src.splitlines()[0] and re.search(r"double x\d+_\d+ = ", src) is not None
        got, info = _emulate(P, ccs, **opts)
        assert info["evaluated"] == 1 << (ccs[0] - 1)
        assert abs(got - ref) <= 1e-13 * abs_sum + 1e-15, (ccs[0], kappa, u, got, ref)
    assert twins == len(cases)
    # every number of copied columns the static block allows
    for ccs, kappa, u in cases[3:6] + cases[-3:]:
        ref, abs_sum = O.perm_nw(ccs)
        for m in (-1, 1, 2, 3):
            opts = dict(chunk_log2=kappa, unroll_log2=u, zero_skip=False, exact=False, copy_cols=m)
            head = P.perm_codegen(ccs, **opts).splitlines()[0]
            assert (" copies=" in head) == (m > 0), (ccs[0], kappa, u, m, head)
            got, info = _emulate(P, ccs, **opts)
            assert info["evaluated"] == 1 << (ccs[0] - 1)
            assert abs(got - ref) <= 1e-13 * abs_sum + 1e-15, (ccs[0], kappa, u, m, got, ref)
    # the exact mode pairs too: the pair's bracket is an integer (y units),
    # its residue d R_1; with two levels or more the residues and |term| sums
    # move up beside the FP64 accumulators, and the error bound's length is
    # the chunk's accumulator operations (at least chunk_log2); residues and
    # the recovered count against the oracle, with and without copies
    # (n = 15, seed 6: a level takes more than 16 moves before it multiplies,
    # so the count-limited reductions are emitted too)
    for ccs, kappa, u, m in ((W.single_01(16, 0.2, 2), 7, 3, 0), (W.single_01(20, 0.1, 6), 12, 4, 0),
                             (W.single_01(20, 0.1, 6), 12, 4, 3), (W.single_01(18, 0.15, 3), 9, 5, -1),
                             (W.single_01(15, 0.15, 6), 12, 9, 0)):
        opts = dict(chunk_log2=kappa, unroll_log2=u, zero_skip=False, copy_cols=m)
        src = P.perm_codegen(ccs, **opts)
        head = src.splitlines()[0]
        assert "pair0" in head and " nested" in head, head
        # residue moves whose reduction waits until the residue multiplies
        assert re.search(r"\br\d+ = t\d+;", src), head
        if ccs[0] == 15:
            assert re.search(r"\br\d+ = fma\(-t\d+, pmod, t\d+\);", src), head
        if m:
            assert (" copies=" in head) == (m > 0), head  # 0: the plan's choice
        bl = P.compile_info(ccs, **opts)["exact_bound_log2"]
        assert kappa <= bl <= kappa + 3, (kappa, bl)
        res = []
        for pm in P.exact_primes():
            got, info = _emulate(P, ccs, prime=pm, **opts)
            assert info["exact"] == 0 and info["evaluated"] == 1 << (ccs[0] - 1)
            res.append(info["resid"])
        perm = O.perm_int(ccs)
        v, est, bound, cert, more = P.exact_recover(ccs[0], info["hi"], info["lo"], info["abs_sum"],
                                                    info["exact_bound_log2"], res[:1])
        assert cert and v == perm, (ccs[0], v, perm)
        v3 = P.exact_recover(ccs[0], info["hi"], info["lo"], info["abs_sum"], info["exact_bound_log2"], res)[0]
        assert v3 == perm
    # not paired: zero-aware kernels, HYBRID
    ccs = W.single_01(16, 0.2, 2)
    for opts in (dict(zero_skip=True, exact=False), dict(zero_skip=True), dict(zero_skip=False, mode="hybrid")):
        assert "pair0" not in P.perm_codegen(ccs, chunk_log2=7, **opts).splitlines()[0], opts
