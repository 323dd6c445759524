// preprocess.cpp -- ordering (Alg. 4), partitioning (Alg. 5), the gfx950
// thread-count model, the cached-product level plan and the chunk schedule.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>

#include "exact.h"
#include "perm_internal.h"

namespace permx {

const DeviceShape &device_shape() {
    static DeviceShape s;  // MI355X: 256 CUs x 4 SIMDs, 512 VGPRs per lane per SIMD
    return s;
}

// ---------------------------------------------------------------------------
// Alg. 4 (PermanentOrdering, Sec. V).  Repeatedly choose the column with the
// fewest nonzeros in rows not yet ordered (lowest index on ties), then order
// its not-yet-ordered rows (ascending row index).  Each newly ordered row
// lowers the count of every not-yet-chosen column it touches.  Rows that no
// column touches (empty rows) go last, ascending.
// ---------------------------------------------------------------------------
void permanent_ordering(const Ccs &a, std::vector<int> &rowPerm, std::vector<int> &colPerm) {
    const int n = a.n;
    // row -> columns (CSR pattern)
    std::vector<int> rptr(n + 1, 0), cids(a.nnz());
    for (int p = 0; p < a.nnz(); ++p) rptr[a.rowidx[p] + 1]++;
    for (int i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
    {
        std::vector<int> fill(rptr.begin(), rptr.end() - 1);
        for (int j = 0; j < n; ++j)
            for (int p = a.colptr[j]; p < a.colptr[j + 1]; ++p) cids[fill[a.rowidx[p]]++] = j;
    }
    std::vector<int> unordered_count(n);
    std::vector<char> chosen(n, 0), ordered(n, 0);
    for (int j = 0; j < n; ++j) unordered_count[j] = a.colptr[j + 1] - a.colptr[j];
    rowPerm.clear();
    colPerm.clear();
    for (int step = 0; step < n; ++step) {
        int best = -1;
        for (int j = 0; j < n; ++j)
            if (!chosen[j] && (best < 0 || unordered_count[j] < unordered_count[best])) best = j;
        chosen[best] = 1;
        colPerm.push_back(best);
        for (int p = a.colptr[best]; p < a.colptr[best + 1]; ++p) {
            const int r = a.rowidx[p];
            if (ordered[r]) continue;
            ordered[r] = 1;
            rowPerm.push_back(r);
            for (int q = rptr[r]; q < rptr[r + 1]; ++q)
                if (!chosen[cids[q]]) unordered_count[cids[q]]--;
        }
    }
    for (int i = 0; i < n; ++i)
        if (!ordered[i]) rowPerm.push_back(i);
}

// Ascending column degree (the degree sort of Sec. VI-B), rows unchanged.
void degree_ordering(const Ccs &a, std::vector<int> &rowPerm, std::vector<int> &colPerm) {
    const int n = a.n;
    rowPerm.resize(n);
    colPerm.resize(n);
    for (int i = 0; i < n; ++i) rowPerm[i] = colPerm[i] = i;
    std::stable_sort(colPerm.begin(), colPerm.end(), [&](int x, int y) {
        return a.colptr[x + 1] - a.colptr[x] < a.colptr[y + 1] - a.colptr[y];
    });
}

// ---------------------------------------------------------------------------
// Alg. 5 (Partitioning, Sec. V).  For each prefix of columns 0..j: nrows is
// the largest row index touched so far plus one, x needs 2*nrows 32-bit
// registers, register updates cost 2*nrows*(1 - 2^-(j+1)), global updates
// (n - nrows) * 2^-(j+1) * GRratio; the score is tau(registers) divided by
// their sum.  A better score, or a column that adds no row (nrows == k),
// moves the boundary to k = nrows, c = j + 1.
// ---------------------------------------------------------------------------
void partitioning(const Ccs &ordered, const double *tau, double gr_ratio, int *k_out, int *c_out) {
    const int n = ordered.n;
    int k = 0, c = 0, nrows = 0;
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        int top = 0;
        for (int p = ordered.colptr[j]; p < ordered.colptr[j + 1]; ++p) top = std::max(top, ordered.rowidx[p] + 1);
        nrows = std::max(nrows, top);
        const int regs = 2 * nrows;
        const double freq = std::ldexp(1.0, -(j + 1));
        const double reg_cost = regs * (1.0 - freq);
        const double glob_cost = (n - nrows) * freq * gr_ratio;
        const double score = tau[regs] / (reg_cost + glob_cost);
        if (score > best || nrows == k) {
            best = score;
            k = nrows;
            c = j + 1;
        }
    }
    *k_out = k;
    *c_out = c;
}

// CalculateNoThreads of Alg. 5 for gfx950: threads resident on the device when
// each lane holds r registers of x on top of the kernel's other registers.
// VGPRs are allocated in granules of 8; a SIMD holds 512 per lane and at most
// 8 waves.
std::vector<double> tau_model(int n, int base_vgprs) {
    const DeviceShape &d = device_shape();
    std::vector<double> tau(2 * n + 1);
    for (int r = 0; r <= 2 * n; ++r) {
        const int v = (base_vgprs + r + 7) / 8 * 8;
        const int waves = std::min(d.max_waves_per_simd, d.vgprs_per_simd_lane / v);
        tau[r] = (double)d.cus * d.simds_per_cu * waves * 64;
    }
    return tau;
}

namespace {

// VGPRs a lane needs besides x and the cached products: two accumulators,
// the lane sign, chunk index, temporaries of the product trees and the
// reduction.  The AUTO level budget uses it as is; Alg. 5's thread-count
// model starts from it and is then given the count measured from the
// compiled HYBRID kernel (its VGPRs minus two per register row: 74..132 on
// n = 24..44 matrices, far above this estimate, because the cold rows'
// loaded values and the product tree's temporaries stay in registers).
constexpr int kBaseVgprs = 28;
// Exact mode's further registers in the plan's budget: the residue and |term|
// accumulators and the prime with its reciprocal.  (The compiler's count did
// not follow the level count here: the n = 40 0/1 kernel took 136 VGPRs with
// 12 levels and 138 with 9.)
constexpr int kExactBaseVgprs = 6;

// Chunk log2 (Gray steps per lane) and static block log2, measured on
// MI355X.  All-terms kernels: about 2^21 lanes (8 resident rounds of the 4096
// wave slots at 4 waves per SIMD), chunks of 2^8 .. 2^14 steps, blocks of
// 2^7 (the paper's grid n = 40, p = 0.1 .. 0.5, and a real n = 36 matrix:
// 2.5 % less time than 2^18 / 2^6 over all six, 20 % at n = 36).  Pruning
// kernels (zero-aware skipping): about 2^23 lanes, at most 2^16 steps, blocks
// of 2^6, since shorter chunks let more whole chunks and intervals be pruned
// (three n = 40 0/1 matrices: 19 ms in all against 25 ms at 2^18).  At least
// 2^(n-30) steps, so that the partial sums stay at 2^21 workgroups (32 MiB)
// or fewer up to n = 60, and at most 2^30 (the kernel's limit).
int auto_kappa(int n, bool zero_skip) {
    const int total = n - 1;  // log2 of the number of Gray indices
    int kappa = total - (zero_skip ? 23 : 21);
    kappa = std::max(kappa, std::min(total, 8));
    kappa = std::min(kappa, zero_skip ? 16 : 14);
    kappa = std::max(kappa, total - 31);  // at most 2^31 chunks (2^23 workgroups of partials)
    return std::min(kappa, std::min(total, 30));
}

int auto_unroll(bool zero_skip) { return zero_skip ? 6 : 7; }

// Automatic chunk size of a matrix that the plan can pair (AUTO, every term,
// FP64, column 0 with one or two entries): 2^15 Gray steps once that leaves
// at least 2^21 chunks (n >= 37), so that the whole chunk is one static
// block of 2^13 paired steps whose first 13 columns can be copied (n = 40:
// 0.080 FP64 operations per term against 0.090 at 2^14, 1.85 ms against
// 2.15).  Otherwise auto_kappa's.
int auto_kappa_plan(const Ccs &B, const perm_opts &o, bool zero_skip, bool exact) {
    const int n = B.n;
    int kappa = auto_kappa(n, zero_skip);
    const int d0 = n >= 2 ? B.colptr[1] - B.colptr[0] : 0;
    if (o.mode == PERM_MODE_AUTO && !zero_skip && !exact && (d0 == 1 || d0 == 2) && n - 1 - 15 >= 21)
        kappa = std::max(kappa, 15);
    return kappa;
}

// Copies of the most frequent columns' rows (nested kernels): at most this
// many extra doubles per lane in the automatic choice.  With pairing the
// matrices are sparse, values the loop never changes leave it, and one
// wave per SIMD with the fewest operations is fastest (n = 40: copies of
// 12 columns in 354 VGPRs, 2.3 ms, against 3.3 ms with 10 in 304); without
// pairing the rows are dense and the rest of the kernel takes more
// registers (n = 36, d = 0.30: copies of 6 columns spill, of 4 fit 336
// VGPRs).
constexpr int kMaxCopyValuesPaired = 400;
constexpr int kMaxCopyValues = 112;
// exact mode (paired): the copies' values with the levels' residues; 128
// keeps the n = 40 workload's kernel within 256 VGPRs (two waves per SIMD)
constexpr int kMaxCopyValuesExact = 128;

// Nested kernels without pairing replace the cached products only at this
// fraction of their FP64 operations or below (see make_plan).
constexpr double kNestedGain = 0.6;

// Largest static block (log2) of kernels other than nested ones with pairing.
constexpr int kMaxUnrollCached = 9;

// Paired FP64 kernels take static blocks beyond 2^9 steps by default only
// when their best count at 2^9 is at most this many FP64 operations per
// term (n = 40, d = 0.10: 0.35; ER n = 40..45, p = 0.1: 0.11..0.15; a
// column-0 pair in ER n = 40..45, p = 0.2..0.3: 1.7..4.2).
constexpr double kBigBlockMaxOps = 0.6;

// The extra doubles the copies of the walk's first m columns keep (the
// generator's layout: rows, multi-row levels, the tracked bracket).
int copy_values(const Plan *p, int m) {
    const Ccs &B = p->B;
    const int cbase = p->pair0 ? 1 : 0;
    const bool dtrack = p->pair0 && B.colptr[1] - B.colptr[0] == 2;
    std::vector<unsigned> Tr(p->n, 0u), Tl(p->nlevels, 0u);
    std::vector<int> lsize(p->nlevels, 0);
    unsigned T0 = 0u;
    for (int r = 0; r < p->n; ++r) lsize[p->row_level[r]]++;
    for (int c = cbase; c < cbase + m && c < p->n; ++c)
        for (int q = B.colptr[c]; q < B.colptr[c + 1]; ++q) {
            const int r = B.rowidx[q];
            if (p->pair0 && p->row_level[r] == 0) {
                if (dtrack) T0 |= 1u << (c - cbase);
            } else {
                Tr[r] |= 1u << (c - cbase);
                Tl[p->row_level[r]] |= 1u << (c - cbase);
            }
        }
    long cv = 0;
    for (int r = 0; r < p->n; ++r) cv += (1l << __builtin_popcount(Tr[r])) - 1;
    // a level's copies (exact mode: with their residues)
    for (int l = 1; l < p->nlevels; ++l)
        if (lsize[l] > 1) cv += ((1l << __builtin_popcount(Tl[l])) - 1) * (p->exact ? 2 : 1);
    cv += (1l << __builtin_popcount(T0)) - 1;
    return (int)std::min<long>(cv, INT_MAX);
}

// The number m of the walk's first columns whose rows are kept in copies
// (nested kernels): the generator counts the FP64 operations of candidate
// step loops (the flips of copied columns leave every value unchanged, so
// much of what follows them depends only on values the loop never changes
// and leaves the loop).  Candidates: the largest m whose copies fit the
// register allowance (more copied columns almost always mean fewer
// operations) and the two below it; the fewest operations win, a further
// column having to save at least 1 %.  copy_cols forces m (-1: none).  *base
// gets the count without copies.  Returns -1 if nothing was counted.
int choose_copies(const Plan *p, const perm_opts &o, int mmax, LoopCount *best, LoopCount *base, int cap = 0) {
    mmax = p->u >= 1 ? std::max(0, mmax) : 0;
    const int want = o.copy_cols < 0 ? 0 : o.copy_cols > 0 ? std::min(o.copy_cols, mmax) : -1;
    if (cap <= 0) cap = p->exact ? kMaxCopyValuesExact : p->pair0 ? kMaxCopyValuesPaired : kMaxCopyValues;
    std::vector<int> cands;
    if (want >= 0) {
        cands.push_back(want);
    } else {
        int top = mmax;
        while (top > 0 && copy_values(p, top) > cap) --top;
        for (int m = std::max(0, top - 2); m <= top; ++m) cands.push_back(m);
    }
    if (cands.front() != 0) cands.insert(cands.begin(), 0);  // the count without copies, for *base
    int mbest = -1;
    for (int m : cands) {
        Plan q = *p;
        q.copy_cols = m;
        LoopCount lc;
        generate_source(q, &lc);
        if (!lc.counted) continue;
        if (m == 0 && base) *base = lc;
        if (want >= 0 && m != want) continue;
        if (mbest < 0 || lc.ops_per_step < 0.99 * best->ops_per_step) {
            mbest = m;
            *best = lc;
        }
    }
    return mbest;
}

bool integer_valued(const Ccs &a) {
    for (double v : a.val)
        if (v != std::floor(v)) return false;
    return true;
}

}  // namespace

perm_status make_plan(const Ccs &a, const perm_opts &o, Plan *p, std::string *err, int tau_base) {
    char buf[256];
    const int n = a.n;
    p->n = n;
    p->nnz = a.nnz();
    p->mode = o.mode;
    // x_i is an exact zero at many Gray indices only when the values are
    // integers (then 2 x_i is an integer); real-valued inputs almost never
    // produce one, and the checks would only cost registers.  0 = auto.
    const bool zs = o.zero_skip > 0 ? true : o.zero_skip < 0 ? false : integer_valued(a);
    if (o.mode < PERM_MODE_AUTO || o.mode > PERM_MODE_HYBRID) {
        *err = "unknown mode";
        return PERM_EINVAL;
    }
    // Exact mode: every value an integer, and every row's |y| bound (the sum
    // of its |a|) within one sub-product bound.  0 = auto (on when possible).
    if (o.exact < -1 || o.exact > 1) {
        *err = "exact must be -1 (off), 0 (automatic) or 1 (required)";
        return PERM_EINVAL;
    }
    bool ex = false;
    if (o.exact >= 0) {
        bool ok = integer_valued(a);
        std::vector<double> rowabs(n, 0.0);
        for (int q = 0; q < a.nnz(); ++q) rowabs[a.rowidx[q]] += std::fabs(a.val[q]);
        for (int r = 0; r < n && ok; ++r) ok = rowabs[r] <= kExactPartMax;
        if (o.exact == 1 && !ok) {
            *err = "exact = 1 needs integer values with every row's sum of |a| at most 2^20";
            return PERM_EINVAL;
        }
        ex = ok;
    }
    if (o.mode == PERM_MODE_PURE)
        degree_ordering(a, p->rowPerm, p->colPerm);
    else
        permanent_ordering(a, p->rowPerm, p->colPerm);
    p->B = permute(a, p->rowPerm, p->colPerm);
    if (ex)
        for (double &v : p->B.val) v *= 2.0;  // y = 2x: every x update and start value an integer
    p->exact = ex;
    const Ccs &B = p->B;

    // first flipped column (0..n-2) touching each ordered row; n-1 if none
    std::vector<int> first(n, n - 1);
    for (int j = 0; j < n - 1; ++j)
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) first[B.rowidx[q]] = std::min(first[B.rowidx[q]], j);

    const double gr = o.gr_ratio > 0 ? o.gr_ratio : 16.0;
    const int budget = o.vgpr_budget > 0 ? o.vgpr_budget : 128;
    p->tau_base = tau_base > 0 ? tau_base : kBaseVgprs;
    std::vector<double> tau = tau_model(n, p->tau_base);
    int k5 = n, c5 = n;
    partitioning(B, tau.data(), gr, &k5, &c5);

    // ---- register / global split ----
    int k = n, c = n - 1;
    if (o.mode == PERM_MODE_HYBRID) {
        k = k5;
        c = std::min(c5, n - 1);
        if (o.force_k > 0 || o.force_c > 0) {
            if (o.force_k <= 0 || o.force_c <= 0 || o.force_k > n || o.force_c > n) {
                *err = "force_k and force_c must both be in [1, n]";
                return PERM_EINVAL;
            }
            k = o.force_k;
            c = std::min(o.force_c, n - 1);
        }
    }
    // AUTO keeps all of x in VGPRs: at n <= 64 that is at most 128 registers,
    // which a gfx950 lane can hold with 3 or more waves per SIMD.
    // every row touched by a register-only column must be a register row
    for (int j = 0; j < c; ++j)
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q)
            if (B.rowidx[q] >= k) {
                snprintf(buf, sizeof buf, "partition (k=%d, c=%d) invalid: column %d touches row %d", k, c, j,
                         B.rowidx[q]);
                *err = buf;
                return PERM_EINVAL;
            }
    p->k = k;
    p->c = c;
    p->cold = k < n;

    // ---- levels ----
    // register rows [0, k) are grouped by the first flipped column that
    // touches them; the cold rows, if any, form the last level.
    std::vector<int> lev_begin;  // first column of each register level
    if (o.mode == PERM_MODE_AUTO) {
        std::vector<int> firsts;
        for (int r = 0; r < k; ++r) firsts.push_back(std::min(first[r], c));
        std::sort(firsts.begin(), firsts.end());
        firsts.erase(std::unique(firsts.begin(), firsts.end()), firsts.end());
        lev_begin = firsts;
        if (lev_begin.empty() || lev_begin[0] != 0) lev_begin.insert(lev_begin.begin(), 0);
        const int cold_levels = p->cold ? 1 : 0;
        // rows that no in-chunk column (index < kappa) touches are constant
        // inside a chunk: once their level product is formed at the chunk
        // start their registers are free, so only the other rows count
        const int kap = o.chunk_log2 > 0 ? std::min(o.chunk_log2, std::max(n - 1, 0)) : auto_kappa_plan(B, o, zs, ex);
        int live_rows = 0;
        for (int r = 0; r < k; ++r)
            if (first[r] < kap) ++live_rows;
        // exact mode: a residue beside each cached product, and the residue
        // and error-bound accumulators.  With zero-aware skipping the walk
        // keeps no residues (they are formed again where terms are evaluated,
        // so their registers are live only there): 2 per level, as in FP64.
        const int per_level = (ex && !zs) ? 4 : 2;
        auto vgprs = [&](int nlev) {
            return 2 * live_rows + per_level * (nlev + cold_levels - 1) + kBaseVgprs + (ex ? kExactBaseVgprs : 0);
        };
        int cap = o.max_levels > 0 ? o.max_levels : INT_MAX;
        while ((int)lev_begin.size() > 1 && ((int)lev_begin.size() > cap || vgprs((int)lev_begin.size()) > budget))
            lev_begin.pop_back();  // merge the two highest (least often touched) levels
    } else {
        lev_begin = {0};  // PURE, HYBRID: one register level (the paper's register product)
    }
    const int nreg_levels = (int)lev_begin.size();
    p->nlevels = nreg_levels + (p->cold ? 1 : 0);
    p->lev_begin = lev_begin;
    if (p->cold) p->lev_begin.push_back(c);
    p->lev_begin.push_back(n);
    p->row_level.assign(n, 0);
    for (int r = 0; r < n; ++r) {
        if (r >= k) {
            p->row_level[r] = p->nlevels - 1;
            continue;
        }
        const int f = std::min(first[r], c);
        int l = 0;
        while (l + 1 < nreg_levels && lev_begin[l + 1] <= f) ++l;
        p->row_level[r] = l;
    }
    // exact mode: each level's rows in consecutive sub-products whose bound
    // (product of the rows' sums of |a|) stays within kExactPartMax
    if (ex) {
        std::vector<double> bound(n, 0.0);
        for (int q = 0; q < B.nnz(); ++q) bound[B.rowidx[q]] += std::fabs(B.val[q]) / 2;
        p->level_parts.assign(p->nlevels, {});
        std::vector<double> cur(p->nlevels, 0.0);
        for (int r = 0; r < n; ++r) {
            const int l = p->row_level[r];
            auto &parts = p->level_parts[l];
            if (parts.empty() || cur[l] * bound[r] > kExactPartMax) {
                parts.push_back({});
                cur[l] = 1.0;
            }
            parts.back().push_back(r);
            cur[l] *= bound[r];
        }
    }
    p->col_top.assign(n, 0);
    for (int j = 0; j < n - 1; ++j) {
        int t = 0;
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) t = std::max(t, p->row_level[B.rowidx[q]]);
        p->col_top[j] = t;
    }

    // ---- x at Gray index 0 (Alg. 1's initialisation, with a_{i,n-1} = 0 when absent) ----
    {
        std::vector<long double> rowsum(n, 0.0L), last(n, 0.0L);
        for (int j = 0; j < n; ++j)
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
                rowsum[B.rowidx[q]] += (long double)B.val[q];
                if (j == n - 1) last[B.rowidx[q]] = (long double)B.val[q];
            }
        for (int r = 0; r < n; ++r) p->base_x_hi[r] = (double)(last[r] - rowsum[r] / 2);
    }

    // ---- schedule ----
    const int total_log2 = n - 1;
    p->kappa = o.chunk_log2 > 0 ? o.chunk_log2 : auto_kappa_plan(B, o, zs, ex);
    if (p->kappa > total_log2) p->kappa = total_log2;
    if (p->kappa > 30) {
        *err = "chunk_log2 must be <= 30";
        return PERM_EINVAL;
    }
    if (total_log2 - p->kappa > 40) {
        *err = "too many chunks: raise chunk_log2";
        return PERM_ETOOBIG;
    }
    p->u = o.unroll_log2 > 0 ? o.unroll_log2 : auto_unroll(zs);
    if (p->u > 13) {
        *err = "unroll_log2 must be <= 13";
        return PERM_EINVAL;
    }
    p->u = std::max(0, std::min(p->u, p->kappa - 1));
    p->block = o.block > 0 ? o.block : 256;
    if (o.cold_tier < 0 || o.cold_tier > 1) {
        *err = "cold_tier must be 0 (global memory) or 1 (LDS)";
        return PERM_EINVAL;
    }
    p->cold_lds = p->cold && o.cold_tier == 1;
    if (p->cold_lds) {
        // [row][lane] doubles per workgroup: at most 40 KiB by default (four
        // workgroups per CU in 160 KiB), at most 64 KiB when the block is given
        const int64_t lane_bytes = 8 * (int64_t)(n - p->k);
        if (o.block <= 0) {
            int b = 256;
            while (b > 64 && (int64_t)b * lane_bytes > 40960) b -= 64;
            p->block = b;
        }
        if ((int64_t)p->block * lane_bytes > 65536) {
            *err = "cold rows do not fit LDS at this block size";
            return PERM_EINVAL;
        }
    }
    p->zero_skip = zs;
    if (o.waves_per_simd < -1 || o.waves_per_simd > 8) {
        *err = "waves_per_simd must be -1 (compiler's choice), 0 (automatic) or 1..8";
        return PERM_EINVAL;
    }
    p->waves_per_simd = std::max(0, o.waves_per_simd);
    if (o.copy_cols < -1 || o.copy_cols > 13) {
        *err = "copy_cols must be -1 (none), 0 (automatic) or 1..13";
        return PERM_EINVAL;
    }
    if (!(o.block_queue == -1 || o.block_queue == 0 || o.block_queue == 8 || o.block_queue == 16 ||
          o.block_queue == 32 || o.block_queue == 64)) {
        *err = "block_queue must be -1 (off), 0 (automatic) or 8, 16, 32, 64 slots per wave";
        return PERM_EINVAL;
    }
    p->queue_slots = o.block_queue;
    if (p->block % 64 != 0 || p->block > 1024) {
        *err = "block must be a multiple of 64 and at most 1024";
        return PERM_EINVAL;
    }
    // column-0 pairing (AUTO, every term evaluated, FP64): level 0 is then
    // exactly column 0's rows (the rows first touched by column 0)
    p->pair0 = false;
    {
        const int d0 = n >= 2 ? B.colptr[1] - B.colptr[0] : 0;
        bool ok = o.mode == PERM_MODE_AUTO && !zs && !p->cold && p->nlevels >= 2 && p->kappa >= 3 &&
                  (d0 == 1 || d0 == 2);
        for (int r = 0; r < n && ok; ++r)
            if ((p->row_level[r] == 0) != (first[r] == 0)) ok = false;
        if (ok && ex) {
            // exact mode: the bracket (an integer in y units) must stay within
            // kExactPartMax, like any sub-product whose residue is formed
            std::vector<double> yb(n, 0.0);  // |y_r| <= half the row's sum of |2a|
            for (int q = 0; q < B.nnz(); ++q) yb[B.rowidx[q]] += std::fabs(B.val[q]) / 2;
            const int q0 = B.colptr[0];
            double bd = std::fabs(B.val[q0]);
            if (d0 == 2) {
                const double ar = std::fabs(B.val[q0]), as = std::fabs(B.val[q0 + 1]);
                bd = ar * yb[B.rowidx[q0 + 1]] + as * yb[B.rowidx[q0]] + ar * as;
            }
            if (bd > kExactPartMax) ok = false;
        }
        if (ok) {
            p->pair0 = true;
            // nested kernels: static blocks as long as the chunk allows, up
            // to 2^13 paired steps (FP64) or 2^9 (exact: the residues take
            // registers of their own, fewer columns are copied), by default
            // (the more of the walk's columns are static, the more can be
            // kept in copies)
            if (o.unroll_log2 == 0) p->u = ex ? 9 : 13;
            p->u = std::min(p->u, p->kappa - 2);  // a static block of paired steps fits the chunk's half
            // FP64: 64-lane workgroups by default (n = 40: 1.76-1.81 ms
            // against 1.82-1.84 with 256; the code per lane is the same)
            if (!ex && o.block <= 0) p->block = 64;
            // two entries: the row that lower (more often flipped) columns
            // touch goes in the outer FMA of the bracket, so that a flip of
            // it alone costs one operation
            p->pair_r = B.rowidx[B.colptr[0]];
            p->pair_s = d0 == 2 ? B.rowidx[B.colptr[0] + 1] : -1;
            if (d0 == 2) {
                int fr = n, fs = n;
                for (int j = n - 2; j >= 1; --j)
                    for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
                        if (B.rowidx[q] == p->pair_r) fr = j;
                        if (B.rowidx[q] == p->pair_s) fs = j;
                    }
                if (fr < fs) std::swap(p->pair_r, p->pair_s);
            }
        }
    }

    // ---- FP64 operations per step (matches what generate_source emits) ----
    std::vector<int> level_size(p->nlevels, 0);
    for (int r = 0; r < n; ++r) level_size[p->row_level[r]]++;
    p->ops_of_col.assign(n, 0.0);
    double ops = 0.0, exact_ops = 0.0;
    const double steps = std::ldexp(1.0, n - 1);
    const int L = p->nlevels;
    // A level that the flipped column does not touch keeps its x values, so
    // the compiler reuses that level's product from the previous step (the
    // same values); only touched levels' products and the chain multiplies
    // S_l = P_l * S_{l+1}, l <= top, are executed.
    std::vector<char> touched(L, 0);
    for (int j = 0; j < n - 1; ++j) {
        const int t = p->col_top[j];
        std::fill(touched.begin(), touched.end(), 0);
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) touched[p->row_level[B.rowidx[q]]] = 1;
        double oj = B.colptr[j + 1] - B.colptr[j];  // x updates
        for (int l = 0; l <= t; ++l)
            if (touched[l]) oj += std::max(0, level_size[l] - 1);
        for (int l = 1; l <= t; ++l)
            if (l < L - 1) oj += 1;  // chain multiply by S_{l+1}
        if (L > 1) oj += 1;          // accumulate: fma(P_0, S_1, acc)
        if (ex) {
            // residue chain: one reduction (4 operations) per sub-product of
            // each refreshed level (the top level's first needs none), the
            // level-0 sub-products but one, then the residue FMA and the two
            // error-bound sums
            double xo = 0.0;
            for (int l = 1; l <= t; ++l) xo += 4.0 * ((double)p->level_parts[l].size() - (l + 1 < L ? 0.0 : 1.0));
            xo += 4.0 * ((double)p->level_parts[0].size() - 1.0) + 3.0;
            oj += xo;
            exact_ops += std::ldexp(1.0, n - j - 2) * xo;
        }
        p->ops_of_col[j] = oj;
        ops += std::ldexp(1.0, n - j - 2) * oj;
    }
    p->ops_per_step = ops / steps;
    p->exact_ops_per_step = exact_ops / steps;
    // the accumulate FMA replaces a multiply and an add of Alg. 1 (counts 2)
    p->flops_per_step = (ops + (steps - 1.0)) / steps;
    if (p->pair0) {
        // Paired walk: column 0 never flips; a step flipping column j >= 1
        // updates its rows, refreshes the levels above 0 as before, forms
        // P(x) - P(x + a) of level 0 only when the column touches level 0
        // (else the compiler reuses it: two FMAs for two rows, a literal for
        // one) and adds the pair with one FMA (exact mode) or through the
        // nested accumulators (FP64).  Each FMA of the two-row difference,
        // the accumulate and the accumulators' moves does a multiply and an
        // add the sum needs (2 flops each).
        const int d0 = B.colptr[1] - B.colptr[0];
        // nested form: FP64, and the exact mode too (residues and |term|
        // sums move up beside the FP64 accumulators)
        const bool nest = L >= 2;
        double pops = 0.0, pfl = 0.0, pxo = 0.0;
        for (int j = 1; j < n - 1; ++j) {
            const int t = p->col_top[j];
            std::fill(touched.begin(), touched.end(), 0);
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) touched[p->row_level[B.rowidx[q]]] = 1;
            // x updates (nested accumulation: level 0 lives in the bracket)
            double oj = 0.0;
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q)
                if (!nest || p->row_level[B.rowidx[q]] != 0) oj += 1.0;
            for (int l = 1; l <= t; ++l)
                if (touched[l]) oj += std::max(0, level_size[l] - 1);
            if (nest) {
                // nested accumulation: c_0 .. c_{t-1} move up through the
                // level products (t operations) and the bracket starts c_0;
                // with no level above 0 touched, the bracket adds to c_0
                oj += t > 0 ? t : 1;
            } else {
                for (int l = 1; l <= t; ++l)
                    if (l < L - 1) oj += 1;  // chain multiply by S_{l+1}
                oj += 1;                     // accumulate: fma(bracket, S_1, acc)
            }
            // the bracket fma(a_r, x_s, fma(a_s, x_r, a_r a_s)): the inner
            // FMA only when x_r changed, the outer when either did; nested
            // accumulation keeps the bracket itself (one add of a constant)
            double bops = 0.0;
            if (nest) {
                if (d0 == 2 && touched[0]) oj += 1.0;
            } else if (d0 == 2) {
                bool tr = false, ts = false;
                for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
                    tr = tr || B.rowidx[q] == p->pair_r;
                    ts = ts || B.rowidx[q] == p->pair_s;
                }
                bops = tr ? 2.0 : ts ? 1.0 : 0.0;
            }
            oj += bops;
            const double cnt = std::ldexp(1.0, n - j - 2);
            double xo = 0.0;
            if (ex) {
                // residue chain of the refreshed levels (four operations per
                // sub-product, the top level's first needs none), then the
                // pair's residue FMA and the error bound's FMA
                for (int l = 1; l <= t; ++l)
                    xo += 4.0 * ((double)p->level_parts[l].size() - (l + 1 < L ? 0.0 : 1.0));
                xo += 2.0;
                oj += xo;
                pxo += cnt * xo;
            }
            p->ops_of_col[j] = oj;
            pops += cnt * oj;
            pfl += cnt * (oj + bops + (nest ? 0.0 : 1.0));
        }
        p->copy_cols = 0;
        p->nested = nest;
        if (nest) {
            LoopCount best;
            int m = -2;
            if (!ex && o.unroll_log2 == 0 && p->u > kMaxUnrollCached) {
                // the long default block only where the copies leave few
                // operations: the count at 2^9-step blocks (copies within the
                // allowance of dense rows) decides; above kBigBlockMaxOps the
                // plan keeps those blocks and copies (a chunk-long block of a
                // denser matrix is code the compiler takes minutes over, and
                // its copies spill)
                Plan q = *p;
                q.u = kMaxUnrollCached;
                LoopCount small;
                const int ms = choose_copies(&q, o, std::min(q.u, n - 2), &small, nullptr, kMaxCopyValues);
                if (ms >= 0 && small.ops_per_step > kBigBlockMaxOps) {
                    p->u = q.u;
                    m = ms;
                    best = small;
                }
            }
            if (m == -2) m = choose_copies(p, o, std::min(p->u, n - 2), &best, nullptr);
            if (m >= 0) {
                p->copy_cols = m;
                pops = best.ops_per_step * steps;
                pfl = best.flops_per_step * steps;
                if (ex) pxo = 0.0;  // counted with the rest
                p->acc_log2 = best.acc_log2;
            }
            if (ex && p->acc_log2 == 0) {
                // no count: each of a chunk's paired steps moves at most L
                // accumulators and adds one bracket
                const double F = std::ldexp(1.0, p->kappa - 1) * (L + 1) + n + 2;
                while (std::ldexp(1.0, p->acc_log2) < F) ++p->acc_log2;
            }
        }
        p->ops_of_col[0] = 0.0;
        p->ops_per_step = pops / steps;
        p->flops_per_step = pfl / steps;
        p->exact_ops_per_step = pxo / steps;
    }
    // Static blocks beyond 2^9 steps only for nested kernels with pairing
    // (other kernels' blocks of that size compile for minutes and gain
    // nothing): larger values given are reduced.
    if (!(p->pair0 && p->nested)) p->u = std::min(p->u, kMaxUnrollCached);
    // Nested accumulation without pairing (AUTO, all terms, FP64): level 0's
    // own product starts c_0, and the copied columns are 0..m-1.  Taken when
    // the generator's count of its best form is at most kNestedGain of the
    // cached products': these kernels' copies of dense rows take most of
    // the registers (one wave per SIMD at n = 36..40, densities 0.2..0.5,
    // 51-69 % FP64 issue against about 90 % for the cached products), so
    // fewer operations pay only when they are clearly fewer (ER n = 40:
    // 0.39 of the count at p = 0.3 ran 1.4x faster, 0.65 at p = 0.5 14 %
    // slower).  Copies asked for (copy_cols > 0) take the nested form.
    if (!p->pair0 && o.mode == PERM_MODE_AUTO && !zs && !ex && !p->cold && L >= 2 && p->kappa >= 2) {
        Plan q = *p;
        q.nested = true;
        // static blocks of 2^6 steps by default: without pairing the steps
        // are denser, and longer blocks compile slowly for little gain
        if (o.unroll_log2 == 0) q.u = std::max(0, std::min(6, p->kappa - 1));
        q.u = std::min(q.u, kMaxUnrollCached);
        LoopCount best;
        const int m = choose_copies(&q, o, std::min(q.u, n - 1), &best, nullptr);
        if (m >= 0 && (o.copy_cols > 0 || best.ops_per_step <= kNestedGain * p->ops_per_step)) {
            *p = q;
            p->copy_cols = m;
            p->ops_per_step = best.ops_per_step;
            p->flops_per_step = best.flops_per_step;
        }
    }
    return PERM_OK;
}

}  // namespace permx
