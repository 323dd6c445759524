/*
 * perm_oracle.c -- reference CPU implementation of the permanent of a sparse
 * n x n matrix, used ONLY as test infrastructure.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The product path (the HIP library under
 * paper_2501_15126_amd/) never links, includes or calls it, and this file
 * shares no code, header, table or helper with that path.  Inputs are plain
 * arrays; the seeded input generators live in their own module.
 *
 * Everything here is written to be checked by eye against the paper
 * (Elbek & Kaya, "Fully-Automated Code Generation for Efficient Computation of
 * Sparse Matrix Permanents on GPUs", arXiv 2501.15126):
 *
 *   oracle_perm_brute      Eq. (1): sum over all permutations.
 *   oracle_perm_ryser      Eq. (2): Ryser's inclusion-exclusion over all 2^n
 *                          column subsets, no Gray code.
 *   oracle_nw_range        Alg. 1 (SparsePerman, Sec. II): the Nijenhuis-Wilf
 *                          variant in Gray-code order, evaluated over a range
 *                          of Gray indices, in long double.
 *   oracle_nw_int_range    the same sum for 0/1 matrices in exact integer
 *                          arithmetic (2x is an integer), with zero skipping.
 *   oracle_gray / oracle_changed_bit
 *                          Gray code and the (j, s) pair of Alg. 1, taken from
 *                          the XOR definition (not from Theorem 1).
 *   oracle_permanent_ordering  Alg. 4 (PermanentOrdering, Sec. V).
 *   oracle_partitioning        Alg. 5 (Partitioning, Sec. V).
 *   oracle_structural_rank     size of a maximum matching of the bipartite
 *                              row/column graph (perm = 0 when it is < n).
 *
 * Readings of the paper taken here (each one is listed with its reason in the
 * project's design notes):
 *   - Indices are 0-based.  Column n-1 is the fixed Nijenhuis-Wilf column;
 *     Gray codes have n-1 bits and flip columns 0..n-2.
 *   - The x initialisation of Alg. 1 is x_i = a_{i,n-1} - (sum_j a_ij)/2 with
 *     a_{i,n-1} = 0 when row i has no entry in column n-1 (the printed line
 *     reads the last stored entry of the row, which is a_{i,n-1} only when
 *     that entry exists).
 *   - Term g (0 <= g < 2^(n-1)) is (-1)^g * prod_i x_i(Gray_g), where x(S) is
 *     the initial x plus the columns in S.  Term 0 is the initial product of
 *     Alg. 1; the loop adds terms 1..2^(n-1)-1.  The permanent is the sum of
 *     all terms times (4 (n mod 2) - 2).
 *   - A range [g_begin, g_end) starts from x(Gray_{g_begin}) built directly,
 *     as the chunked parallel scheme of Sec. II-A does for each thread.
 *
 * Floating point: long double (x87 80-bit, 64-bit significand) throughout.
 * Threads: a range is split into T equal contiguous sub-ranges, one per
 * thread, each restarting x at its first index; the T partial sums are added
 * in thread order, so a result depends only on (input, range, T).
 */
#include <limits.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_N 64

typedef long double ld;

/* ------------------------------------------------------------------------ */
/* Gray code, the Gray-code step of Alg. 1                                 */
/* ------------------------------------------------------------------------ */

/* Binary reflected Gray code of index g. */
uint64_t oracle_gray(uint64_t g) { return g ^ (g >> 1); }

/* For 1 <= g: the column j whose bit differs between Gray_g and Gray_{g-1}
 * (j = log2(Gray_g XOR Gray_{g-1})) and the direction s = 2 * Gray_g[j] - 1
 * (+1 = inclusion, -1 = exclusion).  Returns 0, or -1 for g = 0. */
int oracle_changed_bit(uint64_t g, int *j_out, int *s_out) {
    if (g == 0) return -1;
    uint64_t d = oracle_gray(g) ^ oracle_gray(g - 1);
    int j = 0;
    while (((d >> j) & 1u) == 0) ++j; /* log2 of a power of two */
    *j_out = j;
    *s_out = (int)(2 * ((oracle_gray(g) >> j) & 1u)) - 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): brute force over permutations (dense row-major input)           */
/* ------------------------------------------------------------------------ */

static void brute_rec(int n, const double *a, int i, int *used, ld prod, ld *acc) {
    if (i == n) {
        *acc += prod;
        return;
    }
    for (int j = 0; j < n; ++j) {
        /* a permutation that uses a zero entry contributes exactly 0 */
        if (used[j] || a[i * n + j] == 0.0) continue;
        used[j] = 1;
        brute_rec(n, a, i + 1, used, prod * (ld)a[i * n + j], acc);
        used[j] = 0;
    }
}

int oracle_perm_brute(int n, const double *a, double *hi, double *lo) {
    if (n < 1 || n > 12) return -1;
    int used[12] = {0};
    ld acc = 0;
    brute_rec(n, a, 0, used, 1.0L, &acc);
    *hi = (double)acc;
    *lo = (double)(acc - (ld)*hi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (2): Ryser over every subset S of {0..n-1} (dense row-major input)   */
/* ------------------------------------------------------------------------ */

int oracle_perm_ryser(int n, const double *a, double *hi, double *lo) {
    if (n < 1 || n > 24) return -1;
    ld total = 0;
    for (uint64_t S = 0; S < (1ull << n); ++S) {
        ld prod = 1;
        int card = 0;
        for (int j = 0; j < n; ++j) card += (int)((S >> j) & 1u);
        for (int i = 0; i < n; ++i) {
            ld rowsum = 0;
            for (int j = 0; j < n; ++j)
                if ((S >> j) & 1u) rowsum += (ld)a[i * n + j];
            prod *= rowsum;
        }
        total += (card % 2 == 1) ? -prod : prod;
    }
    if (n % 2 == 1) total = -total;
    *hi = (double)total;
    *lo = (double)(total - (ld)*hi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* CCS input checks shared by the sparse entry points of this file          */
/* ------------------------------------------------------------------------ */

static int ccs_ok(int n, const int *colptr, const int *rowidx) {
    if (n < 1 || n > ORACLE_MAX_N || colptr[0] != 0) return 0;
    for (int j = 0; j < n; ++j) {
        if (colptr[j + 1] < colptr[j]) return 0;
        for (int p = colptr[j]; p < colptr[j + 1]; ++p)
            if (rowidx[p] < 0 || rowidx[p] >= n) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 over a Gray-index range, long double                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    const int *colptr, *rowidx;
    const double *val;
    uint64_t b, e; /* [b, e) */
    ld sum, abs_sum;
} nw_job;

/* x(Gray_g) for the Nijenhuis-Wilf variant: the initialisation of x in Alg. 1 (under the
 * a_{i,n-1} reading), then the columns whose bit is set in Gray_g. */
static void nw_x_at(const nw_job *J, uint64_t g, ld *x) {
    int n = J->n;
    ld rowsum[ORACLE_MAX_N], last[ORACLE_MAX_N];
    for (int i = 0; i < n; ++i) rowsum[i] = last[i] = 0;
    for (int j = 0; j < n; ++j)
        for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) {
            rowsum[J->rowidx[p]] += (ld)J->val[p];
            if (j == n - 1) last[J->rowidx[p]] = (ld)J->val[p];
        }
    for (int i = 0; i < n; ++i) x[i] = last[i] - rowsum[i] / 2;
    uint64_t G = oracle_gray(g);
    for (int j = 0; j < n - 1; ++j)
        if ((G >> j) & 1u)
            for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) x[J->rowidx[p]] += (ld)J->val[p];
}

static void *nw_worker(void *arg) {
    nw_job *J = (nw_job *)arg;
    int n = J->n;
    ld x[ORACLE_MAX_N];
    ld sum = 0, abs_sum = 0;
    if (J->b < J->e) {
        nw_x_at(J, J->b, x);
        ld prod = 1;
        for (int i = 0; i < n; ++i) prod *= x[i];
        sum += (J->b % 2 == 1) ? -prod : prod;
        abs_sum += fabsl(prod);
        for (uint64_t g = J->b + 1; g < J->e; ++g) {
            int j, s;
            oracle_changed_bit(g, &j, &s);                  /* which column changes */
            for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) /* x update */
                x[J->rowidx[p]] += (ld)s * (ld)J->val[p];
            prod = 1;                                        /* product */
            for (int i = 0; i < n; ++i) prod *= x[i];
            sum += (g % 2 == 1) ? -prod : prod;              /* signed sum */
            abs_sum += fabsl(prod);
        }
    }
    J->sum = sum;
    J->abs_sum = abs_sum;
    return NULL;
}

/* Sum of terms g in [g_begin, g_end) (no final factor), plus the sum of the
 * absolute values of the same terms.  Both are returned as hi + lo double
 * pairs of the long double value. */
int oracle_nw_range(int n, const int *colptr, const int *rowidx, const double *val, uint64_t g_begin,
                    uint64_t g_end, int nthreads, double out[4]) {
    if (!ccs_ok(n, colptr, rowidx)) return -1;
    uint64_t total = 1ull << (n - 1);
    if (g_begin > g_end || g_end > total) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    nw_job jobs[256];
    pthread_t th[256];
    uint64_t len = g_end - g_begin;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].n = n;
        jobs[t].colptr = colptr;
        jobs[t].rowidx = rowidx;
        jobs[t].val = val;
        jobs[t].b = g_begin + len / (uint64_t)nthreads * (uint64_t)t + ((uint64_t)t < len % (uint64_t)nthreads ? (uint64_t)t : len % (uint64_t)nthreads);
        jobs[t].e = jobs[t].b + len / (uint64_t)nthreads + ((uint64_t)t < len % (uint64_t)nthreads ? 1u : 0u);
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, nw_worker, &jobs[t]);
    nw_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    ld sum = 0, abs_sum = 0;
    for (int t = 0; t < nthreads; ++t) {
        sum += jobs[t].sum;
        abs_sum += jobs[t].abs_sum;
    }
    out[0] = (double)sum;
    out[1] = (double)(sum - (ld)out[0]);
    out[2] = (double)abs_sum;
    out[3] = (double)(abs_sum - (ld)out[2]);
    return 0;
}

/* Permanent by Alg. 1 over the full range: the sum of all 2^(n-1) terms
 * times 4 (n mod 2) - 2 (the final scaling of Alg. 1). */
int oracle_perm_nw(int n, const int *colptr, const int *rowidx, const double *val, int nthreads,
                   double out[4]) {
    if (n < 1 || n > ORACLE_MAX_N) return -1;
    int rc = oracle_nw_range(n, colptr, rowidx, val, 0, 1ull << (n - 1), nthreads, out);
    if (rc) return rc;
    ld f = (ld)(4 * (n % 2) - 2);
    ld s = ((ld)out[0] + (ld)out[1]) * f;
    ld a = ((ld)out[2] + (ld)out[3]) * 2;
    out[0] = (double)s;
    out[1] = (double)(s - (ld)out[0]);
    out[2] = (double)a;
    out[3] = (double)(a - (ld)out[2]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 for 0/1 matrices in exact integer arithmetic                       */
/* ------------------------------------------------------------------------ */
/* With y_i = 2 x_i, every y_i is an integer: y_i = 2 a_{i,n-1} - d_i +
 * 2 |S intersect row_i| (d_i = row degree).  Term g becomes (-1)^g prod y_i =
 * 2^n times the real term, so the full sum T equals (-1)^(n-1) 2^(n-1) perm.
 * Products and sums are taken modulo 2^128 (unsigned wrap-around, exact in
 * that ring); the caller recovers T as a signed value when |T| < 2^127.  A
 * product with a zero factor is exactly zero and is skipped. */

typedef unsigned __int128 u128;

typedef struct {
    int n;
    const int *colptr, *rowidx;
    uint64_t b, e;
    u128 sum;
    uint64_t nonzero_terms;
} nwi_job;

static void *nwi_worker(void *arg) {
    nwi_job *J = (nwi_job *)arg;
    int n = J->n;
    int64_t y[ORACLE_MAX_N], deg[ORACLE_MAX_N], last[ORACLE_MAX_N];
    for (int i = 0; i < n; ++i) deg[i] = last[i] = 0;
    for (int j = 0; j < n; ++j)
        for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) {
            deg[J->rowidx[p]] += 1;
            if (j == n - 1) last[J->rowidx[p]] = 1;
        }
    u128 sum = 0;
    uint64_t nonzero_terms = 0;
    if (J->b < J->e) {
        for (int i = 0; i < n; ++i) y[i] = 2 * last[i] - deg[i];
        uint64_t G = oracle_gray(J->b);
        for (int j = 0; j < n - 1; ++j)
            if ((G >> j) & 1u)
                for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) y[J->rowidx[p]] += 2;
        int zeros = 0;
        for (int i = 0; i < n; ++i) zeros += (y[i] == 0);
        for (uint64_t g = J->b; g < J->e; ++g) {
            if (g > J->b) {
                int j, s;
                oracle_changed_bit(g, &j, &s);
                for (int p = J->colptr[j]; p < J->colptr[j + 1]; ++p) {
                    int r = J->rowidx[p];
                    zeros -= (y[r] == 0);
                    y[r] += 2 * s;
                    zeros += (y[r] == 0);
                }
            }
            if (zeros == 0) {
                u128 prod = 1;
                for (int i = 0; i < n; ++i) prod *= (u128)(__int128)y[i];
                sum += (g % 2 == 1) ? (u128)0 - prod : prod;
                ++nonzero_terms;
            }
        }
    }
    J->sum = sum;
    J->nonzero_terms = nonzero_terms;
    return NULL;
}

/* Sum of integer terms over [g_begin, g_end) modulo 2^128, as (low, high)
 * 64-bit words; out[2] = number of terms without a zero factor. */
int oracle_nw_int_range(int n, const int *colptr, const int *rowidx, uint64_t g_begin, uint64_t g_end,
                        int nthreads, uint64_t out[3]) {
    if (!ccs_ok(n, colptr, rowidx)) return -1;
    uint64_t total = 1ull << (n - 1);
    if (g_begin > g_end || g_end > total) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    nwi_job jobs[256];
    pthread_t th[256];
    uint64_t len = g_end - g_begin;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].n = n;
        jobs[t].colptr = colptr;
        jobs[t].rowidx = rowidx;
        jobs[t].b = g_begin + len / (uint64_t)nthreads * (uint64_t)t + ((uint64_t)t < len % (uint64_t)nthreads ? (uint64_t)t : len % (uint64_t)nthreads);
        jobs[t].e = jobs[t].b + len / (uint64_t)nthreads + ((uint64_t)t < len % (uint64_t)nthreads ? 1u : 0u);
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, nwi_worker, &jobs[t]);
    nwi_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    u128 sum = 0;
    uint64_t nz = 0;
    for (int t = 0; t < nthreads; ++t) {
        sum += jobs[t].sum;
        nz += jobs[t].nonzero_terms;
    }
    out[0] = (uint64_t)sum;
    out[1] = (uint64_t)(sum >> 64);
    out[2] = nz;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 4: PermanentOrdering                                                */
/* ------------------------------------------------------------------------ */
/* Readings: argmin ties go to the lowest column index; the rows of the chosen
 * column are visited in CCS (ascending row) order; only columns not yet
 * chosen have their count decremented (a chosen column holds the "infinity"
 * sentinel and is never chosen again); rows touched by no column (empty rows)
 * are appended at the end in ascending order. */
int oracle_permanent_ordering(int n, const int *colptr, const int *rowidx, int *rowPerm, int *colPerm) {
    if (!ccs_ok(n, colptr, rowidx)) return -1;
    int nnz = colptr[n];
    /* CSR of the pattern, built from the CCS */
    int *rptr = (int *)calloc((size_t)n + 1, sizeof(int));
    int *cids = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    for (int p = 0; p < nnz; ++p) rptr[rowidx[p] + 1] += 1;
    for (int i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
    for (int j = 0; j < n; ++j)
        for (int p = colptr[j]; p < colptr[j + 1]; ++p) {
            int r = rowidx[p];
            cids[rptr[r] + fill[r]++] = j;
        }
    int cdeg[ORACLE_MAX_N], chosen[ORACLE_MAX_N], rmark[ORACLE_MAX_N];
    for (int j = 0; j < n; ++j) {
        cdeg[j] = colptr[j + 1] - colptr[j];
        chosen[j] = 0;
    }
    for (int i = 0; i < n; ++i) rmark[i] = 0;
    int ridx = 0;
    for (int cidx = 0; cidx < n; ++cidx) {
        int col = -1;
        for (int j = 0; j < n; ++j)
            if (!chosen[j] && (col < 0 || cdeg[j] < cdeg[col])) col = j;
        colPerm[cidx] = col;
        chosen[col] = 1;
        cdeg[col] = INT_MAX;
        for (int p = colptr[col]; p < colptr[col + 1]; ++p) {
            int row = rowidx[p];
            if (!rmark[row]) {
                rmark[row] = 1;
                rowPerm[ridx++] = row;
                for (int q = rptr[row]; q < rptr[row + 1]; ++q)
                    if (!chosen[cids[q]]) cdeg[cids[q]] -= 1;
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (!rmark[i]) rowPerm[ridx++] = i;
    free(rptr);
    free(cids);
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 5: Partitioning                                                     */
/* ------------------------------------------------------------------------ */
/* Input: CCS of the already ordered matrix; tau[r] = estimated number of
 * threads that can run when each uses r 32-bit registers for x (the
 * CalculateNoThreads step, a hardware model supplied by the caller) for
 * r = 0..2n; grratio = relative cost of a global to a register update.
 * Output: k (rows of x held in registers) and c (columns that update only
 * registers), chosen by the score tau / (regCost + globCost). */
int oracle_partitioning(int n, const int *colptr, const int *rowidx, const double *tau, double grratio,
                        int *k_out, int *c_out, double *best_out) {
    if (!ccs_ok(n, colptr, rowidx)) return -1;
    int k = 0, c = 0, nrows = 0;
    double bestScore = 0;
    for (int j = 0; j < n; ++j) {
        int maxrow = -1;
        for (int p = colptr[j]; p < colptr[j + 1]; ++p)
            if (rowidx[p] > maxrow) maxrow = rowidx[p];
        if (maxrow + 1 > nrows) nrows = maxrow + 1;
        int nregisters = nrows * 2;
        double pj = ldexp(1.0, -(j + 1));
        double regCost = nregisters * (1.0 - pj);
        double globCost = (n - nrows) * pj * grratio;
        double t = tau[nregisters];
        double currentScore = t / (regCost + globCost);
        if (currentScore > bestScore || nrows == k) {
            bestScore = currentScore;
            k = nrows;
            c = j + 1;
        }
    }
    *k_out = k;
    *c_out = c;
    if (best_out) *best_out = bestScore;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Structural rank: maximum matching by augmenting paths                    */
/* ------------------------------------------------------------------------ */

static int augment(int col, const int *colptr, const int *rowidx, int *row_match, int *seen) {
    for (int p = colptr[col]; p < colptr[col + 1]; ++p) {
        int r = rowidx[p];
        if (seen[r]) continue;
        seen[r] = 1;
        if (row_match[r] < 0 || augment(row_match[r], colptr, rowidx, row_match, seen)) {
            row_match[r] = col;
            return 1;
        }
    }
    return 0;
}

int oracle_structural_rank(int n, const int *colptr, const int *rowidx) {
    if (!ccs_ok(n, colptr, rowidx)) return -1;
    int row_match[ORACLE_MAX_N], seen[ORACLE_MAX_N];
    for (int i = 0; i < n; ++i) row_match[i] = -1;
    int size = 0;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) seen[i] = 0;
        size += augment(j, colptr, rowidx, row_match, seen);
    }
    return size;
}
