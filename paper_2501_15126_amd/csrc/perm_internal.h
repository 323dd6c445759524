// perm_internal.h -- host-side data structures of libperm_mi355x.
//
// The pipeline of one permanent (the paper's "input matrix -> generate ->
// compile -> run -> output" script of Sec. VI-E, rebuilt as a library):
//   validate + normalise CCS (Sec. II CSR/CSC definitions)
//   structural check (a maximum matching; perm = 0 when it is not perfect)
//   ordering (Alg. 4, or ascending column degree) and partition (Alg. 5)
//   level plan for cached partial products (generalises Sec. V's cached
//     global product)
//   code generation (Sec. III-B, Listings 2-5, rebuilt for gfx950) + hipRTC
//   chunk schedule (Theorem 1, Lemma 2; power-of-two aligned chunks)
//   launch, per-workgroup double-double partials, fixed-order final sum.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "perm.h"

namespace permx {

// A validated CCS with explicit zeros removed.
struct Ccs {
    int n = 0;
    std::vector<int32_t> colptr, rowidx;
    std::vector<double> val;
    int nnz() const { return (int)rowidx.size(); }
};

// ---- ccs.cpp ---------------------------------------------------------------
perm_status normalize_ccs(const perm_csc *a, Ccs *out, std::string *err);
// Size of a maximum matching between rows and columns (Hopcroft-Karp).
int structural_rank(const Ccs &a);
// B = A[rowPerm, colPerm] (position -> original index), rows ascending per column.
Ccs permute(const Ccs &a, const std::vector<int> &rowPerm, const std::vector<int> &colPerm);

// ---- preprocess.cpp --------------------------------------------------------
// Alg. 4 (PermanentOrdering).
void permanent_ordering(const Ccs &a, std::vector<int> &rowPerm, std::vector<int> &colPerm);
// Columns by ascending nonzero count (stable), rows unchanged.
void degree_ordering(const Ccs &a, std::vector<int> &rowPerm, std::vector<int> &colPerm);
// Alg. 5 (Partitioning) on an ordered matrix.
void partitioning(const Ccs &ordered, const double *tau, double gr_ratio, int *k, int *c);
// gfx950 thread-count model: tau[r] for r = 0..2n registers of x per lane.
std::vector<double> tau_model(int n, int base_vgprs);

struct DeviceShape {
    int cus = 256;          // compute units
    int simds_per_cu = 4;
    int vgprs_per_simd_lane = 512;
    int max_waves_per_simd = 8;
};
const DeviceShape &device_shape();

struct Plan {
    int n = 0, nnz = 0, mode = PERM_MODE_AUTO;
    std::vector<int> rowPerm, colPerm;  // ordered position -> original index
    Ccs B;                              // the ordered matrix
    int k = 0;                          // rows [0, k) in VGPRs, [k, n) in global memory
    int c = 0;                          // flipped columns [0, c) touch only rows < k
    // Cached product levels.  Level l holds rows whose first flipped column
    // lies in [lev_begin[l], lev_begin[l+1]); the last level also holds rows
    // touched only by the fixed column n-1.  S_l = product of x over levels
    // >= l is kept for l >= 1.
    int nlevels = 1;
    std::vector<int> lev_begin;         // size nlevels + 1, lev_begin[nlevels] = n
    std::vector<int> row_level;         // level of each ordered row
    std::vector<int> col_top;           // highest level touched by each flipped column
    bool cold = false;                  // last level lives outside VGPRs (rows >= k)
    bool cold_lds = false;              // ... in LDS ([row][lane] per workgroup), else global memory
    int kappa = 0;                      // chunk = 2^kappa Gray steps per lane
    int u = 0;                          // static unrolled block = 2^u steps
    int block = 256;
    int waves_per_simd = 0;             // > 0: occupancy hint for the compiler
    int queue_slots = 0;                // per-wave queue of partly needed blocks: slots,
                                        // 0 = the most that fit, -1 = none
    bool zero_skip = true;              // skip chunks / blocks whose terms are exactly 0
    // Column-0 pairing: the two terms of Gray indices 2i and 2i+1 (which
    // differ only in column 0) are summed by one expression, (-1)^i S_1
    // (P(x) - P(x + a)), P the product of column 0's rows (level 0) and x
    // kept without column 0; the walk then flips columns 1..n-2 only, over
    // half as many steps.  Set for AUTO all-terms kernels (FP64, or the
    // exact mode when the bracket stays within the sub-product bound) whose
    // column 0 has one or two entries; kappa and u then count these paired steps:
    // a chunk still covers 2^kappa Gray indices, walked in 2^(kappa-1) steps,
    // and a static block is 2^u paired steps.
    bool pair0 = false;
    int pair_r = -1, pair_s = -1;       // column 0's rows: bracket fma(a_r, x_s, fma(a_s, x_r, a_r a_s))
    // Nested accumulation (FP64 AUTO all-terms kernels, see the generator):
    // per-level products and accumulators instead of cached products.
    bool nested = false;
    // Nested kernels: the rows of the walk's first copy_cols columns (its
    // most frequent flips) kept with every combination of those columns'
    // entries in or out, so that flipping one only selects other copies;
    // chosen by the generator's operation count (0: none).
    int copy_cols = 0;
    // Exact mode: log2 of a bound on the accumulator operations any term's
    // value passes through in one chunk (the error bound's length; the
    // cached-product kernels use kappa, one accumulate per term).
    int acc_log2 = 0;
    // Exact mode (integer-valued matrices): B holds 2a, so x is y = 2x, an
    // integer; the kernel also keeps the term sum modulo a prime and the two
    // sums of its error bound (exact.h).  Each level's product is formed from
    // sub-products of the rows in level_parts[l], each bounded by kExactPartMax.
    bool exact = false;
    std::vector<std::vector<std::vector<int>>> level_parts;
    double base_x_hi[PERM_MAX_N];       // x_r at Gray index 0 (Alg. 1's initialisation)
    int tau_base = 0;                   // VGPRs besides x in Alg. 5's thread-count model
    double ops_per_step = 0, flops_per_step = 0;
    double exact_ops_per_step = 0;      // of ops_per_step: residue and error-bound operations
    std::vector<double> ops_of_col;     // FP64 VALU ops of one step flipping column j
};

// tau_base: VGPRs a lane needs besides its register rows of x in the thread
// count model of Alg. 5 (0 = the built-in estimate; the runtime passes the
// count measured from a compiled HYBRID kernel).
perm_status make_plan(const Ccs &a, const perm_opts &o, Plan *p, std::string *err, int tau_base = 0);

// ---- runtime.cpp -----------------------------------------------------------
// Sets the calling thread's perm_last_error() text.
void set_last_error(const std::string &msg);

// ---- codegen.cpp -----------------------------------------------------------
// FP64 operations per Gray term of a generated step loop, counted as the
// code is emitted (nested-accumulation kernels only; see codegen.cpp).
struct LoopCount {
    bool counted = false;
    double ops_per_step = 0, flops_per_step = 0;
    bool loop = false;          // the step loop runs more than once per chunk
    uint64_t iters = 0;         // its iterations per chunk
    double body_ops = 0;        // the generator's count of one iteration's varying operations
    double terms_per_iter = 0;  // Gray terms of one loop iteration
    int sign_fmas = 0;          // FMAs per iteration that add a signed table entry (1 flop each)
    int copy_values = 0;        // extra doubles the copies of columns 1..copy_cols keep
    int acc_log2 = 0;           // log2 of a bound on the accumulator operations per chunk plus n
};
std::string generate_source(const Plan &p, LoopCount *lc = nullptr);
// Kernel entry point name inside every generated module.
extern const char *const kGrayKernelName;

}  // namespace permx
