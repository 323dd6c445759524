/*
 * perm.h -- C ABI of libperm_mi355x.so: the permanent of a sparse n x n
 * matrix on an AMD Instinct MI355X (gfx950), by the Gray-code
 * Nijenhuis-Wilf variant of Ryser's formula with matrix-specific generated
 * kernels (Elbek & Kaya, arXiv 2501.15126).
 *
 * What is computed (Sec. I Eq. (1); Sec. II Eq. (2) and Alg. 1):
 *
 *   perm(A) = sum over permutations s of prod_i a_{i,s(i)}
 *           = (4 (n mod 2) - 2) * sum_{g=0}^{2^(n-1)-1} (-1)^g prod_i x_i(Gray_g)
 *
 * where x_i(S) = a_{i,n-1} - (sum_j a_ij)/2 + sum_{j in S} a_ij and S ranges
 * over subsets of the first n-1 columns in binary reflected Gray-code order.
 *
 * Conventions for every entry point:
 *  - All functions are thread-safe.  The library owns all device memory,
 *    streams, events and generated code objects; the caller owns its inputs
 *    and outputs, which the library never retains after a call returns.
 *  - Matrices are passed in compressed sparse column form (CCS, the paper's
 *    CSC of Sec. II): colptr int32[n+1], rowidx int32[nnz], val double[nnz],
 *    HOST pointers, 0-based indices.  Rules (violations give PERM_EINVAL):
 *      colptr[0] == 0, colptr non-decreasing, colptr[n] == nnz;
 *      0 <= rowidx < n and strictly increasing inside each column;
 *      every val finite.
 *    Explicit zeros are accepted and dropped.  n < 1 -> PERM_EINVAL;
 *    n > PERM_MAX_N -> PERM_ETOOBIG.
 *  - A structurally singular matrix (no perfect matching of its nonzero
 *    pattern) has permanent exactly +0.0, returned without any kernel launch.
 *  - On error, the status is returned and perm_last_error() describes it.
 *  - Results are deterministic: the same input and options give bitwise the
 *    same result (no floating-point atomics; fixed-order reductions).
 */
#ifndef PERM_MI355X_H
#define PERM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PERM_MAX_N 64

typedef enum {
    PERM_OK = 0,
    PERM_EINVAL = 1,      /* malformed input or option */
    PERM_ETOOBIG = 2,     /* n or a size beyond what the library supports */
    PERM_ENOMEM = 3,      /* host or device allocation failed */
    PERM_EDEVICE = 4,     /* HIP runtime error or no usable gfx950 device */
    PERM_ECOMPILE = 5,    /* hipRTC failed to compile a generated kernel */
    PERM_EAGAIN = 6,      /* server: admission refused, try again later */
    PERM_ENOTREADY = 7,   /* server: result not ready yet */
    PERM_ECANCELED = 8    /* the computation was cancelled */
} perm_status;

/* One sparse matrix in CCS form (host memory, caller-owned). */
typedef struct {
    int32_t n;
    const int32_t *colptr;
    const int32_t *rowidx;
    const double *val;
} perm_csc;

/* Kernel families.
 *  PERM_MODE_AUTO    Alg. 4 ordering; x fully in VGPRs with a multi-level
 *                    cache of partial products (the default).
 *  PERM_MODE_PURE    x fully in VGPRs, columns in ascending-degree order, the
 *                    whole product recomputed every step (the paper's
 *                    register-only generated kernel, Sec. III-IV).
 *  PERM_MODE_HYBRID  Alg. 4 ordering and Alg. 5 partition: rows < k in VGPRs,
 *                    rows >= k in global memory with their product cached and
 *                    recomputed only when a column >= c flips (Sec. V). */
typedef enum { PERM_MODE_AUTO = 0, PERM_MODE_PURE = 1, PERM_MODE_HYBRID = 2 } perm_mode;

/* Options; pass NULL for all defaults, or zero-initialise and set fields. */
typedef struct {
    int32_t mode;          /* perm_mode */
    int32_t chunk_log2;    /* log2 of Gray steps per lane chunk; 0 = automatic (FP64 kernels
                              with column-0 pairing at n >= 37: 15) */
    int32_t unroll_log2;   /* log2 of the static unrolled block, at most 13; 0 = automatic (7,
                              zero-aware kernels 6, nested kernels without pairing 6, kernels
                              with column-0 pairing 13, exact 9).  Always at most chunk_log2 - 1,
                              paired kernels chunk_log2 - 2; values above 9 are reduced to 9
                              except for nested kernels with pairing */
    int32_t block;         /* threads per workgroup, multiple of 64, <= 1024; 0 = 256 (FP64
                              kernels with column-0 pairing: 64) */
    int32_t vgpr_budget;   /* target VGPRs per lane for the level plan; 0 = 128 */
    int32_t force_k;       /* > 0: override Alg. 5's k (HYBRID only), with force_c */
    int32_t force_c;       /* > 0: override Alg. 5's c (HYBRID only) */
    int32_t max_levels;    /* > 0: cap on cached product levels (AUTO); 0 = budget-driven */
    int32_t zero_skip;     /* zero-aware skipping (exact): a wave skips a chunk, a
                              block of 2^(u+1) - 1 steps or any aligned power-of-two
                              interval of Gray indices whose terms all contain a
                              factor that is exactly 0 in every lane.  0 = auto (on
                              when every value is an integer, where such zeros are
                              common), 1 = on, -1 = off */
    int32_t batch_mode;    /* perm_batch: 0 = one launch per kernel instance, one wave per
                              work item (64 chunks of one matrix), each instance on its own
                              class stream so instances overlap (default); 1 = persistent
                              instances captured in one graph: switched off, PERM_EINVAL
                              (a GPU test of it stopped making progress, cause not found);
                              2 = one matrix per launch, synchronised
                              after each (the sequential baseline); 3 = the launches of 0 on
                              one stream.  perm_batch also reads `block` (64, 128 or 256
                              threads per workgroup; 0 = 256) */
    int32_t batch_kappa_shift; /* perm_batch: added to the default chunk log2 */
    int32_t cold_tier;     /* HYBRID: where rows >= k live; 0 = global memory (the paper's
                              scheme), 1 = LDS, [row][lane] per workgroup (the block is
                              then chosen so that a workgroup's rows fit 40 KiB, four
                              workgroups per CU) */
    double gr_ratio;       /* Alg. 5 global/register update cost ratio; 0 = 16 */
    void *hip_stream;      /* hipStream_t to launch on; NULL = the library's stream */
    /* Optional host output: per-workgroup partial sums of the Gray-term sum
     * (before the final factor), as (hi, lo) double pairs, workgroup b
     * covering Gray indices [b*W, (b+1)*W) with W = block * 2^chunk_log2.
     * Filled only if the capacity (in workgroups) is large enough. */
    double *block_partials;
    int64_t block_partials_cap;
    int32_t progress;      /* > 0: perm_sparse_ex prints one line to stderr as each of
                              its launches (at most 2^42 Gray steps each) completes */
    int32_t waves_per_simd; /* occupancy the generated kernel is compiled for.
                              1..8: that many waves per SIMD (the compiler keeps the
                              kernel within 512 / waves VGPRs, spilling if it must);
                              -1: the compiler's own choice; 0 = automatic: the
                              compiler's choice, except that a kernel it holds to 4
                              waves (97..128 VGPRs) whose rows are not in LDS is
                              compiled again for 5 waves, one held to 3 waves
                              (129..168) again for 4, and that build is used if it
                              spills at most 128 bytes per lane */
    int32_t block_queue;   /* zero-aware kernels: a block of 2^(u+1) - 1 steps that only some
                              lanes of a wave need is queued (its start state, in LDS) and
                              evaluated after the walks, one block per thread of the
                              workgroup, instead of by the whole wave in place; a full queue
                              falls back to in place.  Slots per wave: 8, 16, 32 or 64
                              (used if the queue fits 40 KiB of LDS per workgroup); 0 =
                              the most of those that fit; -1 = off.  Only where the
                              block's rows live in VGPRs */
    int32_t exact;         /* exact integer results for integer-valued matrices: the kernels
                              run on y = 2x (then an integer), keep the term sum modulo a
                              prime below 2^24 and a rigorous bound on the FP64 sum's
                              rounding error; the integer congruent to the residue nearest
                              the FP64 estimate is returned when the bound is below half the
                              modulus, else the kernel runs again with the next prime (at
                              most three, residues combined by the Chinese remainder
                              theorem) while |perm| may be below 2^53.  0 = auto (on for
                              integer values whose rows' sums of |a| are at most 2^20),
                              1 = required (PERM_EINVAL otherwise), -1 = off (FP64 only) */
    int32_t exact_passes;  /* exact mode: run at least this many passes (primes), 1..3;
                              0 = as many as the certificate needs */
    int32_t copy_cols;     /* AUTO all-terms kernels in nested form (per-level products and
                              accumulators; always with column-0 pairing, FP64 or exact,
                              otherwise in FP64 when the generator's count of FP64 operations
                              is at most 0.6 of the cached products'): the rows of the walk's
                              m most frequent columns are kept in 2^(columns touching them)
                              copies (each with those columns' entries in or out), so that
                              flipping one of them only selects other copies, and the other
                              flips move every copy.  0 = the m (up to unroll_log2) with the
                              fewest FP64 operations in the generator's count whose copies
                              stay within an allowance of extra doubles per lane (paired FP64
                              400, exact 128 with each level copy's residue counted, dense
                              rows 112), 1..13 = that m (at most unroll_log2; takes the nested
                              form), -1 = none */
} perm_opts;

/* Statistics of one call (all optional to read). */
typedef struct {
    double kernel_ms;       /* device time of the Gray-kernel launch(es): HIP
                               events recorded on the launch stream */
    double reduce_ms;       /* device time of the final reduction kernel */
    double compile_ms;      /* hipRTC compile + module load; 0 on a cache hit */
    double host_ms;         /* validate + structure check + order + partition + codegen;
                               a repeated call with byte-identical input and options
                               reuses the plan and code (about a microsecond) */
    double total_ms;        /* wall time of the whole call */
    double steps;           /* Gray-code steps evaluated: 2^(n-1) */
    double ops_per_step;    /* FP64 VALU operations per step of the generated
                               code, weighted by column frequency (Lemma 1) */
    double flops_per_step;  /* same, counting an FMA that replaces a multiply
                               and an add the method needs as 2 */
    double sum_hi, sum_lo;  /* the Gray-term sum before the final factor */
    double evaluated_steps; /* lane-steps whose product the kernel evaluated, over
                               all launched lanes (inactive padding lanes included;
                               a queued block counts once, for the thread that
                               evaluates it); below steps when zero-aware
                               skipping removed work */
    int64_t nblocks;        /* workgroups launched */
    int64_t nchunks;        /* lane chunks (2^(n-1-chunk_log2)) */
    int32_t n, nnz;         /* after dropping explicit zeros */
    int32_t mode;           /* kernel family actually used */
    int32_t k, c;           /* register rows / register-only columns */
    int32_t levels;         /* cached product levels */
    int32_t chunk_log2, unroll_log2, block;
    int32_t vgprs, sgprs, scratch_bytes, lds_bytes;
    int32_t waves_per_simd; /* occupancy reported by the HIP occupancy API */
    int32_t cache_hit;      /* plan or generated code object reused */
    int32_t singular;       /* 1 if answered as 0 by the structural check */
    int32_t waves_hint;     /* waves per SIMD the kernel was compiled for; 0 = none */
    int32_t vgpr_spills;    /* VGPRs the compiler spilled to scratch */
    int32_t exact;          /* 1: the result is the exact integer permanent (certified, or the
                               structural zero); 0: exact mode ran but the result is the FP64
                               estimate (|perm| at least 2^53, or no certificate after three
                               primes); -1: not in exact mode */
    int32_t exact_passes;   /* kernel passes (primes) of the exact mode */
    double estimate;        /* the FP64 estimate of the permanent */
    double err_bound;       /* exact mode: rigorous bound on |estimate - perm| */
    double exact_ops_per_step; /* of ops_per_step: the exact mode's residue and bound operations */
    int32_t exact_bound_log2;  /* exact mode: log2 of the operation count per chunk that the
                                  error bound takes (perm_exact_recover's chunk_log2 for this
                                  kernel: chunk_log2, or more with nested accumulators); 0 outside
                                  the exact mode */
    int32_t copy_cols;         /* nested kernels: copied columns of the kernel that ran (a paired
                                  FP64 build that spilled is compiled again with fewer; pass this
                                  and waves_hint to perm_codegen for the text that ran); 0 = none */
} perm_stats;

/* Permanent of one matrix (Alg. 1 end to end).  Returns NaN on error
 * (see perm_last_error).  Synchronous. */
double perm_sparse(int32_t n, const int32_t *colptr, const int32_t *rowidx, const double *val);

/* Same with options and statistics.  *out receives the permanent.  opts and
 * st may be NULL.  Synchronous: returns after the result is on the host. */
perm_status perm_sparse_ex(const perm_csc *a, const perm_opts *opts, double *out, perm_stats *st);

/* Permanents (Eq. (1), by Alg. 1) of `count` matrices (any mix of sizes
 * n <= 44; larger n gives PERM_ETOOBIG: use perm_sparse_ex), out[i] for mats[i].  Synchronous.  Uses kernels compiled into the
 * library (no per-matrix hipRTC): x in registers as 4-row groups, each
 * matrix's columns as data, 64 chunks of one matrix per wave, one launch per
 * kernel instance (group count, zero-skip kind), each instance on a stream
 * of its own (batch_mode selects other launch forms).  A matrix's result
 * depends only on that matrix and the options, not on the rest of the batch
 * (bitwise).  Results agree with perm_sparse_ex within the
 * FP64 tolerance, not bitwise (different kernels).  Any invalid matrix fails
 * the whole call (PERM_EINVAL, perm_last_error names its index). */
perm_status perm_batch(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out);

typedef struct {
    double wall_ms;        /* whole call */
    double prep_ms;        /* host preparation of all matrices */
    double kernel_ms;      /* device time of the launches (events on the stream) */
    double steps;          /* Gray-code steps of the nonsingular matrices */
    int32_t count;         /* matrices */
    int32_t singular;      /* answered 0 by the structural check */
    int32_t launches;      /* kernel launches issued */
    int32_t pad;
    double fp64_ops;       /* FP64 operations the batch kernels execute (an FMA is one),
                              counted exactly per chunk without zero-aware skipping */
    double flops;          /* the same with an FMA counted as 2 */
    double exact_ops;      /* of fp64_ops: the exact mode's residue and bound operations */
    int32_t exact_certified;   /* matrices whose result is the exact integer (exact mode, or
                                  structurally singular) */
    int32_t exact_uncertified; /* exact-mode matrices left at the FP64 estimate */
    int32_t passes;        /* kernel passes run (exact mode: one per prime needed) */
    int32_t graph_captures; /* graph captures of the process so far (0 while batch_mode 1
                              is switched off) */
} perm_batch_stats;

/* perm_batch with statistics (st may be NULL). */
perm_status perm_batch_ex(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out,
                          perm_batch_stats *st);

/* perm_batch_ex for callers that cannot allocate device memory (code that a
 * caller captures into a HIP graph, tight serving loops, hosts that forbid
 * allocation after start-up).  It allocates no device or pinned host memory
 * and frees none: the staged matrices, the wave partials and the per-matrix
 * sums live in a fixed region of PERM_NOALLOC_SCRATCH_BYTES bytes per device,
 * a device array of the library whose address is looked up once, when the
 * library first sets up the device.  Inputs are copied from ordinary host
 * memory; host-side preparation uses the ordinary heap, on the calling thread.
 * Same kernels, same work order and so bitwise the same results as
 * perm_batch_ex with the same opts, except that every launch goes on one
 * stream (opts->hip_stream, else the library's): batch_mode is ignored.
 * A batch whose buffers do not fit the region fails with PERM_ETOOBIG (its
 * message gives the bytes needed); split it, or use perm_batch_ex.
 * The region keeps the last call's contents; every buffer a call reads is
 * written by that call first, so nothing needs clearing.  Synchronous, and
 * serialised with every other call of the library in this process by its
 * lock, so calls from several threads never share the region at once; each
 * process holds its own copy of the region. */
#define PERM_NOALLOC_SCRATCH_BYTES (64u << 20)
perm_status perm_batch_noalloc(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out,
                               perm_batch_stats *st);

/* ---- Autotuning ---------------------------------------------------------- */

typedef struct {
    double default_ms;      /* device time of the starting options on the sample */
    double best_ms;         /* device time of the returned options on the sample */
    double sample_fraction; /* fraction of the work each candidate ran (batch: 1) */
    double tune_ms;         /* wall time of the whole search, compiles included */
    int32_t candidates;     /* option sets timed, the starting one included */
    int32_t pad;
} perm_tune_stats;

/* Picks launch options for one matrix by timing its generated kernel: starting
 * from opts (NULL = defaults), it tries in turn the register/global split
 * (AUTO; HYBRID with Alg. 5's partition and the cold rows in global memory or
 * in LDS), the chunk size (log2 of the Gray steps per lane, +-1 and +-2 around
 * the current, then past a winning +-2 one step at a time, at most 3 more),
 * the static block (+-1, then on the winning side one step at a time, at most
 * 3 more), the threads per workgroup (64, 128, 256), the block queue of
 * zero-aware kernels (off, 16, 32, 64 slots) and the compiled occupancy (-1,
 * 4, 5, 6), keeping a candidate only if it is at least 2 % faster.  Every
 * candidate runs on the same sample of the Gray-index space: 8 evenly spaced
 * slices, each of 2^19 chunks of the current chunk + 2 (so every launch fills
 * the GPU; chunks past that run fewer), or the whole space when that is no
 * larger; best of 3 passes (one pass above 100 ms).
 * Candidates that the planner rejects are skipped.  *best receives the winning options (pass them to
 * perm_sparse_ex); candidates' plans and code stay in the plan cache.  The
 * result of the permanent does not depend on these options beyond FP64
 * rounding (bitwise for the occupancy).  The paper takes the thread count
 * from the occupancy API (Alg. 3) and Alg. 5's GRratio from preliminary
 * benchmarks; here the launch shape and the split are chosen by timing. */
perm_status perm_autotune(const perm_csc *a, const perm_opts *opts, perm_opts *best, perm_tune_stats *st);

/* Picks perm_batch options for a batch by running it whole (batch_mode 0, or
 * 3 if given): the threads per workgroup (64, 128, 256)
 * and then batch_kappa_shift (+-1, +-2), each kept if at least 2 % faster
 * in device time (best of 3 runs).  Results are bitwise independent of
 * batch_mode and block; batch_kappa_shift changes the chunking, so results
 * may differ in the last bits (integer-valued matrices: not at all, their
 * results are exact). */
perm_status perm_batch_autotune(int32_t count, const perm_csc *mats, const perm_opts *opts, perm_opts *best,
                                perm_tune_stats *st);

/* ---- Serving: submit / poll with continuous batching ------------------- */

/* A server owns a scheduler thread, a device-memory arena of
 * `device_mem_budget` bytes (0 = 1 GiB) and at most `max_inflight` requests
 * that were submitted and not yet collected (0 = 4096).  Requests use the
 * precompiled batch kernels (no per-request hipRTC) with opts' zero_skip, and
 * chunks 2^3 times smaller than perm_batch's (batch_kappa_shift - 3), so that
 * rounds interleave requests at a finer grain.  Admission is in arrival
 * order, as arena memory frees.
 * Every scheduling round runs `round_steps` Gray steps (0 = 1.6e10, about
 * 20 ms of device work): first all of the remaining work of every small request
 * (at most a quarter of a round left), then the larger requests in arrival
 * order, each as much as it can use.  Two rounds are in flight, so requests
 * that arrive while others run join the next round.  Each kernel instance
 * (ng) has its own stream.  A request's result is bitwise the same whether
 * it runs alone or in any mix, and equals perm_batch's with the same options
 * except batch_kappa_shift lowered by 3.  Returns NULL on
 * error (perm_last_error).  The server uses the device current at creation. */
typedef struct perm_server perm_server;
perm_server *perm_server_create(const perm_opts *opts, size_t device_mem_budget, int32_t max_inflight,
                                double round_steps);

/* Validates and copies the matrix, answers structurally singular ones at once
 * (0), and queues the rest.  *ticket identifies the request.  PERM_EAGAIN when
 * max_inflight requests are outstanding; PERM_ETOOBIG when the request alone
 * needs more than the arena.  Thread-safe. */
perm_status perm_submit(perm_server *s, const perm_csc *a, uint64_t *ticket);

/* PERM_ENOTREADY while the request runs; PERM_OK with *out once it is done
 * (the ticket is then released); PERM_EINVAL for an unknown ticket;
 * PERM_EDEVICE if the device failed.  Non-blocking, thread-safe. */
perm_status perm_poll(perm_server *s, uint64_t ticket, double *out);

/* perm_poll that blocks until the request is done. */
perm_status perm_wait(perm_server *s, uint64_t ticket, double *out);

typedef struct {
    uint64_t submitted, completed, rounds;
    uint64_t pending, active;       /* queued (not admitted) / admitted, running */
    uint64_t arena_bytes, arena_used, arena_peak;
    double busy_ms;                 /* wall time with at least one round in flight */
    uint64_t exact_certified;       /* exact-mode requests answered with the certified integer */
    uint64_t exact_uncertified;     /* exact-mode requests left at the FP64 estimate */
    uint64_t extra_passes;          /* exact-mode passes beyond each request's first (next primes) */
} perm_server_stats;
perm_status perm_server_get_stats(perm_server *s, perm_server_stats *st);

/* Finishes all submitted work, stops the scheduler and frees the server.
 * Results not collected are discarded. */
void perm_server_destroy(perm_server *s);

/* ---- Introspection of the host-side steps (used by tests) -------------- */

/* The preprocessing decisions for a matrix without running it.
 * row_perm / col_perm (caller buffers of n int32, may be NULL) receive the
 * ordering: ordered position -> original index (Alg. 4, or ascending column
 * degree in PURE mode).  tau (caller buffer of 2n+1 doubles, may be NULL)
 * receives the thread-count model used by Alg. 5 (threads resident on the
 * device when each uses r registers for x, r = 0..2n).  *k, *c receive
 * Alg. 5's partition (AUTO and PURE report k = n, c = n - 1), *levels the
 * number of cached product levels, *structural_rank the size of a maximum
 * matching of the pattern (after dropping explicit zeros). */
perm_status perm_plan(const perm_csc *a, const perm_opts *opts, int32_t *row_perm, int32_t *col_perm,
                      double *tau, int32_t *k, int32_t *c, int32_t *levels, int32_t *structural_rank);

/* Alg. 5 alone on an already ordered pattern, with a caller-supplied tau
 * table (2n+1 entries) and GRratio. */
perm_status perm_partition(const perm_csc *ordered, const double *tau, double gr_ratio, int32_t *k,
                           int32_t *c);

/* The HIP source text generated for a matrix.  Writes at most cap bytes
 * (NUL-terminated when it fits) and the full length to *len.  Generation only:
 * with waves_per_simd 0 (automatic) the text carries no occupancy attribute;
 * passing perm_stats.waves_hint (and, where nonzero, copy_cols) of a run gives
 * the exact text that ran. */
perm_status perm_codegen(const perm_csc *a, const perm_opts *opts, char *buf, size_t cap, size_t *len);

/* Compile the generated kernel for a matrix with hipRTC (gfx950; no GPU
 * needed) without launching it, and report the plan and the code object's
 * resources (vgprs, sgprs, scratch_bytes, lds_bytes, compile_ms) in *st. */
perm_status perm_compile_info(const perm_csc *a, const perm_opts *opts, perm_stats *st);

/* The data the precompiled batch kernels use for one matrix (introspection
 * for tests): desc[0..7] = n, ng (4-row groups), chunk log2, zero-skip flag,
 * highest group of the in-chunk columns, structurally singular flag, exact
 * mode flag (values then doubled: x holds y = 2x), 0;
 * vals (cap doubles) = column groups [j][ng][4] for flipped columns j, then
 * the 4*ng starting values of x; tops (cap ints) = highest group per flipped
 * column.  *nvals / *ntops receive the needed sizes. */
perm_status perm_batch_describe(const perm_csc *a, const perm_opts *opts, int32_t desc[8], double *vals,
                                size_t vals_cap, size_t *nvals, int32_t *tops, size_t tops_cap, size_t *ntops);

/* The exact mode's integer recovery (introspection for tests; exact mode,
 * Sec. II Alg. 1 on y = 2x).  Input: an n x n integer-valued matrix's Gray
 * term sum in y units (products of 2x) as a double-double (hi, lo), the sum
 * of |terms| A, the chunk log2 (no accumulator took more than 2^chunk_log2
 * terms), and resid[0..passes-1], the term sum modulo the library's primes
 * (perm_exact_primes; any representatives, exact integers).  Output:
 * out[0] = the permanent (the exact integer when *certified), out[1] = the
 * FP64 estimate (4 (n mod 2) - 2) 2^-n (hi + lo), out[2] = the rigorous bound
 * on |estimate - perm|; *more = 1 when another prime could certify a result
 * that may be below 2^53 in magnitude.  PERM_EINVAL for n outside 1..64 or
 * passes outside 0..3. */
perm_status perm_exact_recover(int32_t n, double hi, double lo, double abs_sum, int32_t chunk_log2, int32_t passes,
                               const double *resid, double out[3], int32_t *certified, int32_t *more);

/* The exact mode's primes, in the order of the passes (3 values). */
void perm_exact_primes(double out[3]);

/* Description of the last error on the calling thread (never NULL; valid
 * until the next library call on that thread). */
const char *perm_last_error(void);

/* Library version string. */
const char *perm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PERM_MI355X_H */
