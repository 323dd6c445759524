// batch_host.h -- host-side preparation of matrices for the precompiled batch
// kernels, and a reusable device job (see batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "batch.h"
#include "exact.h"
#include "perm_internal.h"

namespace permx {

struct BatchOptions {
    int zero_skip = 0;    // 0 auto (integer-valued matrices), 1 on, -1 off
    int kappa_shift = 0;  // added to the default chunk log2 (autotuning)
    int exact = 0;        // 0 auto (integer-valued matrices whose groups' bounds allow it), 1 required, -1 off
};

// One matrix made ready for the batch kernels.
struct PreparedMatrix {
    Ccs a;                     // validated input (explicit zeros dropped)
    int n = 0, ng = 0, kappa = 0;
    bool singular = false;
    bool zero_skip = false;
    bool exact = false;        // values doubled (y = 2x); residues and the error bound's sum kept
    int chunk_top = 0;
    uint64_t nchunks = 0;
    std::vector<double> vals;  // [j][ng][4] column groups, then 4*ng base values
    size_t base_index = 0;     // index of the base values in vals
    std::vector<int32_t> tops; // top group per flipped column
    double fp64_ops = 0.0;     // FP64 operations of all chunks (an FMA is one), no skipping
    double fp64_fmas = 0.0;    // the FMAs among them
    double exact_ops = 0.0;    // of fp64_ops: the exact mode's residue and bound operations
};

int batch_kappa(int n, int shift);
perm_status prepare_batch_matrix(const perm_csc *m, const BatchOptions &bo, PreparedMatrix *pm, std::string *err);

// The waves of one kernel instance (ng) of a launch, as ranges plus the
// per-workgroup first-range table the kernel starts its search from.
struct WavePlan {
    int ng = 0;
    bool zero_skip = false;
    bool exact = false;
    std::vector<BatchRange> ranges;
    std::vector<int32_t> blk_first;
    uint64_t nwaves = 0;
    // appends waves for items item0 .. item0 + count - 1 of matrix `mat`,
    // whose partials go to out0 .. out0 + count - 1 (count > 0)
    void add(int32_t mat, uint64_t item0, uint64_t count, uint64_t out0);
    void clear() {
        ranges.clear();
        blk_first.clear();
        nwaves = 0;
    }
};

// The library's kernel-class streams (kernel instance ng runs on stream
// ng % kBatchStreams), created on first use on the current device.  Default
// priority, non-blocking.
hipError_t batch_class_streams(hipStream_t out[kBatchStreams]);

// How perm_batch issues its launches.
enum class BatchLaunch {
    Streams,  // each kernel instance on its class stream, forked from and joined to the caller's stream
    Graph,    // persistent instances (resident waves taking items from a counter) on their class
              // streams, captured into one graph; the graph is kept and launched again while
              // the launch layout and buffers stay the same
    Single,   // all launches on the caller's stream
};

// Device buffers and a captured graph for running prepared matrices.
struct BatchJob {
    BatchMat *d_mats = nullptr;
    BatchRange *d_ranges = nullptr;
    int32_t *d_blk = nullptr;
    double *d_vals = nullptr;
    int32_t *d_tops = nullptr;
    FinishDesc *d_fin = nullptr;
    double *d_partials = nullptr;
    double *d_out = nullptr;
    size_t cap_mats = 0, cap_ranges = 0, cap_blk = 0, cap_vals = 0, cap_tops = 0, cap_fin = 0, cap_partials = 0,
           cap_out = 0;
    char *h_stage = nullptr;
    size_t cap_stage = 0;
    double *h_out = nullptr;
    size_t cap_hout = 0;
    unsigned long long *d_counters = nullptr;  // persistent form: one item counter per instance
    size_t cap_counters = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_fork = nullptr;
    hipEvent_t ev_join[kBatchStreams] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::string graph_sig;   // launch layout the graph was captured for
    int graph_captures = 0;  // captures so far (a relaunch does not count)
    int block = 256;         // threads per workgroup of the batch kernels: 64, 128 or 256
    // Allocation-free form: when `arena` is set, every device buffer of a pass
    // is carved from [arena, arena + arena_bytes) (nothing is allocated or
    // freed; a pass that does not fit fails with PERM_ETOOBIG), inputs are
    // staged in ordinary host memory, and only BatchLaunch::Single is allowed.
    char *arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<char> arena_stage;   // host staging of the allocation-free form
    std::vector<double> arena_hout;
    // Creates the timing events (done once, at set-up).
    hipError_t init_events();

    ~BatchJob();
    // Runs all matrices (singular ones are answered 0 without work) and writes
    // out[i] for mats[i].  Exact-mode matrices whose result is not certified
    // after a pass run again with the next prime (exact.h), and all of them
    // until min_passes primes have run.  Synchronous on
    // `stream`.  Optional: exact_state[i] = 1 certified exact, 0 exact mode
    // but uncertified, -1 not in exact mode; *passes = passes run.
    perm_status run(const std::vector<const PreparedMatrix *> &mats, double *out, hipStream_t stream,
                    BatchLaunch how, double *kernel_ms, std::string *err, int *exact_state = nullptr,
                    int *passes = nullptr, int min_passes = 0);

  private:
    // One pass: raw[kPartStride i ..] = (term sum hi, lo, residue, sum |term|)
    // of mats[i] with the prime kExactPrimes[prime[i]] for exact ones.
    perm_status run_pass(const std::vector<const PreparedMatrix *> &mats, const std::vector<int> &prime,
                         double *raw, hipStream_t stream, BatchLaunch how, double *kernel_ms, std::string *err);
};

}  // namespace permx
