// batch_host.h -- host-side preparation of matrices for the precompiled batch
// kernels, and a reusable device job (see batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "batch.h"
#include "perm_internal.h"

namespace permx {

struct BatchOptions {
    int zero_skip = 0;    // 0 auto (integer-valued matrices), 1 on, -1 off
    int kappa_shift = 0;  // added to the default chunk log2 (autotuning)
};

// One matrix made ready for the batch kernels.
struct PreparedMatrix {
    Ccs a;                     // validated input (explicit zeros dropped)
    int n = 0, ng = 0, kappa = 0;
    bool singular = false;
    bool zero_skip = false;
    int chunk_top = 0;
    uint64_t nchunks = 0;
    std::vector<double> vals;  // [j][ng][4] column groups, then 4*ng base values
    size_t base_index = 0;     // index of the base values in vals
    std::vector<int32_t> tops; // top group per flipped column
};

int batch_kappa(int n, int shift);
perm_status prepare_batch_matrix(const perm_csc *m, const BatchOptions &bo, PreparedMatrix *pm, std::string *err);

// Device buffers and a captured graph for running prepared matrices.
struct BatchJob {
    BatchMat *d_mats = nullptr;
    BatchItem *d_items = nullptr;
    double *d_vals = nullptr;
    int32_t *d_tops = nullptr;
    FinishDesc *d_fin = nullptr;
    double *d_partials = nullptr;
    double *d_out = nullptr;
    size_t cap_mats = 0, cap_items = 0, cap_vals = 0, cap_tops = 0, cap_fin = 0, cap_partials = 0, cap_out = 0;
    char *h_stage = nullptr;
    size_t cap_stage = 0;
    double *h_out = nullptr;
    size_t cap_hout = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    ~BatchJob();
    // Runs all matrices (singular ones are answered 0 without work) and writes
    // out[i] for mats[i].  Synchronous on `stream`.
    perm_status run(const std::vector<const PreparedMatrix *> &mats, double *out, hipStream_t stream, bool use_graph,
                    double *kernel_ms, std::string *err);
};

}  // namespace permx
