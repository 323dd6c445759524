// batch.cpp -- host side of the precompiled batch kernels: per-matrix
// preparation (validation, structural check, Alg. 4 ordering, pre-signed
// 4-row column groups, chunk plan) and the device job that runs a whole
// batch as one captured graph of launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "batch.h"
#include "batch_host.h"
#include "perm_internal.h"

namespace permx {

int batch_kappa(int n, int shift) {
    const int total = n - 1;
    if (total <= 0) return 0;
    // about 2^7 chunks (two waves) per matrix at n <= 24, chunks of 2^16
    // steps above; at least 2^5 steps per chunk when n allows it
    int kappa = std::min(std::max(total - 7 + shift, std::min(total, 5)), 16 + shift);
    return std::max(0, std::min(kappa, total));
}

perm_status prepare_batch_matrix(const perm_csc *m, const BatchOptions &bo, PreparedMatrix *pm, std::string *err) {
    perm_status s = normalize_ccs(m, &pm->a, err);
    if (s != PERM_OK) return s;
    const Ccs &a = pm->a;
    const int n = a.n;
    pm->n = n;
    pm->singular = structural_rank(a) < n;
    if (pm->singular) return PERM_OK;
    std::vector<int> rp, cp;
    permanent_ordering(a, rp, cp);
    const Ccs B = permute(a, rp, cp);
    const int ng = (n + 3) / 4;
    pm->ng = ng;
    pm->kappa = batch_kappa(n, bo.kappa_shift);
    // tops and column groups: [j][g][4]
    const int CS = ng * 4;
    pm->tops.assign(std::max(1, n - 1), 0);
    pm->vals.assign((size_t)std::max(1, n - 1) * CS + 4 * ng, 0.0);
    for (int j = 0; j < n - 1; ++j) {
        int top = 0;
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
            const int r = B.rowidx[q];
            top = std::max(top, r / 4);
            pm->vals[(size_t)j * CS + r] = B.val[q];
        }
        pm->tops[j] = top;
    }
    // x at Gray index 0 (Alg. 1 lines 1-5, a_{i,n-1} = 0 when absent); padding rows 1
    double *base = &pm->vals[(size_t)std::max(1, n - 1) * CS];
    {
        std::vector<long double> rowsum(n, 0.0L), last(n, 0.0L);
        for (int j = 0; j < n; ++j)
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
                rowsum[B.rowidx[q]] += (long double)B.val[q];
                if (j == n - 1) last[B.rowidx[q]] = (long double)B.val[q];
            }
        for (int r = 0; r < 4 * ng; ++r) base[r] = r < n ? (double)(last[r] - rowsum[r] / 2) : 1.0;
    }
    pm->base_index = (size_t)std::max(1, n - 1) * CS;
    pm->chunk_top = 0;
    for (int j = 0; j < std::min(pm->kappa, n - 1); ++j) pm->chunk_top = std::max(pm->chunk_top, pm->tops[j]);
    if (bo.zero_skip > 0) {
        pm->zero_skip = true;
    } else if (bo.zero_skip < 0) {
        pm->zero_skip = false;
    } else {
        pm->zero_skip = true;
        for (double v : B.val)
            if (v != std::floor(v)) pm->zero_skip = false;
    }
    pm->nchunks = (uint64_t)1 << (n - 1 - pm->kappa);
    return PERM_OK;
}

namespace {

template <typename T>
perm_status grow(T **p, size_t *cap, size_t need, std::string *err) {
    if (need <= *cap) return PERM_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t want = std::max<size_t>(need + need / 2, 256);
    if (hipMalloc(p, want * sizeof(T)) != hipSuccess) {
        *err = "device allocation failed (" + std::to_string(want * sizeof(T)) + " bytes)";
        *p = nullptr;
        return PERM_ENOMEM;
    }
    *cap = want;
    return PERM_OK;
}

template <typename T>
perm_status grow_host(T **p, size_t *cap, size_t need, std::string *err) {
    if (need <= *cap) return PERM_OK;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    size_t want = std::max<size_t>(need + need / 2, 256);
    if (hipHostMalloc(reinterpret_cast<void **>(p), want * sizeof(T), hipHostMallocDefault) != hipSuccess) {
        *err = "pinned host allocation failed";
        *p = nullptr;
        return PERM_ENOMEM;
    }
    *cap = want;
    return PERM_OK;
}

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            *err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
            return PERM_EDEVICE;                                                        \
        }                                                                               \
    } while (0)

}  // namespace

BatchJob::~BatchJob() {
    if (d_mats) (void)hipFree(d_mats);
    if (d_items) (void)hipFree(d_items);
    if (d_vals) (void)hipFree(d_vals);
    if (d_tops) (void)hipFree(d_tops);
    if (d_fin) (void)hipFree(d_fin);
    if (d_partials) (void)hipFree(d_partials);
    if (d_out) (void)hipFree(d_out);
    if (h_stage) (void)hipHostFree(h_stage);
    if (h_out) (void)hipHostFree(h_out);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
}

perm_status BatchJob::run(const std::vector<const PreparedMatrix *> &mats, double *out, hipStream_t stream,
                          bool use_graph, double *kernel_ms, std::string *err) {
    const int count = (int)mats.size();
    // order the matrices by kernel instance (ng) so that each instance's
    // items are contiguous; results go back to the caller's order
    std::vector<int> order;
    for (int i = 0; i < count; ++i)
        if (!mats[i]->singular) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return mats[x]->ng < mats[y]->ng;
    });
    for (int i = 0; i < count; ++i)
        if (mats[i]->singular) out[i] = 0.0;
    const int nm = (int)order.size();
    if (nm == 0) {
        if (kernel_ms) *kernel_ms = 0.0;
        return PERM_OK;
    }
    std::vector<BatchMat> hm(nm);
    std::vector<BatchItem> hitems;
    std::vector<FinishDesc> fin(nm);
    size_t nvals = 0, ntops = 0;
    for (int k = 0; k < nm; ++k) {
        const PreparedMatrix &pm = *mats[order[k]];
        BatchMat &d = hm[k];
        d.n = pm.n;
        d.ng = pm.ng;
        d.kappa = pm.kappa;
        d.zero_skip = pm.zero_skip ? 1 : 0;
        d.chunk_top = pm.chunk_top;
        d.pad = 0;
        d.nchunks = pm.nchunks;
        d.col_off = nvals;
        d.base_off = nvals + pm.base_index;
        d.top_off = ntops;
        nvals += pm.vals.size();
        ntops += pm.tops.size();
        fin[k].part = hitems.size();
        fin[k].n = pm.n;
        fin[k].pad = 0;
        for (uint64_t c = 0; c < pm.nchunks; c += 64) hitems.push_back(BatchItem{k, 0, c, (uint64_t)hitems.size()});
        fin[k].count = hitems.size() - fin[k].part;
    }
    const size_t nitems = hitems.size();
    perm_status s;
    if ((s = grow(&d_mats, &cap_mats, (size_t)nm, err)) != PERM_OK) return s;
    if ((s = grow(&d_items, &cap_items, nitems, err)) != PERM_OK) return s;
    if ((s = grow(&d_vals, &cap_vals, nvals, err)) != PERM_OK) return s;
    if ((s = grow(&d_tops, &cap_tops, ntops, err)) != PERM_OK) return s;
    if ((s = grow(&d_fin, &cap_fin, (size_t)nm, err)) != PERM_OK) return s;
    if ((s = grow(&d_partials, &cap_partials, 2 * nitems, err)) != PERM_OK) return s;
    if ((s = grow(&d_out, &cap_out, (size_t)nm, err)) != PERM_OK) return s;
    // one pinned staging buffer for all inputs
    const size_t bytes = nm * sizeof(BatchMat) + nitems * sizeof(BatchItem) + nvals * sizeof(double) +
                         ntops * sizeof(int32_t) + nm * sizeof(FinishDesc) + 64;
    if ((s = grow_host(&h_stage, &cap_stage, bytes, err)) != PERM_OK) return s;
    if ((s = grow_host(&h_out, &cap_hout, (size_t)nm, err)) != PERM_OK) return s;
    char *p = h_stage;
    auto stage = [&](const void *src, size_t n) {
        char *at = p;
        memcpy(p, src, n);
        p += (n + 7) / 8 * 8;
        return at;
    };
    char *s_mats = stage(hm.data(), nm * sizeof(BatchMat));
    char *s_items = stage(hitems.data(), nitems * sizeof(BatchItem));
    char *s_vals = p;
    for (int k = 0; k < nm; ++k) {
        const PreparedMatrix &pm = *mats[order[k]];
        memcpy(p, pm.vals.data(), pm.vals.size() * sizeof(double));
        p += pm.vals.size() * sizeof(double);
    }
    char *s_tops = p;
    for (int k = 0; k < nm; ++k) {
        const PreparedMatrix &pm = *mats[order[k]];
        memcpy(p, pm.tops.data(), pm.tops.size() * sizeof(int32_t));
        p += pm.tops.size() * sizeof(int32_t);
    }
    p = s_tops + (ntops * sizeof(int32_t) + 7) / 8 * 8;
    char *s_fin = stage(fin.data(), nm * sizeof(FinishDesc));

    HIP_OK(hipMemcpyAsync(d_mats, s_mats, nm * sizeof(BatchMat), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_items, s_items, nitems * sizeof(BatchItem), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_vals, s_vals, nvals * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_tops, s_tops, ntops * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_fin, s_fin, nm * sizeof(FinishDesc), hipMemcpyHostToDevice, stream));

    if (!ev0) {
        HIP_OK(hipEventCreate(&ev0));
        HIP_OK(hipEventCreate(&ev1));
    }
    HIP_OK(hipEventRecord(ev0, stream));
    // the launches: one per kernel instance, then the per-matrix finish
    auto enqueue = [&]() -> perm_status {
        size_t i0 = 0;
        while (i0 < nitems) {
            const BatchMat &d0 = hm[hitems[i0].mat];
            size_t i1 = i0;
            while (i1 < nitems && hm[hitems[i1].mat].ng == d0.ng) ++i1;
            HIP_OK(launch_batch_items(d0.ng, d_items + i0, (int64_t)(i1 - i0), d_mats, d_vals, d_tops,
                                      d_partials, stream));
            i0 = i1;
        }
        HIP_OK(launch_batch_finish(d_fin, nm, d_partials, d_out, stream));
        return PERM_OK;
    };
    if (use_graph) {
        if (graph_exec) {
            hipGraphExecDestroy(graph_exec);
            graph_exec = nullptr;
        }
        if (graph) {
            hipGraphDestroy(graph);
            graph = nullptr;
        }
        HIP_OK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        perm_status es = enqueue();
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(stream, &g);
        if (es != PERM_OK) {
            if (g) hipGraphDestroy(g);
            return es;
        }
        if (ce != hipSuccess) {
            *err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ce);
            return PERM_EDEVICE;
        }
        graph = g;
        HIP_OK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
        HIP_OK(hipGraphLaunch(graph_exec, stream));
    } else {
        perm_status es = enqueue();
        if (es != PERM_OK) return es;
    }
    HIP_OK(hipEventRecord(ev1, stream));
    HIP_OK(hipMemcpyAsync(h_out, d_out, nm * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (kernel_ms) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, ev0, ev1));
        *kernel_ms = ms;
    }
    for (int k = 0; k < nm; ++k) out[order[k]] = h_out[k];
    return PERM_OK;
}

}  // namespace permx
