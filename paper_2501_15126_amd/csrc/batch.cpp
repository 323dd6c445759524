// batch.cpp -- host side of the precompiled batch kernels: per-matrix
// preparation (validation, structural check, Alg. 4 ordering, pre-signed
// 4-row column groups, chunk plan) and the device job that runs a whole
// batch: one launch per kernel instance, each on its class stream (or all on
// one stream, optionally captured as a graph), then one finish launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>

#include "batch.h"
#include "batch_host.h"
#include "perm_internal.h"

namespace permx {

int batch_kappa(int n, int shift) {
    const int total = n - 1;
    if (total <= 0) return 0;
    // about 2^9 chunks (eight waves) per matrix up to n = 23, chunks of 2^13
    // steps above (a wave then runs well under a millisecond, the grain at
    // which the server interleaves requests); at least 2^5 steps per chunk
    // when n allows it
    int kappa = std::min(std::max(total - 9 + shift, std::min(total, 5)), 13 + shift);
    // at most 2^22 work items (64-chunk waves) per matrix: 64 MiB of partials
    kappa = std::max(kappa, total - 28);
    return std::max(0, std::min(kappa, total));
}

perm_status prepare_batch_matrix(const perm_csc *m, const BatchOptions &bo, PreparedMatrix *pm, std::string *err) {
    perm_status s = normalize_ccs(m, &pm->a, err);
    if (s != PERM_OK) return s;
    const Ccs &a = pm->a;
    const int n = a.n;
    pm->n = n;
    if (n > kBatchMaxN) {
        *err = "n = " + std::to_string(n) + " is beyond the batch kernels (n <= " + std::to_string(kBatchMaxN) +
               "); use perm_sparse_ex";
        return PERM_ETOOBIG;
    }
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
    // x at Gray index 0 (Alg. 1's initialisation, a_{i,n-1} = 0 when absent); padding rows 1
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
    // exact mode: integer values, and every 4-row group's bound (the product
    // of its rows' sums of |a|, a bound on |product of y|) within
    // kExactPartMax, so that a group product times a residue stays exact
    {
        bool ok = bo.exact >= 0;
        for (double v : B.val)
            if (v != std::floor(v)) ok = false;
        std::vector<double> rowabs(4 * ng, 1.0);
        for (int r = 0; r < n; ++r) rowabs[r] = 0.0;
        for (int q = 0; q < B.nnz(); ++q) rowabs[B.rowidx[q]] += std::fabs(B.val[q]);
        for (int g = 0; g < ng && ok; ++g)
            ok = rowabs[4 * g] * rowabs[4 * g + 1] * rowabs[4 * g + 2] * rowabs[4 * g + 3] <= kExactPartMax;
        if (bo.exact == 1 && !ok) {
            *err = "exact = 1 needs integer values with every 4-row group's bound at most 2^20";
            return PERM_EINVAL;
        }
        pm->exact = ok;
        if (ok) {
            // y = 2x: the column values and the start values of the n real rows
            for (size_t i = 0; i < pm->base_index; ++i) pm->vals[i] *= 2.0;
            for (int r = 0; r < n; ++r) base[r] *= 2.0;
        }
    }
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
    // Work of the batch kernel, counted from its code: a step flipping a
    // column with top group t updates groups t..0 (4 FMAs each), refreshes
    // the suffix products of groups t..1 (3 multiplies for the group, one
    // more unless it is the last group) and adds the term (4 multiplies, one
    // FMA).  Local step l flips column ctz(l); every chunk also runs one
    // weight-0 step on column 0 and starts with the columns at or above
    // kappa - 1, the suffix products and the first term.
    {
        auto step_ops = [&](int t, double *fmas) {
            double ops = 9.0;
            for (int g = 1; g <= t; ++g) ops += (g + 1 < ng) ? 8.0 : 7.0;
            *fmas = 5.0 + 4.0 * t;
            return ops;
        };
        const int kap = pm->kappa;
        double ops = 0.0, fmas = 0.0, f = 0.0;
        for (int j = 0; j < kap; ++j) {  // column j flips 2^(kappa-1-j) times per chunk
            const double cnt = std::ldexp(1.0, kap - 1 - j);
            ops += cnt * step_ops(pm->tops[j], &f);
            fmas += cnt * f;
        }
        if (kap >= 1) {
            ops += step_ops(pm->tops[0], &f);
            fmas += f;
        }
        const double init_fmas = (double)(n - 1 - std::max(kap - 1, 0)) * 4.0 * ng;
        ops += init_fmas + 4.0 * (ng - 1) + 4.0;
        fmas += init_fmas;
        if (pm->exact) {
            // per step: a residue reduction (two multiplies, a rounding, an
            // FMA) per refreshed group below the top one, the residue FMA and
            // the |term| FMA; per 512 steps a reduction of the residue sum
            double xo = 0.0, xf = 0.0;
            for (int j = 0; j < kap; ++j) {
                const double cnt = std::ldexp(1.0, kap - 1 - j);
                const int t = std::min(pm->tops[j], ng - 2);
                xo += cnt * (4.0 * std::max(t, 0) + 2.0);
                xf += cnt * (1.0 * std::max(t, 0) + 2.0);
            }
            xo += 3.0 * (std::ldexp(1.0, kap) / 512.0 + 1.0) + 4.0 * std::max(ng - 2, 0) + 2.0;
            ops += xo;
            fmas += xf;
            pm->exact_ops = xo * (double)((uint64_t)1 << (n - 1 - kap));
        }
        pm->fp64_ops = ops * (double)pm->nchunks;
        pm->fp64_fmas = fmas * (double)pm->nchunks;
    }
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

void WavePlan::add(int32_t mat, uint64_t item0, uint64_t count, uint64_t out0) {
    const int32_t r = (int32_t)ranges.size();
    ranges.push_back(BatchRange{mat, 0, nwaves, item0, out0});
    // workgroups whose first wave (4b) lies in [nwaves, nwaves + count)
    const uint64_t b1 = (nwaves + count + 3) / 4;
    while (blk_first.size() < b1) blk_first.push_back(r);
    nwaves += count;
}

hipError_t batch_class_streams(hipStream_t out[kBatchStreams]) {
    static hipStream_t streams[kBatchStreams] = {};
    static bool made = false;
    if (!made) {
        for (int i = 0; i < kBatchStreams; ++i) {
            const hipError_t e = hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
        made = true;
    }
    for (int i = 0; i < kBatchStreams; ++i) out[i] = streams[i];
    return hipSuccess;
}

hipError_t BatchJob::init_events() {
    if (ev0) return hipSuccess;
    hipError_t e;
    if ((e = hipEventCreate(&ev0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&ev1)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming)) != hipSuccess) return e;
    for (int i = 0; i < kBatchStreams; ++i)
        if ((e = hipEventCreateWithFlags(&ev_join[i], hipEventDisableTiming)) != hipSuccess) return e;
    return hipSuccess;
}

BatchJob::~BatchJob() {
    if (arena) return;  // the buffers are views of the allocation-free region
    if (d_mats) (void)hipFree(d_mats);
    if (d_ranges) (void)hipFree(d_ranges);
    if (d_blk) (void)hipFree(d_blk);
    if (d_vals) (void)hipFree(d_vals);
    if (d_tops) (void)hipFree(d_tops);
    if (d_fin) (void)hipFree(d_fin);
    if (d_partials) (void)hipFree(d_partials);
    if (d_out) (void)hipFree(d_out);
    if (d_counters) (void)hipFree(d_counters);
    if (h_stage) (void)hipHostFree(h_stage);
    if (h_out) (void)hipHostFree(h_out);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
}

perm_status BatchJob::run(const std::vector<const PreparedMatrix *> &mats, double *out, hipStream_t stream,
                          BatchLaunch how, double *kernel_ms, std::string *err, int *exact_state, int *passes,
                          int min_passes) {
    const int count = (int)mats.size();
    std::vector<double> raw((size_t)kPartStride * std::max(count, 1), 0.0);
    std::vector<int> prime(count, 0);
    double kms = 0.0;
    perm_status s = run_pass(mats, prime, raw.data(), stream, how, &kms, err);
    if (s != PERM_OK) return s;
    int npass = 1;
    std::vector<ExactSums> es(count);
    std::vector<int> todo;  // exact-mode matrices still to recover
    for (int i = 0; i < count; ++i) {
        const PreparedMatrix &pm = *mats[i];
        const double *r = &raw[(size_t)kPartStride * i];
        if (exact_state) exact_state[i] = pm.singular ? 1 : pm.exact ? 0 : -1;
        if (pm.singular) {
            out[i] = 0.0;
        } else if (!pm.exact) {
            out[i] = (r[0] + r[1]) * ((pm.n % 2 == 1) ? 2.0 : -2.0);  // final factor 4 (n mod 2) - 2
        } else {
            es[i].hi = r[0];
            es[i].lo = r[1];
            es[i].abs_sum = r[3];
            es[i].chunk_log2 = pm.kappa;
            es[i].resid[0] = r[2];
            es[i].passes = 1;
            todo.push_back(i);
        }
    }
    // exact mode: recover; the uncertified ones run again with the next prime
    while (!todo.empty()) {
        std::vector<int> again;
        for (int i : todo) {
            const ExactOutcome eo = exact_recover(mats[i]->n, es[i]);
            out[i] = eo.value;
            if (exact_state) exact_state[i] = eo.certified ? 1 : 0;
            const bool forced = es[i].passes < std::min(min_passes, kExactMaxPasses);
            if ((!eo.certified && eo.more) || forced) again.push_back(i);
        }
        if (again.empty()) break;
        std::vector<const PreparedMatrix *> sub;
        std::vector<int> pr;
        for (int i : again) {
            sub.push_back(mats[i]);
            pr.push_back(es[i].passes);
        }
        std::vector<double> raw2((size_t)kPartStride * sub.size(), 0.0);
        double k2 = 0.0;
        s = run_pass(sub, pr, raw2.data(), stream, how, &k2, err);
        if (s != PERM_OK) return s;
        kms += k2;
        ++npass;
        for (size_t q = 0; q < again.size(); ++q) {
            ExactSums &e = es[again[q]];
            e.resid[e.passes++] = raw2[kPartStride * q + 2];
        }
        todo = again;
    }
    if (kernel_ms) *kernel_ms = kms;
    if (passes) *passes = npass;
    return PERM_OK;
}

perm_status BatchJob::run_pass(const std::vector<const PreparedMatrix *> &mats, const std::vector<int> &prime,
                               double *raw, hipStream_t stream, BatchLaunch how, double *kernel_ms,
                               std::string *err) {
    const int count = (int)mats.size();
    // order the matrices by kernel instance (ng, zero skip, exact), largest
    // work first within an instance; results go back to the caller's order
    std::vector<int> order;
    for (int i = 0; i < count; ++i)
        if (!mats[i]->singular) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (mats[x]->ng != mats[y]->ng) return mats[x]->ng < mats[y]->ng;
        if (mats[x]->zero_skip != mats[y]->zero_skip) return mats[y]->zero_skip;
        if (mats[x]->exact != mats[y]->exact) return mats[y]->exact;
        return mats[x]->n > mats[y]->n;
    });
    const int nm = (int)order.size();
    if (nm == 0) {
        if (kernel_ms) *kernel_ms = 0.0;
        return PERM_OK;
    }
    std::vector<BatchMat> hm(nm);
    std::vector<FinishDesc> fin(nm);
    std::vector<WavePlan> plans;
    size_t nvals = 0, ntops = 0;
    uint64_t nparts = 0;
    for (int k = 0; k < nm; ++k) {
        const PreparedMatrix &pm = *mats[order[k]];
        BatchMat &d = hm[k];
        d.n = pm.n;
        d.ng = pm.ng;
        d.kappa = pm.kappa;
        d.zero_skip = pm.zero_skip ? 1 : 0;
        d.chunk_top = pm.chunk_top;
        d.exact = pm.exact ? 1 : 0;
        d.nchunks = pm.nchunks;
        d.col_off = nvals;
        d.base_off = nvals + pm.base_index;
        d.top_off = ntops;
        d.pmod = pm.exact ? kExactPrimes[prime[order[k]]] : 0.0;
        d.pinv = pm.exact ? 1.0 / d.pmod : 0.0;
        nvals += pm.vals.size();
        ntops += pm.tops.size();
        const uint64_t items = (pm.nchunks + 63) / 64;
        if (plans.empty() || plans.back().ng != pm.ng || plans.back().zero_skip != pm.zero_skip ||
            plans.back().exact != pm.exact) {
            plans.emplace_back();
            plans.back().ng = pm.ng;
            plans.back().zero_skip = pm.zero_skip;
            plans.back().exact = pm.exact;
        }
        plans.back().add(k, 0, items, nparts);
        fin[k] = FinishDesc{nparts, items, pm.n, pm.exact ? 1 : 0, d.pmod, d.pinv};
        nparts += items;
    }
    size_t nranges = 0, nblk = 0;
    for (const WavePlan &w : plans) {
        nranges += w.ranges.size();
        nblk += w.blk_first.size();
    }
    perm_status s;
    // all inputs staged in one host buffer (pinned, or ordinary host memory
    // in the allocation-free form)
    const size_t bytes = nm * sizeof(BatchMat) + nranges * sizeof(BatchRange) + nblk * sizeof(int32_t) +
                         nvals * sizeof(double) + ntops * sizeof(int32_t) + nm * sizeof(FinishDesc) + 64;
    char *stage = nullptr;
    double *hout = nullptr;
    if (arena) {
        if (how != BatchLaunch::Single) {
            *err = "the allocation-free form launches on one stream only";
            return PERM_EINVAL;
        }
        // views of the fixed region, 256-byte aligned; nothing is allocated
        size_t off = 0;
        auto carve = [&](auto **pp, size_t n) {
            off = (off + 255) / 256 * 256;
            *pp = reinterpret_cast<std::remove_reference_t<decltype(**pp)> *>(arena + off);
            off += n * sizeof(**pp);
        };
        carve(&d_mats, (size_t)nm);
        carve(&d_ranges, nranges);
        carve(&d_blk, nblk);
        carve(&d_vals, nvals);
        carve(&d_tops, ntops);
        carve(&d_fin, (size_t)nm);
        carve(&d_partials, (size_t)kPartStride * nparts);
        carve(&d_out, (size_t)kPartStride * nm);
        if (off > arena_bytes) {
            *err = "the batch needs " + std::to_string(off) + " bytes of device scratch; the allocation-free form "
                   "holds " + std::to_string(arena_bytes) + " (split the batch, or use perm_batch)";
            return PERM_ETOOBIG;
        }
        if (arena_stage.size() < bytes) arena_stage.resize(bytes);
        if (arena_hout.size() < (size_t)kPartStride * nm) arena_hout.resize((size_t)kPartStride * nm);
        stage = arena_stage.data();
        hout = arena_hout.data();
    } else {
        if ((s = grow(&d_mats, &cap_mats, (size_t)nm, err)) != PERM_OK) return s;
        if ((s = grow(&d_ranges, &cap_ranges, nranges, err)) != PERM_OK) return s;
        if ((s = grow(&d_blk, &cap_blk, nblk, err)) != PERM_OK) return s;
        if ((s = grow(&d_vals, &cap_vals, nvals, err)) != PERM_OK) return s;
        if ((s = grow(&d_tops, &cap_tops, ntops, err)) != PERM_OK) return s;
        if ((s = grow(&d_fin, &cap_fin, (size_t)nm, err)) != PERM_OK) return s;
        if ((s = grow(&d_partials, &cap_partials, (size_t)kPartStride * nparts, err)) != PERM_OK) return s;
        if ((s = grow(&d_out, &cap_out, (size_t)kPartStride * nm, err)) != PERM_OK) return s;
        if ((s = grow_host(&h_stage, &cap_stage, bytes, err)) != PERM_OK) return s;
        if ((s = grow_host(&h_out, &cap_hout, (size_t)kPartStride * nm, err)) != PERM_OK) return s;
        stage = h_stage;
        hout = h_out;
    }
    char *p = stage;
    auto align8 = [&]() { p = stage + ((size_t)(p - stage) + 7) / 8 * 8; };
    char *s_mats = p;
    memcpy(p, hm.data(), nm * sizeof(BatchMat));
    p += nm * sizeof(BatchMat);
    align8();
    char *s_ranges = p;
    for (const WavePlan &w : plans) {
        memcpy(p, w.ranges.data(), w.ranges.size() * sizeof(BatchRange));
        p += w.ranges.size() * sizeof(BatchRange);
    }
    char *s_blk = p;
    for (const WavePlan &w : plans) {
        memcpy(p, w.blk_first.data(), w.blk_first.size() * sizeof(int32_t));
        p += w.blk_first.size() * sizeof(int32_t);
    }
    align8();
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
    align8();
    char *s_fin = p;
    memcpy(p, fin.data(), nm * sizeof(FinishDesc));

    HIP_OK(hipMemcpyAsync(d_mats, s_mats, nm * sizeof(BatchMat), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_ranges, s_ranges, nranges * sizeof(BatchRange), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_blk, s_blk, nblk * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_vals, s_vals, nvals * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_tops, s_tops, ntops * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_OK(hipMemcpyAsync(d_fin, s_fin, nm * sizeof(FinishDesc), hipMemcpyHostToDevice, stream));

    HIP_OK(init_events());
    const bool persistent = how == BatchLaunch::Graph;
    const bool branches = how == BatchLaunch::Streams || how == BatchLaunch::Graph;
    // persistent form: one item counter and a resident-size grid per instance
    std::vector<int> grids(plans.size(), 0);
    if (persistent) {
        if ((s = grow(&d_counters, &cap_counters, plans.size(), err)) != PERM_OK) return s;
        for (size_t i = 0; i < plans.size(); ++i) {
            const WavePlan &w = plans[i];
            const int rb = batch_resident_blocks(w.ng, w.zero_skip, w.exact, block);
            if (rb <= 0) {
                *err = "occupancy query of the persistent batch kernel failed";
                return PERM_EDEVICE;
            }
            const int64_t need = ((int64_t)w.nwaves + block / 64 - 1) / (block / 64);
            grids[i] = (int)std::min<int64_t>(rb, need);
        }
    }
    HIP_OK(hipEventRecord(ev0, stream));
    hipStream_t cls[kBatchStreams];
    if (branches) HIP_OK(batch_class_streams(cls));
    // the launches: one per kernel instance (each instance on its class
    // stream, forked from and joined to `stream`), then the per-matrix finish
    auto enqueue = [&]() -> perm_status {
        bool used[kBatchStreams] = {};
        size_t r0 = 0, b0 = 0;
        if (persistent) HIP_OK(launch_counters_reset(d_counters, (int)plans.size(), stream));
        if (branches) HIP_OK(hipEventRecord(ev_fork, stream));
        for (size_t i = 0; i < plans.size(); ++i) {
            const WavePlan &w = plans[i];
            hipStream_t st = stream;
            if (branches) {
                const int c = w.ng % kBatchStreams;
                st = cls[c];
                if (!used[c]) HIP_OK(hipStreamWaitEvent(st, ev_fork, 0));
                used[c] = true;
            }
            BatchLaunchArgs la;
            la.ranges = d_ranges + r0;
            la.nranges = (int)w.ranges.size();
            la.blk_first = d_blk + b0;
            la.nwaves = (int64_t)w.nwaves;
            la.mats = d_mats;
            la.vals = d_vals;
            la.tops = d_tops;
            la.partials = d_partials;
            HIP_OK(launch_batch_ranges(w.ng, w.zero_skip, w.exact, la, block, persistent ? d_counters + i : nullptr,
                                       grids[i], st));
            r0 += w.ranges.size();
            b0 += w.blk_first.size();
        }
        for (int c = 0; c < kBatchStreams; ++c)
            if (used[c]) {
                HIP_OK(hipEventRecord(ev_join[c], cls[c]));
                HIP_OK(hipStreamWaitEvent(stream, ev_join[c], 0));
            }
        HIP_OK(launch_batch_finish(d_fin, nm, d_partials, d_out, stream));
        return PERM_OK;
    };
    if (how == BatchLaunch::Graph) {
        // The captured graph depends only on the launch layout and the device
        // buffers (the data are copied in before it runs), so a later batch
        // with the same layout relaunches it without capturing again.
        std::string sig;
        auto put = [&](const void *q, size_t n) { sig.append(static_cast<const char *>(q), n); };
        const void *ptrs[] = {d_ranges, d_blk, d_mats, d_vals, d_tops, d_partials, d_fin, d_out, d_counters};
        put(ptrs, sizeof ptrs);
        put(&nm, sizeof nm);
        put(&block, sizeof block);
        for (size_t i = 0; i < plans.size(); ++i) {
            const WavePlan &w = plans[i];
            const int64_t f[] = {w.ng, w.zero_skip, w.exact, (int64_t)w.ranges.size(), (int64_t)w.nwaves, grids[i]};
            put(f, sizeof f);
        }
        if (!graph_exec || sig != graph_sig) {
            if (graph_exec) {
                (void)hipGraphExecDestroy(graph_exec);
                graph_exec = nullptr;
            }
            if (graph) {
                (void)hipGraphDestroy(graph);
                graph = nullptr;
            }
            graph_sig.clear();
            HIP_OK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            perm_status es = enqueue();
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(stream, &g);
            if (es != PERM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return es;
            }
            if (ce != hipSuccess) {
                *err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ce);
                return PERM_EDEVICE;
            }
            graph = g;
            HIP_OK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
            graph_sig = sig;
            ++graph_captures;
        }
        HIP_OK(hipGraphLaunch(graph_exec, stream));
    } else {
        perm_status es = enqueue();
        if (es != PERM_OK) return es;
    }
    HIP_OK(hipEventRecord(ev1, stream));
    HIP_OK(hipMemcpyAsync(hout, d_out, (size_t)kPartStride * nm * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    if (kernel_ms) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, ev0, ev1));
        *kernel_ms = ms;
    }
    for (int k = 0; k < nm; ++k)
        for (int c = 0; c < kPartStride; ++c) raw[(size_t)kPartStride * order[k] + c] = hout[kPartStride * k + c];
    return PERM_OK;
}

}  // namespace permx
