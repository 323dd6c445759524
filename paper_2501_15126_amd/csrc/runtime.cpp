// runtime.cpp -- the C ABI of libperm_mi355x (include/perm.h): device state,
// launch of generated kernels, the fixed-order reduction and the
// introspection entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_host.h"
#include "exact.h"
#include "jit.h"
#include "perm_internal.h"
#include "reduce.h"

using namespace permx;

namespace {

thread_local std::string t_err = "no error";

perm_status fail(perm_status s, const std::string &msg) {
    t_err = msg;
    return s;
}

#define HIP_TRY(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(PERM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Workgroups per launch; larger jobs are split into several launches over
// consecutive chunk ranges (each launch writes its own partials range).  A
// launch also covers at most 2^42 Gray steps (under 3 s even for dense
// matrices), so no single dispatch runs for long.
constexpr int64_t kMaxBlocksPerLaunch = 1 << 16;
constexpr double kMaxStepsPerLaunch = 4398046511104.0;  // 2^42

struct LoadedKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int waves_per_simd = 0;
};

struct DeviceState {
    bool ready = false;
    int device = -1;
    std::string arch;
    hipStream_t stream = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    double *partials = nullptr;
    size_t partials_cap = 0;  // doubles
    double *xg = nullptr;
    size_t xg_cap = 0;        // doubles
    unsigned long long *counts = nullptr;  // evaluated terms per workgroup
    size_t counts_cap = 0;
    double *xparts = nullptr;  // exact mode: (residue, sum |term|) per workgroup
    double *stage = nullptr;   // the final reduction's per-slice results (6 doubles each)
    size_t stage_cap = 0;
    size_t xparts_cap = 0;
    double *out = nullptr;    // 2 doubles, the evaluated-term total (u64), then the 3 exact-mode sums
    double *host_out = nullptr;  // pinned host copy of out
    std::unordered_map<std::string, LoadedKernel> kernels;  // source -> module
};

std::mutex g_mu;  // serialises device use (the library is thread-safe, not concurrent)
DeviceState g_dev;
// device buffers and graph of perm_batch (used under g_mu); never destroyed,
// so that no HIP call runs during static destruction at process exit
BatchJob &g_batch_job = *new BatchJob;
// perm_batch_noalloc's job: its buffers are views of the batch kernels'
// fixed device region, set at device set-up
BatchJob &g_noalloc_job = *new BatchJob;

perm_status ensure_device() {
    if (g_dev.ready) return PERM_OK;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) return fail(PERM_EDEVICE, "no HIP device available");
    HIP_TRY(hipGetDevice(&g_dev.device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, g_dev.device));
    g_dev.arch = prop.gcnArchName;
    if (g_dev.arch.compare(0, 6, "gfx950") != 0)
        return fail(PERM_EDEVICE, "device " + g_dev.arch + " is not gfx950 (MI355X); kernels are built for gfx950 only");
    HIP_TRY(hipStreamCreateWithFlags(&g_dev.stream, hipStreamNonBlocking));
    for (auto &ev : g_dev.ev) HIP_TRY(hipEventCreate(&ev));
    HIP_TRY(hipMalloc(&g_dev.out, 8 * sizeof(double)));
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&g_dev.host_out), 8 * sizeof(double), hipHostMallocDefault));
    // the allocation-free batch form: the device address of the fixed region
    // (this device's copy) and its timing events, once, here
    void *scr = nullptr;
    HIP_TRY(batch_scratch_address(&scr));
    g_noalloc_job.arena = static_cast<char *>(scr);
    g_noalloc_job.arena_bytes = kNoallocScratchBytes;
    HIP_TRY(g_noalloc_job.init_events());
    g_dev.ready = true;
    return PERM_OK;
}

perm_status ensure_buffer(double **buf, size_t *cap, size_t need) {
    if (need <= *cap) return PERM_OK;
    if (*buf) HIP_TRY(hipFree(*buf));
    *buf = nullptr;
    *cap = 0;
    size_t want = need + need / 4;
    if (hipMalloc(buf, want * sizeof(double)) != hipSuccess) {
        *buf = nullptr;
        return fail(PERM_ENOMEM, "device allocation of " + std::to_string(want * 8) + " bytes failed");
    }
    *cap = want;
    return PERM_OK;
}

perm_status load_kernel(const std::string &src, const CodeObject &co, int block, LoadedKernel **out) {
    auto it = g_dev.kernels.find(src);
    if (it == g_dev.kernels.end()) {
        LoadedKernel k;
        HIP_TRY(hipModuleLoadData(&k.mod, co.code.data()));
        HIP_TRY(hipModuleGetFunction(&k.fn, k.mod, kGrayKernelName));
        int blocks_per_cu = 0;
        HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, k.fn, block, 0));
        k.waves_per_simd = blocks_per_cu * (block / 64) / 4;
        it = g_dev.kernels.emplace(src, k).first;
    }
    *out = &it->second;
    return PERM_OK;
}

perm_opts defaults(const perm_opts *o) {
    perm_opts d;
    memset(&d, 0, sizeof d);
    if (o) d = *o;
    return d;
}

// Validation, structural check, plan and source: everything before the GPU.
struct Prepared {
    Ccs a;
    int rank = 0;
    bool singular = false;
    Plan plan;
    std::string src;
    LoopCount lc;  // the generator's count of the step loop's FP64 operations
    double host_ms = 0;
};

// Nested-accumulation kernels: the FP64 operations per Gray term that
// ops_per_step and flops_per_step report are those of the compiled kernel,
// per chunk over the chunk's terms: the step loop's FP64 instructions times
// its iterations, plus the rest of the kernel's once (the chunk's start,
// what the compiler moved out of the loop, the lane's reduction).  An FMA
// counts 2 flops except one adding a signed table entry.  The compiler
// makes these fewer than the generator's count by simplifications of its
// own.
void use_compiled_count(Prepared *p, const CodeObject &co) {
    if (!p->lc.counted || co.all_add < 0 || p->lc.terms_per_iter <= 0 || p->lc.iters < 1) return;
    const double it = (double)p->lc.iters;
    const double t = p->lc.terms_per_iter * it;  // Gray terms of one chunk
    const double all = co.all_add + co.all_mul + co.all_fma;
    const double all_fl = co.all_add + co.all_mul + 2.0 * co.all_fma - p->lc.sign_fmas;
    if (!p->lc.loop) {
        // one pass over the chunk: straight-line code, each instruction once
        p->plan.ops_per_step = all / t;
        p->plan.flops_per_step = all_fl / t;
        return;
    }
    if (co.loop_add < 0) return;
    const double loop = co.loop_add + co.loop_mul + co.loop_fma;
    // the loop found in the machine code must be the step loop: far fewer
    // FP64 instructions than the generator counts for one iteration means
    // it was not found, and the generator's count stays
    if (loop < 0.25 * p->lc.body_ops) return;
    const double loop_fl = co.loop_add + co.loop_mul + 2.0 * co.loop_fma - p->lc.sign_fmas;
    p->plan.ops_per_step = (loop * it + (all - loop)) / t;
    p->plan.flops_per_step = (loop_fl * it + (all_fl - loop_fl)) / t;
}

perm_status prepare(const perm_csc *m, const perm_opts &o, Prepared *p, bool want_source, int tau_base = 0) {
    auto t0 = std::chrono::steady_clock::now();
    std::string err;
    perm_status s = normalize_ccs(m, &p->a, &err);
    if (s != PERM_OK) return fail(s, err);
    p->rank = structural_rank(p->a);
    p->singular = p->rank < p->a.n;
    if (!p->singular || !want_source) {
        s = make_plan(p->a, o, &p->plan, &err, tau_base);
        if (s != PERM_OK) return fail(s, err);
        if (want_source && !p->singular) p->src = generate_source(p->plan, &p->lc);
    }
    p->host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return PERM_OK;
}

// Largest per-lane scratch accepted from the second, higher-occupancy build
// of the automatic occupancy choice (16 doubles).
constexpr int kAutoWavesMaxScratch = 128;

// Compiles p->src.  With the occupancy left automatic, a kernel that the
// compiler holds to 4 waves per SIMD (97..128 VGPRs; 512 VGPRs per SIMD lane,
// allocated in steps of 8) is generated and compiled again for 5 waves, and
// one held to 3 waves (129..168 VGPRs) again for 4; the second build replaces
// the first if it spills little: one more wave hides more of the FP64
// dependency and branch latency than the few spilled values cost.  Kernels
// with LDS-resident rows are left alone (their LDS use already bounds the
// occupancy).
perm_status compile_prepared_build(Prepared *p, const perm_opts &o, CodeObject *co, std::string *err) {
    perm_status s = compile_source(p->src, co, err);
    if (s != PERM_OK) return s;
    // Paired kernels in nested form with automatically chosen copies: a build
    // that spills is generated again with one copied column fewer, up to
    // three times (ER n = 48, p = 0.1, chunks of 2^16: copies of 13 columns
    // spill 492 bytes per lane and run 975 ms, of 12 none, 455 ms).  In the
    // exact mode the error bound's length is taken from the new code's
    // count.  (Unpaired nested kernels keep their copies: untimed there, and
    // one column fewer adds 24 % to the operations of an n = 36 0/1 kernel
    // whose build spills a little.)
    for (int tries = 0; tries < 3 && co->scratch_bytes > 0; ++tries) {
        const Plan &pl = p->plan;
        if (!(pl.pair0 && pl.nested && o.copy_cols == 0 && pl.copy_cols >= 1)) break;
        Plan q = pl;
        q.copy_cols -= 1;
        LoopCount lc;
        std::string src2 = generate_source(q, &lc);
        if (q.exact) {
            if (!lc.counted) break;
            q.acc_log2 = std::max(q.acc_log2, lc.acc_log2);
        }
        CodeObject c2;
        std::string err2;
        if (compile_source(src2, &c2, &err2) != PERM_OK) break;  // keep the build we have
        c2.compile_ms += co->compile_ms;
        c2.cache_hit = c2.cache_hit && co->cache_hit;
        p->plan = q;
        p->src = std::move(src2);
        *co = std::move(c2);
    }
    if (o.waves_per_simd != 0 || p->plan.cold_lds) return s;
    if (co->vgprs <= 96 || co->vgprs > 168) return PERM_OK;
    Plan q = p->plan;
    q.waves_per_simd = co->vgprs <= 128 ? 5 : 4;
    std::string src5 = generate_source(q);
    CodeObject c5;
    std::string err5;
    if (compile_source(src5, &c5, &err5) != PERM_OK) return PERM_OK;  // keep the first build
    if (c5.scratch_bytes < 0 || c5.scratch_bytes > kAutoWavesMaxScratch) return PERM_OK;
    c5.compile_ms += co->compile_ms;
    c5.cache_hit = c5.cache_hit && co->cache_hit;
    p->plan.waves_per_simd = q.waves_per_simd;
    p->src = std::move(src5);
    *co = std::move(c5);
    return PERM_OK;
}

perm_status compile_prepared(Prepared *p, const perm_opts &o, CodeObject *co, std::string *err) {
    const perm_status s = compile_prepared_build(p, o, co, err);
    if (s == PERM_OK) use_compiled_count(p, *co);
    return s;
}

// compile_prepared, then for a HYBRID plan whose partition is not forced:
// Alg. 5 once more with the thread-count model of the compiled kernel (its
// VGPRs besides the register rows of x replace the estimate); a different
// (k, c) is compiled and replaces the first.
perm_status compile_plan(const perm_csc *m, const perm_opts &o, Prepared *p, CodeObject *co, std::string *err) {
    perm_status s = compile_prepared(p, o, co, err);
    if (s != PERM_OK) return s;
    const Plan &pl = p->plan;
    if (pl.mode != PERM_MODE_HYBRID || o.force_k > 0 || co->vgprs <= 0) return PERM_OK;
    const int base = co->vgprs - 2 * pl.k;
    if (base <= 0 || std::abs(base - pl.tau_base) < 8) return PERM_OK;
    Prepared q;
    s = prepare(m, o, &q, true, base);
    if (s != PERM_OK) {
        *err = "re-planning with the measured register model failed";
        return s;
    }
    if (q.plan.k == pl.k && q.plan.c == pl.c) {
        p->plan.tau_base = base;
        return PERM_OK;
    }
    CodeObject c2;
    s = compile_prepared(&q, o, &c2, err);
    if (s != PERM_OK) return s;
    c2.compile_ms += co->compile_ms;
    q.host_ms += p->host_ms;
    *p = std::move(q);
    *co = std::move(c2);
    return PERM_OK;
}

// Length of the exact mode's error bound: a chunk's accumulate operations
// (one per term for the cached-product kernels; nested accumulators: the
// generator's count of every accumulator operation of a chunk, plus n).
int exact_bound_log2(const Plan &pl) { return pl.nested ? std::max(pl.acc_log2, pl.kappa) : pl.kappa; }

void fill_plan_stats(const Prepared &p, perm_stats *st) {
    st->n = p.a.n;
    st->nnz = p.a.nnz();
    st->host_ms = p.host_ms;
    st->steps = std::ldexp(1.0, p.a.n - 1);
    st->singular = p.singular ? 1 : 0;
    if (p.singular) return;
    const Plan &pl = p.plan;
    st->mode = pl.mode;
    st->k = pl.k;
    st->c = pl.c;
    st->levels = pl.nlevels;
    st->chunk_log2 = pl.kappa;
    st->unroll_log2 = pl.u;
    st->block = pl.block;
    st->ops_per_step = pl.ops_per_step;
    st->flops_per_step = pl.flops_per_step;
    st->exact_ops_per_step = pl.exact_ops_per_step;
    st->exact = pl.exact ? 0 : -1;  // set to 1 once a result is certified
    st->exact_bound_log2 = pl.exact ? exact_bound_log2(pl) : 0;
    st->copy_cols = pl.nested ? pl.copy_cols : 0;
    st->nchunks = (int64_t)1 << (pl.n - 1 - pl.kappa);
    st->nblocks = (st->nchunks + pl.block - 1) / pl.block;
}

// Plans and compiled code of recently seen inputs, keyed by the exact input
// bytes and the options that shape the plan.  Validation, the matching,
// Alg. 4/5 and the source text cost about 0.15 ms per call; a repeated call
// with the same matrix skips them (the permanent itself is always computed
// on the device).
struct CachedPlan {
    Prepared p;
    CodeObject co;
    LoadedKernel *kern = nullptr;  // set and read under g_mu
};
std::mutex g_plan_mu;
std::unordered_map<std::string, std::shared_ptr<CachedPlan>> g_plan_cache;
constexpr size_t kPlanCacheMax = 256;

bool plan_key(const perm_csc *m, const perm_opts &o, std::string *key) {
    if (!m || m->n < 0 || m->n > PERM_MAX_N || !m->colptr) return false;
    const int32_t n = m->n;
    const int32_t nnz = m->colptr[n];
    if (nnz < 0 || (int64_t)nnz > (int64_t)n * n || (nnz > 0 && (!m->rowidx || !m->val))) return false;
    key->clear();
    auto put = [&](const void *q, size_t b) { key->append(static_cast<const char *>(q), b); };
    put(&n, sizeof n);
    put(m->colptr, sizeof(int32_t) * ((size_t)n + 1));
    if (nnz > 0) {
        put(m->rowidx, sizeof(int32_t) * (size_t)nnz);
        put(m->val, sizeof(double) * (size_t)nnz);
    }
    const int32_t f[] = {o.mode,     o.chunk_log2, o.unroll_log2, o.block,     o.vgpr_budget,
                         o.force_k,  o.force_c,    o.max_levels,  o.zero_skip, o.cold_tier,
                         o.waves_per_simd, o.block_queue, o.exact, o.copy_cols};
    put(f, sizeof f);
    put(&o.gr_ratio, sizeof o.gr_ratio);
    return true;
}

// The plan and code object for (m, o): from the plan cache, else prepared,
// compiled and cached.
perm_status acquire_plan(const perm_csc *m, const perm_opts &o, std::shared_ptr<CachedPlan> *out, bool *hit) {
    std::string key;
    const bool keyed = plan_key(m, o, &key);
    std::shared_ptr<CachedPlan> cp;
    if (keyed) {
        std::lock_guard<std::mutex> g(g_plan_mu);
        auto it = g_plan_cache.find(key);
        if (it != g_plan_cache.end()) cp = it->second;
    }
    *hit = cp != nullptr;
    if (!cp) {
        cp = std::make_shared<CachedPlan>();
        perm_status s = prepare(m, o, &cp->p, true);
        if (s != PERM_OK) return s;
        if (!cp->p.singular) {
            std::string err;
            s = compile_plan(m, o, &cp->p, &cp->co, &err);
            if (s != PERM_OK) return fail(s, err);
        }
        if (keyed) {
            std::lock_guard<std::mutex> g(g_plan_mu);
            if (g_plan_cache.size() >= kPlanCacheMax) g_plan_cache.clear();
            g_plan_cache.emplace(key, cp);
        }
    }
    *out = std::move(cp);
    return PERM_OK;
}

// What one pass of a plan's kernel over the whole Gray-index space returns.
struct PassOut {
    double hi = 0.0, lo = 0.0;            // term sum (double-double), before the final factor
    double evaluated = 0.0;               // lane-terms evaluated
    double resid = 0.0, abs_sum = 0.0;    // exact mode sums
    double kernel_ms = 0.0, reduce_ms = 0.0;
};

// All launches of one pass (prime: the residue's modulus in exact mode),
// the fixed-order reductions and the copy of the result to the host.  g_mu held.
perm_status run_pass(CachedPlan &cp, double prime, const perm_opts &o, hipStream_t stream, double *block_partials,
                     int64_t block_partials_cap, PassOut *po) {
    const Plan &pl = cp.p.plan;
    LoadedKernel *kern = cp.kern;
    const int64_t nchunks = (int64_t)1 << (pl.n - 1 - pl.kappa);
    const int64_t nblocks = (nchunks + pl.block - 1) / pl.block;
    const double steps_per_block = std::ldexp((double)pl.block, pl.kappa);
    const int64_t launch_blocks = std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>(nblocks, kMaxBlocksPerLaunch),
                             (int64_t)(kMaxStepsPerLaunch / steps_per_block)));
    perm_status s = ensure_buffer(&g_dev.partials, &g_dev.partials_cap, 2 * (size_t)nblocks);
    if (s != PERM_OK) return s;
    s = ensure_buffer(reinterpret_cast<double **>(&g_dev.counts), &g_dev.counts_cap, (size_t)nblocks);
    if (s != PERM_OK) return s;
    if (pl.exact) {
        s = ensure_buffer(&g_dev.xparts, &g_dev.xparts_cap, 2 * (size_t)nblocks);
        if (s != PERM_OK) return s;
    }
    const uint64_t xs = (uint64_t)launch_blocks * pl.block;  // lanes of one launch
    if (pl.cold && !pl.cold_lds) {
        s = ensure_buffer(&g_dev.xg, &g_dev.xg_cap, (size_t)(pl.n - pl.k) * xs);
        if (s != PERM_OK) return s;
    }
    const double pmod = prime, pinv = prime > 0.0 ? 1.0 / prime : 0.0;
    HIP_TRY(hipEventRecord(g_dev.ev[0], stream));
    const int64_t nlaunch = (nblocks + launch_blocks - 1) / launch_blocks;
    std::vector<hipEvent_t> done;  // per launch, only with o.progress
    for (int64_t b0 = 0; b0 < nblocks; b0 += launch_blocks) {
        const int64_t nb = std::min<int64_t>(launch_blocks, nblocks - b0);
        uint64_t chunk_begin = (uint64_t)b0 * pl.block;
        uint64_t chunk_end = std::min<uint64_t>((uint64_t)nchunks, chunk_begin + (uint64_t)nb * pl.block);
        double *part = g_dev.partials + 2 * b0;
        unsigned long long *cnt = g_dev.counts + b0;
        double *xg = g_dev.xg;
        uint64_t xs_arg = xs;
        double *xp = pl.exact ? g_dev.xparts + 2 * b0 : nullptr;
        double pm = pmod, pi = pinv;
        void *args[] = {&chunk_begin, &chunk_end, &part, &cnt, &xg, &xs_arg, &xp, &pm, &pi};
        HIP_TRY(hipModuleLaunchKernel(kern->fn, (unsigned)nb, 1, 1, (unsigned)pl.block, 1, 1, 0, stream, args,
                                      nullptr));
        if (o.progress > 0 && nlaunch > 1) {
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            done.push_back(e);
            HIP_TRY(hipEventRecord(e, stream));
        }
    }
    // all launches are queued; report each as it completes (the device never
    // waits for the host here)
    for (size_t i = 0; i < done.size(); ++i) {
        const hipError_t e = hipEventSynchronize(done[i]);
        fprintf(stderr, "perm: n=%d launch %zu of %lld done\n", pl.n, i + 1, (long long)nlaunch);
        fflush(stderr);
        (void)hipEventDestroy(done[i]);
        if (e != hipSuccess) {
            for (size_t j = i + 1; j < done.size(); ++j) (void)hipEventDestroy(done[j]);
            return fail(PERM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
        }
    }
    HIP_TRY(hipEventRecord(g_dev.ev[1], stream));
    s = ensure_buffer(&g_dev.stage, &g_dev.stage_cap, 6 * (size_t)final_reduce_slices((long long)nblocks));
    if (s != PERM_OK) return s;
    HIP_TRY(launch_final_reduce(g_dev.partials, g_dev.counts, pl.exact ? g_dev.xparts : nullptr, (long long)nblocks,
                                g_dev.stage, g_dev.out, stream));
    HIP_TRY(hipEventRecord(g_dev.ev[2], stream));
    double *hl = g_dev.host_out;  // pinned: the result copy is a plain DMA
    HIP_TRY(hipMemcpyAsync(hl, g_dev.out, (pl.exact ? 5 : 3) * sizeof(double), hipMemcpyDeviceToHost, stream));
    if (block_partials && block_partials_cap >= nblocks)
        HIP_TRY(hipMemcpyAsync(block_partials, g_dev.partials, 2 * sizeof(double) * (size_t)nblocks,
                               hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, g_dev.ev[0], g_dev.ev[1]));
    po->kernel_ms = ms;
    HIP_TRY(hipEventElapsedTime(&ms, g_dev.ev[1], g_dev.ev[2]));
    po->reduce_ms = ms;
    po->hi = hl[0];
    po->lo = hl[1];
    unsigned long long ev = 0;
    memcpy(&ev, &hl[2], sizeof ev);
    po->evaluated = (double)ev;
    if (pl.exact) {
        po->resid = hl[3];
        po->abs_sum = hl[4];
    }
    return PERM_OK;
}

perm_status run_one(const perm_csc *m, const perm_opts *opts, double *out, perm_stats *st_out) {
    auto t0 = std::chrono::steady_clock::now();
    perm_stats st;
    memset(&st, 0, sizeof st);
    const perm_opts o = defaults(opts);
    std::shared_ptr<CachedPlan> cp;
    bool plan_hit = false;
    {
        perm_status s = acquire_plan(m, o, &cp, &plan_hit);
        if (s != PERM_OK) return s;
    }
    const Prepared &p = cp->p;
    const CodeObject &co = cp->co;
    fill_plan_stats(p, &st);
    st.host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() -
                 (plan_hit ? 0.0 : co.compile_ms);
    if (p.singular) {
        *out = 0.0;  // no perfect matching: every permutation product has a zero factor
        st.exact = 1;
        st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (st_out) *st_out = st;
        return PERM_OK;
    }
    st.compile_ms = plan_hit ? 0.0 : co.compile_ms;
    st.cache_hit = (plan_hit || co.cache_hit) ? 1 : 0;
    st.vgprs = co.vgprs;
    st.sgprs = co.sgprs;
    st.scratch_bytes = co.scratch_bytes;
    st.lds_bytes = co.lds_bytes;
    st.waves_hint = p.plan.waves_per_simd;
    st.vgpr_spills = co.vgpr_spills;
    std::lock_guard<std::mutex> g(g_mu);
    perm_status s = ensure_device();
    if (s != PERM_OK) return s;
    if (!cp->kern) {
        s = load_kernel(p.src, co, p.plan.block, &cp->kern);
        if (s != PERM_OK) return s;
    }
    st.waves_per_simd = cp->kern->waves_per_simd;

    const Plan &pl = p.plan;
    if (o.exact_passes < 0 || o.exact_passes > kExactMaxPasses)
        return fail(PERM_EINVAL, "exact_passes must be 0..3");
    hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : g_dev.stream;
    // one pass per prime: the FP64 sum, A and E are the same in every pass
    // (same code, same order); only the residue's prime changes
    PassOut po;
    ExactSums es;
    double kernel_ms = 0.0, reduce_ms = 0.0;
    ExactOutcome eo;
    for (int pass = 0;; ++pass) {
        const double prime = pl.exact ? kExactPrimes[pass] : 0.0;
        s = run_pass(*cp, prime, o, stream, pass == 0 ? o.block_partials : nullptr,
                     pass == 0 ? o.block_partials_cap : 0, &po);
        if (s != PERM_OK) return s;
        kernel_ms += po.kernel_ms;
        reduce_ms += po.reduce_ms;
        if (!pl.exact) break;
        es.hi = po.hi;
        es.lo = po.lo;
        es.abs_sum = po.abs_sum;
        es.chunk_log2 = exact_bound_log2(pl);
        es.resid[pass] = po.resid;
        es.passes = pass + 1;
        eo = exact_recover(pl.n, es);
        if (es.passes >= kExactMaxPasses) break;
        if (es.passes < o.exact_passes) continue;
        if (eo.certified || !eo.more) break;
    }
    st.kernel_ms = kernel_ms;
    st.reduce_ms = reduce_ms;
    st.sum_hi = po.hi;
    st.sum_lo = po.lo;
    st.evaluated_steps = po.evaluated;
    if (pl.exact) {
        // the term sums are in y = 2x units: 2^n times Alg. 1's (exact scaling)
        if (o.block_partials && o.block_partials_cap >= st.nblocks)
            for (int64_t i = 0; i < 2 * st.nblocks; ++i) o.block_partials[i] = std::ldexp(o.block_partials[i], -pl.n);
        st.sum_hi = std::ldexp(po.hi, -pl.n);
        st.sum_lo = std::ldexp(po.lo, -pl.n);
        st.exact = eo.certified ? 1 : 0;
        st.exact_passes = es.passes;
        st.estimate = eo.estimate;
        st.err_bound = eo.err_bound;
        *out = eo.value;
    } else {
        // final factor of Alg. 1: 4 (n mod 2) - 2 = (-1)^(n-1) * 2 (exact scaling)
        const double f = (pl.n % 2 == 1) ? 2.0 : -2.0;
        *out = (po.hi + po.lo) * f;
        st.estimate = *out;
    }
    st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st_out) *st_out = st;
    return PERM_OK;
}

// ---- autotuner -------------------------------------------------------------

// The part of the Gray-index space every tuning candidate is timed on:
// `slices` slices of 2^slice_log2 indices starting at s * 2^(n-1) / slices.
// Each slice is its own launch (or launches), and holds at least 2^19 chunks
// of the largest candidate chunk: 2048 workgroups of 256 lanes, 8 per CU, so
// that every launch fills the GPU as a full run does; when 8 such slices
// would cover the whole space, the whole space is the sample.
struct TuneSample {
    int slices = 1;
    int slice_log2 = 0;
};

constexpr int kTuneSlicesLog2 = 3;
constexpr int kTuneSliceChunksLog2 = 19;

TuneSample tune_sample(int n, int max_kappa) {
    TuneSample t;
    const int total = n - 1;
    const int q = max_kappa + kTuneSliceChunksLog2;
    if (q + kTuneSlicesLog2 >= total) {
        t.slices = 1;
        t.slice_log2 = total;
    } else {
        t.slices = 1 << kTuneSlicesLog2;
        t.slice_log2 = q;
    }
    return t;
}

// One pass of the plan's kernel over the sample: device time between events
// around the launches, and the sample's Gray-term sum (hi, lo).  g_mu held.
perm_status time_sample(CachedPlan &cp, const TuneSample &ts, hipStream_t stream, float *ms, double sum[2]) {
    const Plan &pl = cp.p.plan;
    if (!cp.kern) {
        perm_status s = load_kernel(cp.p.src, cp.co, pl.block, &cp.kern);
        if (s != PERM_OK) return s;
    }
    const int total = pl.n - 1;
    if (pl.kappa > ts.slice_log2) return fail(PERM_EINVAL, "chunk larger than the tuning sample's slices");
    const uint64_t chunks_per_slice = 1ull << (ts.slice_log2 - pl.kappa);
    const uint64_t B = (uint64_t)pl.block;
    const int64_t blocks_per_slice = (int64_t)((chunks_per_slice + B - 1) / B);
    const int64_t launch_blocks = std::min<int64_t>(blocks_per_slice, kMaxBlocksPerLaunch);
    const int64_t nblocks = blocks_per_slice * ts.slices;
    perm_status s = ensure_buffer(&g_dev.partials, &g_dev.partials_cap, 2 * (size_t)nblocks);
    if (s != PERM_OK) return s;
    s = ensure_buffer(reinterpret_cast<double **>(&g_dev.counts), &g_dev.counts_cap, (size_t)nblocks);
    if (s != PERM_OK) return s;
    const uint64_t xs = (uint64_t)launch_blocks * B;
    if (pl.cold && !pl.cold_lds) {
        s = ensure_buffer(&g_dev.xg, &g_dev.xg_cap, (size_t)(pl.n - pl.k) * xs);
        if (s != PERM_OK) return s;
    }
    if (pl.exact) {
        s = ensure_buffer(&g_dev.xparts, &g_dev.xparts_cap, 2 * (size_t)nblocks);
        if (s != PERM_OK) return s;
    }
    // exact mode: timed with the first prime, as a first pass runs
    double pmod = pl.exact ? kExactPrimes[0] : 0.0, pinv = pl.exact ? 1.0 / kExactPrimes[0] : 0.0;
    HIP_TRY(hipEventRecord(g_dev.ev[0], stream));
    int64_t off = 0;
    for (int sl = 0; sl < ts.slices; ++sl) {
        // first chunk of slice sl: (sl * 2^(total - log2 slices)) >> kappa
        const uint64_t g0 = ts.slices == 1 ? 0 : (uint64_t)sl << (total - kTuneSlicesLog2);
        const uint64_t c0 = g0 >> pl.kappa;
        uint64_t chunk_end = c0 + chunks_per_slice;
        for (int64_t b = 0; b < blocks_per_slice; b += launch_blocks) {
            const int64_t nb = std::min<int64_t>(launch_blocks, blocks_per_slice - b);
            uint64_t chunk_begin = c0 + (uint64_t)b * B;
            double *part = g_dev.partials + 2 * off;
            unsigned long long *cnt = g_dev.counts + off;
            double *xg = g_dev.xg;
            uint64_t xs_arg = xs;
            double *xp = pl.exact ? g_dev.xparts + 2 * off : nullptr;
            void *args[] = {&chunk_begin, &chunk_end, &part, &cnt, &xg, &xs_arg, &xp, &pmod, &pinv};
            HIP_TRY(hipModuleLaunchKernel(cp.kern->fn, (unsigned)nb, 1, 1, (unsigned)B, 1, 1, 0, stream, args,
                                          nullptr));
            off += nb;
        }
    }
    HIP_TRY(hipEventRecord(g_dev.ev[1], stream));
    perm_status rs = ensure_buffer(&g_dev.stage, &g_dev.stage_cap, 6 * (size_t)final_reduce_slices((long long)nblocks));
    if (rs != PERM_OK) return rs;
    HIP_TRY(launch_final_reduce(g_dev.partials, g_dev.counts, nullptr, (long long)nblocks, g_dev.stage, g_dev.out,
                                stream));
    HIP_TRY(hipMemcpyAsync(g_dev.host_out, g_dev.out, 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipEventElapsedTime(ms, g_dev.ev[0], g_dev.ev[1]));
    sum[0] = g_dev.host_out[0];
    sum[1] = g_dev.host_out[1];
    return PERM_OK;
}

// Relative gain a candidate must show over the current best to be adopted
// (the spread of repeated sample timings is below 1 %).
constexpr double kTuneMinGain = 0.02;
constexpr int kTuneRepeats = 3;
constexpr double kTuneLongPassMs = 100.0;
// Further steps past a winning edge candidate (chunk) or first step (static
// block), at most.
constexpr int kTuneMaxExtraSteps = 3;

perm_status autotune_one(const perm_csc *a, const perm_opts *opts, perm_opts *best, perm_tune_stats *ts_out) {
    const auto t0 = std::chrono::steady_clock::now();
    perm_tune_stats ts;
    memset(&ts, 0, sizeof ts);
    perm_opts cur = defaults(opts);
    cur.block_partials = nullptr;
    cur.block_partials_cap = 0;
    cur.progress = 0;
    TuneSample smp;  // set from the starting plan's chunk size
    // sampled device time of one option set; the resolved plan in *pl
    auto eval = [&](const perm_opts &c, double *ms, Plan *pl, bool *singular) -> perm_status {
        std::shared_ptr<CachedPlan> cp;
        bool hit = false;
        perm_status s = acquire_plan(a, c, &cp, &hit);
        if (s != PERM_OK) return s;
        *singular = cp->p.singular;
        if (cp->p.singular) return PERM_OK;
        if (pl) *pl = cp->p.plan;
        std::lock_guard<std::mutex> g(g_mu);
        s = ensure_device();
        if (s != PERM_OK) return s;
        hipStream_t stream = c.hip_stream ? (hipStream_t)c.hip_stream : g_dev.stream;
        if (smp.slice_log2 == 0) smp = tune_sample(cp->p.plan.n, cp->p.plan.kappa + 2);
        double bestms = std::numeric_limits<double>::infinity();
        for (int r = 0; r < kTuneRepeats; ++r) {
            float t = 0;
            double sum[2];
            s = time_sample(*cp, smp, stream, &t, sum);
            if (s != PERM_OK) return s;
            bestms = std::min(bestms, (double)t);
            if (t > kTuneLongPassMs) break;  // one pass of a long sample is enough
        }
        *ms = bestms;
        ts.candidates++;
        return PERM_OK;
    };
    Plan plan;
    bool singular = false;
    double best_ms = 0;
    perm_status s = eval(cur, &best_ms, &plan, &singular);
    if (s != PERM_OK) return s;
    if (singular) {
        *best = cur;
        ts.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (ts_out) *ts_out = ts;
        return PERM_OK;
    }
    ts.default_ms = best_ms;
    ts.sample_fraction = std::ldexp((double)smp.slices, smp.slice_log2 - (plan.n - 1));
    // try each candidate of one dimension against the current best; keep the
    // fastest if it gains at least kTuneMinGain
    auto try_dim = [&](const std::vector<perm_opts> &cands) -> perm_status {
        const perm_opts *win = nullptr;
        double win_ms = best_ms * (1.0 - kTuneMinGain);
        Plan win_plan;
        for (const perm_opts &c : cands) {
            double ms = 0;
            Plan pl;
            bool sg = false;
            perm_status r = eval(c, &ms, &pl, &sg);
            if (r == PERM_EINVAL || r == PERM_ECOMPILE) continue;  // not a valid shape here
            if (r != PERM_OK) return r;
            if (ms < win_ms) {
                win = &c;
                win_ms = ms;
                win_plan = pl;
            }
        }
        if (win) {
            cur = *win;
            best_ms = win_ms;
            plan = win_plan;
        }
        return PERM_OK;
    };
    std::vector<perm_opts> cands;
    // 1. register / global split: AUTO (all rows in VGPRs), HYBRID with the
    //    cold rows in global memory or in LDS
    if (cur.mode == PERM_MODE_AUTO || cur.mode == PERM_MODE_HYBRID) {
        cands.clear();
        perm_opts c = cur;
        c.chunk_log2 = c.unroll_log2 = c.block = 0;
        if (cur.mode == PERM_MODE_AUTO) {
            c.mode = PERM_MODE_HYBRID;
            c.cold_tier = 0;
            cands.push_back(c);
            c.cold_tier = 1;
            cands.push_back(c);
        } else {
            c.mode = PERM_MODE_AUTO;
            c.cold_tier = 0;
            cands.push_back(c);
            c.mode = PERM_MODE_HYBRID;
            c.cold_tier = cur.cold_tier == 1 ? 0 : 1;
            cands.push_back(c);
        }
        s = try_dim(cands);
        if (s != PERM_OK) return s;
    }
    // 2. chunk size (log2 of Gray steps per lane); when a candidate at the
    //    edge of the range wins, the search goes on past it one step at a time
    //    while it keeps winning
    {
        const int k0 = plan.kappa;
        cands.clear();
        for (int d : {-2, -1, 1, 2}) {
            const int k = plan.kappa + d;
            if (k < 1 || k > smp.slice_log2) continue;
            perm_opts c = cur;
            c.chunk_log2 = k;
            cands.push_back(c);
        }
        s = try_dim(cands);
        if (s != PERM_OK) return s;
        const int dir = plan.kappa == k0 + 2 ? 1 : plan.kappa == k0 - 2 ? -1 : 0;
        for (int more = 0; dir != 0 && more < kTuneMaxExtraSteps; ++more) {
            const int before = plan.kappa;
            const int k = before + dir;
            if (k < 1 || k > smp.slice_log2) break;
            perm_opts c = cur;
            c.chunk_log2 = k;
            cands.assign(1, c);
            s = try_dim(cands);
            if (s != PERM_OK) return s;
            if (plan.kappa == before) break;
        }
    }
    // 3. static block (log2 of unrolled steps); a side that wins is followed
    //    one step further at a time while it keeps winning
    {
        const int u0 = plan.u;
        cands.clear();
        for (int d : {-1, 1}) {
            const int u = plan.u + d;
            if (u < 1 || u > plan.kappa - 1) continue;
            perm_opts c = cur;
            c.chunk_log2 = plan.kappa;
            c.unroll_log2 = u;
            cands.push_back(c);
        }
        s = try_dim(cands);
        if (s != PERM_OK) return s;
        const int dir = plan.u > u0 ? 1 : plan.u < u0 ? -1 : 0;
        for (int more = 0; dir != 0 && more < kTuneMaxExtraSteps; ++more) {
            const int before = plan.u;
            const int u = before + dir;
            if (u < 1 || u > plan.kappa - 1) break;
            perm_opts c = cur;
            c.chunk_log2 = plan.kappa;
            c.unroll_log2 = u;
            cands.assign(1, c);
            s = try_dim(cands);
            if (s != PERM_OK) return s;
            if (plan.u == before) break;
        }
    }
    // 4. threads per workgroup
    cands.clear();
    for (int b : {64, 128, 256}) {
        if (b == plan.block) continue;
        perm_opts c = cur;
        c.chunk_log2 = plan.kappa;
        c.unroll_log2 = plan.u;
        c.block = b;
        cands.push_back(c);
    }
    s = try_dim(cands);
    if (s != PERM_OK) return s;
    // 5. queue of partly needed blocks (zero-aware kernels): off or its size
    if (plan.zero_skip) {
        cands.clear();
        for (int q : {-1, 16, 32, 64}) {
            if (q == cur.block_queue) continue;
            perm_opts c = cur;
            c.chunk_log2 = plan.kappa;
            c.unroll_log2 = plan.u;
            c.block = plan.block;
            c.block_queue = q;
            cands.push_back(c);
        }
        s = try_dim(cands);
        if (s != PERM_OK) return s;
    }
    // 6. occupancy the kernel is compiled for
    cands.clear();
    for (int w : {-1, 4, 5, 6}) {
        if (w == plan.waves_per_simd || (w == -1 && plan.waves_per_simd == 0)) continue;
        perm_opts c = cur;
        c.chunk_log2 = plan.kappa;
        c.unroll_log2 = plan.u;
        c.block = plan.block;
        c.waves_per_simd = w;
        cands.push_back(c);
    }
    s = try_dim(cands);
    if (s != PERM_OK) return s;
    *best = cur;
    ts.best_ms = best_ms;
    ts.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ts_out) *ts_out = ts;
    return PERM_OK;
}

perm_status autotune_batch(int32_t count, const perm_csc *mats, const perm_opts *opts, perm_opts *best,
                           perm_tune_stats *ts_out) {
    const auto t0 = std::chrono::steady_clock::now();
    perm_tune_stats ts;
    memset(&ts, 0, sizeof ts);
    perm_opts cur = defaults(opts);
    if (cur.batch_mode != 3) cur.batch_mode = 0;  // the sequential baseline is not a candidate
    std::vector<double> out((size_t)std::max(count, 1));
    // device time of the whole batch (the better of kTuneRepeats runs)
    auto eval = [&](const perm_opts &c, double *ms) -> perm_status {
        double b = std::numeric_limits<double>::infinity();
        for (int r = 0; r < kTuneRepeats; ++r) {
            perm_batch_stats bs;
            perm_status s = perm_batch_ex(count, mats, &c, out.data(), &bs);
            if (s != PERM_OK) return s;
            b = std::min(b, bs.kernel_ms);
        }
        *ms = b;
        ts.candidates++;
        return PERM_OK;
    };
    double best_ms = 0;
    perm_status s = eval(cur, &best_ms);
    if (s != PERM_OK) return s;
    ts.default_ms = best_ms;
    ts.sample_fraction = 1.0;
    auto try_all = [&](const std::vector<perm_opts> &cands) -> perm_status {
        int win = -1;
        double win_ms = best_ms * (1.0 - kTuneMinGain);
        for (size_t i = 0; i < cands.size(); ++i) {
            double ms = 0;
            perm_status r = eval(cands[i], &ms);
            if (r != PERM_OK) return r;
            if (ms < win_ms) {
                win = (int)i;
                win_ms = ms;
            }
        }
        if (win >= 0) {
            cur = cands[(size_t)win];
            best_ms = win_ms;
        }
        return PERM_OK;
    };
    // threads per workgroup (launch form: one wave per item on the class
    // streams; the persistent graph form is switched off)
    std::vector<perm_opts> cands;
    for (int b : {64, 128, 256}) {
        if (b == (cur.block > 0 ? cur.block : 256)) continue;
        perm_opts c = cur;
        c.block = b;
        cands.push_back(c);
    }
    s = try_all(cands);
    if (s != PERM_OK) return s;
    // chunk size: shift of the per-matrix chunk log2
    cands.clear();
    for (int d : {-2, -1, 1, 2}) {
        perm_opts c = cur;
        c.batch_kappa_shift = cur.batch_kappa_shift + d;
        cands.push_back(c);
    }
    s = try_all(cands);
    if (s != PERM_OK) return s;
    *best = cur;
    ts.best_ms = best_ms;
    ts.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ts_out) *ts_out = ts;
    return PERM_OK;
}

}  // namespace

void permx::set_last_error(const std::string &msg) { t_err = msg; }

extern "C" {

double perm_sparse(int32_t n, const int32_t *colptr, const int32_t *rowidx, const double *val) {
    perm_csc a{n, colptr, rowidx, val};
    double out = 0.0;
    if (run_one(&a, nullptr, &out, nullptr) != PERM_OK) return std::numeric_limits<double>::quiet_NaN();
    return out;
}

perm_status perm_sparse_ex(const perm_csc *a, const perm_opts *opts, double *out, perm_stats *st) {
    if (!out) return fail(PERM_EINVAL, "null output pointer");
    return run_one(a, opts, out, st);
}

perm_status perm_autotune(const perm_csc *a, const perm_opts *opts, perm_opts *best, perm_tune_stats *st) {
    if (!best) return fail(PERM_EINVAL, "null output options");
    return autotune_one(a, opts, best, st);
}

perm_status perm_batch_autotune(int32_t count, const perm_csc *mats, const perm_opts *opts, perm_opts *best,
                                perm_tune_stats *st) {
    if (!best) return fail(PERM_EINVAL, "null output options");
    if (count < 1 || !mats) return fail(PERM_EINVAL, "bad batch arguments");
    return autotune_batch(count, mats, opts, best, st);
}

}  // extern "C"

namespace {

// perm_batch_ex and its allocation-free form (noalloc: every device buffer is
// a view of the library's fixed scratch region, all launches on one stream,
// the matrices prepared on the calling thread).
perm_status batch_impl(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out,
                       perm_batch_stats *st, bool noalloc) {
    auto t0 = std::chrono::steady_clock::now();
    if (count < 0 || (count > 0 && (!mats || !out))) return fail(PERM_EINVAL, "bad batch arguments");
    const perm_opts o = defaults(opts);
    if (o.batch_mode < 0 || o.batch_mode > 3) return fail(PERM_EINVAL, "batch_mode must be 0, 1, 2 or 3");
    // The persistent form captured across the class streams stopped a GPU
    // test (no progress) without a cause found in this code; until one is
    // shown it stays off.
    if (o.batch_mode == 1)
        return fail(PERM_EINVAL, "batch_mode 1 (persistent instances in a captured graph) is switched off");
    BatchOptions bo;
    bo.zero_skip = o.zero_skip;
    bo.kappa_shift = o.batch_kappa_shift;
    bo.exact = o.exact;
    if (o.exact < -1 || o.exact > 1 || o.exact_passes < 0 || o.exact_passes > kExactMaxPasses)
        return fail(PERM_EINVAL, "exact must be -1, 0 or 1 and exact_passes 0..3");
    std::vector<PreparedMatrix> prep(count);
    std::string err;
    double steps = 0.0, ops = 0.0, fmas = 0.0;
    int singular = 0;
    {
        // the matrices are independent: prepare them on a few host threads
        // (each writes only its own slots), then report the first failure
        std::vector<perm_status> st_of(count, PERM_OK);
        std::vector<std::string> err_of(count);
        const int nthreads =
            noalloc ? 1 : std::max(1, std::min<int>({(int)std::thread::hardware_concurrency(), 8, count / 64}));
        auto work = [&](int t) {
            for (int32_t i = t; i < count; i += nthreads) st_of[i] = prepare_batch_matrix(&mats[i], bo, &prep[i], &err_of[i]);
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
        work(0);
        for (auto &th : pool) th.join();
        for (int32_t i = 0; i < count; ++i)
            if (st_of[i] != PERM_OK) return fail(st_of[i], "matrix " + std::to_string(i) + ": " + err_of[i]);
    }
    for (int32_t i = 0; i < count; ++i) {
        if (prep[i].singular) {
            ++singular;
        } else {
            steps += std::ldexp(1.0, prep[i].n - 1);
            ops += prep[i].fp64_ops;
            fmas += prep[i].fp64_fmas;
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    if (!(o.block == 0 || o.block == 64 || o.block == 128 || o.block == 256))
        return fail(PERM_EINVAL, "perm_batch: block must be 64, 128 or 256 (0 = 256)");
    std::lock_guard<std::mutex> g(g_mu);
    perm_status s = ensure_device();
    if (s != PERM_OK) return s;
    BatchJob &job = noalloc ? g_noalloc_job : g_batch_job;
    job.block = o.block > 0 ? o.block : 256;
    hipStream_t stream = o.hip_stream ? (hipStream_t)o.hip_stream : g_dev.stream;
    double kms = 0.0;
    int launches = 0, passes = 0;
    std::vector<int> xs((size_t)std::max(count, 1), -1);
    if (noalloc) {
        std::vector<const PreparedMatrix *> all;
        for (auto &pm : prep) all.push_back(&pm);
        s = job.run(all, out, stream, BatchLaunch::Single, &kms, &err, xs.data(), &passes, o.exact_passes);
        if (s != PERM_OK) return fail(s, err);
        launches = -1;
    } else if (o.batch_mode == 2) {
        for (int32_t i = 0; i < count; ++i) {
            std::vector<const PreparedMatrix *> one{&prep[i]};
            double k1 = 0.0;
            int np = 0;
            s = job.run(one, &out[i], stream, BatchLaunch::Single, &k1, &err, &xs[i], &np, o.exact_passes);
            if (s != PERM_OK) return fail(s, err);
            kms += k1;
            launches += prep[i].singular ? 0 : 2 * np;
            passes = std::max(passes, np);
        }
    } else {
        std::vector<const PreparedMatrix *> all;
        for (auto &pm : prep) all.push_back(&pm);
        const BatchLaunch how = o.batch_mode == 0   ? BatchLaunch::Streams
                                : o.batch_mode == 1 ? BatchLaunch::Graph
                                                    : BatchLaunch::Single;
        s = job.run(all, out, stream, how, &kms, &err, xs.data(), &passes, o.exact_passes);
        if (s != PERM_OK) return fail(s, err);
        launches = -1;
    }
    if (st) {
        memset(st, 0, sizeof *st);
        st->prep_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st->kernel_ms = kms;
        st->steps = steps;
        st->count = count;
        st->singular = singular;
        st->launches = launches;
        st->fp64_ops = ops;
        st->flops = ops + fmas;
        st->passes = passes;
        st->graph_captures = job.graph_captures;
        for (int32_t i = 0; i < count; ++i) {
            if (xs[i] == 1 && !prep[i].singular) st->exact_certified++;
            if (xs[i] == 0) st->exact_uncertified++;
        }
        double xo = 0.0;
        for (int32_t i = 0; i < count; ++i)
            if (!prep[i].singular) xo += prep[i].exact_ops;
        st->exact_ops = xo;
    }
    return PERM_OK;
}

}  // namespace

extern "C" {

perm_status perm_batch_ex(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out,
                          perm_batch_stats *st) {
    return batch_impl(count, mats, opts, out, st, false);
}

perm_status perm_batch_noalloc(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out,
                               perm_batch_stats *st) {
    return batch_impl(count, mats, opts, out, st, true);
}

perm_status perm_batch(int32_t count, const perm_csc *mats, const perm_opts *opts, double *out) {
    return perm_batch_ex(count, mats, opts, out, nullptr);
}

perm_status perm_plan(const perm_csc *a, const perm_opts *opts, int32_t *row_perm, int32_t *col_perm, double *tau,
                      int32_t *k, int32_t *c, int32_t *levels, int32_t *rank) {
    const perm_opts o = defaults(opts);
    Prepared p;
    perm_status s = prepare(a, o, &p, false);
    if (s != PERM_OK) return s;
    const int n = p.a.n;
    if (rank) *rank = p.rank;
    if (row_perm)
        for (int i = 0; i < n; ++i) row_perm[i] = p.plan.rowPerm[i];
    if (col_perm)
        for (int i = 0; i < n; ++i) col_perm[i] = p.plan.colPerm[i];
    if (tau) {
        std::vector<double> t = tau_model(n, 28);
        for (int i = 0; i <= 2 * n; ++i) tau[i] = t[i];
    }
    if (k) *k = p.plan.k;
    if (c) *c = p.plan.c;
    if (levels) *levels = p.plan.nlevels;
    return PERM_OK;
}

perm_status perm_partition(const perm_csc *ordered, const double *tau, double gr_ratio, int32_t *k, int32_t *c) {
    Ccs a;
    std::string err;
    perm_status s = normalize_ccs(ordered, &a, &err);
    if (s != PERM_OK) return fail(s, err);
    if (!tau || !k || !c) return fail(PERM_EINVAL, "null tau, k or c");
    int kk = 0, cc = 0;
    partitioning(a, tau, gr_ratio > 0 ? gr_ratio : 16.0, &kk, &cc);
    *k = kk;
    *c = cc;
    return PERM_OK;
}

perm_status perm_codegen(const perm_csc *a, const perm_opts *opts, char *buf, size_t cap, size_t *len) {
    const perm_opts o = defaults(opts);
    Prepared p;
    perm_status s = prepare(a, o, &p, true);
    if (s != PERM_OK) return s;
    if (p.singular) return fail(PERM_EINVAL, "structurally singular matrix: no kernel is generated");
    if (len) *len = p.src.size();
    if (buf && cap) {
        size_t nc = std::min(cap - 1, p.src.size());
        memcpy(buf, p.src.data(), nc);
        buf[nc] = '\0';
    }
    return PERM_OK;
}

perm_status perm_compile_info(const perm_csc *a, const perm_opts *opts, perm_stats *st) {
    const perm_opts o = defaults(opts);
    Prepared p;
    perm_status s = prepare(a, o, &p, true);
    if (s != PERM_OK) return s;
    if (!st) return fail(PERM_EINVAL, "null stats");
    memset(st, 0, sizeof *st);
    if (p.singular) {
        fill_plan_stats(p, st);
        return PERM_OK;
    }
    CodeObject co;
    std::string err;
    s = compile_plan(a, o, &p, &co, &err);
    if (s != PERM_OK) return fail(s, err);
    fill_plan_stats(p, st);
    st->waves_hint = p.plan.waves_per_simd;
    st->vgpr_spills = co.vgpr_spills;
    st->compile_ms = co.compile_ms;
    st->cache_hit = co.cache_hit;
    st->vgprs = co.vgprs;
    st->sgprs = co.sgprs;
    st->scratch_bytes = co.scratch_bytes;
    st->lds_bytes = co.lds_bytes;
    return PERM_OK;
}

perm_status perm_batch_describe(const perm_csc *a, const perm_opts *opts, int32_t desc[8], double *vals,
                                size_t vals_cap, size_t *nvals, int32_t *tops, size_t tops_cap, size_t *ntops) {
    const perm_opts o = defaults(opts);
    BatchOptions bo;
    bo.zero_skip = o.zero_skip;
    bo.kappa_shift = o.batch_kappa_shift;
    bo.exact = o.exact;
    PreparedMatrix pm;
    std::string err;
    perm_status s = prepare_batch_matrix(a, bo, &pm, &err);
    if (s != PERM_OK) return fail(s, err);
    if (!desc) return fail(PERM_EINVAL, "null desc");
    desc[0] = pm.n;
    desc[1] = pm.ng;
    desc[2] = pm.kappa;
    desc[3] = pm.zero_skip ? 1 : 0;
    desc[4] = pm.chunk_top;
    desc[5] = pm.singular ? 1 : 0;
    desc[6] = pm.exact ? 1 : 0;
    desc[7] = 0;
    if (nvals) *nvals = pm.vals.size();
    if (ntops) *ntops = pm.tops.size();
    if (vals && vals_cap >= pm.vals.size()) memcpy(vals, pm.vals.data(), pm.vals.size() * sizeof(double));
    if (tops && tops_cap >= pm.tops.size()) memcpy(tops, pm.tops.data(), pm.tops.size() * sizeof(int32_t));
    return PERM_OK;
}

perm_status perm_exact_recover(int32_t n, double hi, double lo, double abs_sum, int32_t chunk_log2, int32_t passes,
                               const double *resid, double out[3], int32_t *certified, int32_t *more) {
    if (n < 1 || n > PERM_MAX_N || passes < 0 || passes > kExactMaxPasses || chunk_log2 < 0 || chunk_log2 > 40 ||
        !out || !certified || !more || (passes > 0 && !resid))
        return fail(PERM_EINVAL, "bad perm_exact_recover arguments");
    ExactSums es;
    es.hi = hi;
    es.lo = lo;
    es.abs_sum = abs_sum;
    es.chunk_log2 = chunk_log2;
    es.passes = passes;
    for (int i = 0; i < passes; ++i) es.resid[i] = resid[i];
    const ExactOutcome eo = exact_recover(n, es);
    out[0] = eo.value;
    out[1] = eo.estimate;
    out[2] = eo.err_bound;
    *certified = eo.certified ? 1 : 0;
    *more = eo.more ? 1 : 0;
    return PERM_OK;
}

void perm_exact_primes(double out[3]) {
    for (int i = 0; i < kExactMaxPasses; ++i) out[i] = kExactPrimes[i];
}

const char *perm_last_error(void) { return t_err.c_str(); }

const char *perm_version(void) { return "perm_mi355x 0.1 (gfx950)"; }

}  // extern "C"
