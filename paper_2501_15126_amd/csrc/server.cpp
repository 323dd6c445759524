// server.cpp -- the submit/poll permanent server (continuous batching).
//
// Requests are validated and prepared for the precompiled batch kernels on
// the submitting thread.  A scheduler thread admits them in arrival order as
// device memory frees up (one arena of `device_mem_budget` bytes holds each
// admitted request's matrix data and partial sums) and runs rounds.  A round
// of `round_steps` Gray steps first finishes every small request (at most a
// quarter of a round left), then gives the rest to the larger requests in
// arrival order, as 64-chunk work items, and issues them as one launch per
// kernel instance on that instance's class stream; the requests whose last items are in the
// round are finished on the same stream.  Two rounds are in flight: while the
// GPU runs one, the scheduler publishes the previous one's results, admits new
// requests and issues the next, so a request that arrives while others run
// joins the next round and the GPU does not wait for the host between rounds.
// A request's upload, items and finish all run on its class stream, in order,
// and its result depends only on its own items and their fixed-order sum, so
// it is bitwise the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "batch_host.h"
#include "exact.h"
#include "perm.h"
#include "perm_internal.h"

using namespace permx;

namespace {

// The server's chunks are 2^3 times smaller than perm_batch's for the same
// options: a request then spans more, shorter waves, so rounds interleave
// requests at a finer grain.  Measured on the serving mix (Poisson, n 12..36):
// at 400 req/s p50 / p99 went from 6.5 / 106 ms (shift 0) to 1.2 / 76 ms
// (-3); -2 and -4 were between, -5 worse again.
constexpr int kServerChunkShift = -3;

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;

// First-fit allocator over [0, size) in kAlign units, with coalescing.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

enum class State { Pending, Active, Done };

struct Request {
    uint64_t ticket = 0;
    PreparedMatrix pm;
    State state = State::Pending;
    perm_status status = PERM_OK;
    double result = 0.0;
    size_t bytes = 0, arena_off = 0;
    size_t vals_bytes = 0;
    uint64_t items_total = 0, next_item = 0;
    Clock::time_point t_submit, t_done;
    // exact mode: sums of the passes so far; pass = index of the running prime
    ExactSums es;
    int pass = 0;
    int exact_state = -1;  // 1 certified exact, 0 exact mode without a certificate, -1 not exact mode
};

size_t request_bytes(const PreparedMatrix &pm, uint64_t items, size_t *vals_bytes) {
    *vals_bytes = (pm.vals.size() * sizeof(double) + kAlign - 1) / kAlign * kAlign;
    const size_t tops = (pm.tops.size() * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign;
    const size_t parts = (items * kPartStride * sizeof(double) + kAlign - 1) / kAlign * kAlign;
    return *vals_bytes + tops + parts;
}

template <typename T>
bool grow_dev(T **p, size_t *cap, size_t need) {
    if (need <= *cap) return true;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = std::max<size_t>(need * 2, 64);
    if (hipMalloc(p, want * sizeof(T)) != hipSuccess) return false;
    *cap = want;
    return true;
}

template <typename T>
bool grow_host(T **p, size_t *cap, size_t need) {
    if (need <= *cap) return true;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = std::max<size_t>(need * 2, 64);
    if (hipHostMalloc(reinterpret_cast<void **>(p), want * sizeof(T), hipHostMallocDefault) != hipSuccess)
        return false;
    *cap = want;
    return true;
}

}  // namespace

// One class stream's share of a round slot: descriptor buffers, pinned
// staging and the event that marks the stream's part of the round done.
struct ClassBuf {
    BatchMat *d_mats = nullptr;
    BatchRange *d_ranges = nullptr;
    int32_t *d_blk = nullptr;
    FinishDesc *d_fin = nullptr;
    double *d_out = nullptr;
    size_t cap_mats = 0, cap_ranges = 0, cap_blk = 0, cap_fin = 0, cap_out = 0;
    char *h_stage = nullptr;
    size_t cap_stage = 0;
    double *h_out = nullptr;
    size_t cap_hout = 0;
    hipEvent_t done = nullptr;
    bool used = false;
    std::vector<Request *> finishing;

    void release() {
        if (d_mats) (void)hipFree(d_mats);
        if (d_ranges) (void)hipFree(d_ranges);
        if (d_blk) (void)hipFree(d_blk);
        if (d_fin) (void)hipFree(d_fin);
        if (d_out) (void)hipFree(d_out);
        if (h_stage) (void)hipHostFree(h_stage);
        if (h_out) (void)hipHostFree(h_out);
        if (done) (void)hipEventDestroy(done);
    }
};

struct Slot {
    ClassBuf cls[kBatchStreams];
    bool busy = false;
};

struct perm_server {
    perm_opts opts;
    BatchOptions bo;
    size_t budget = 0;
    int max_inflight = 0;
    double round_steps = 0;  // Gray steps per round (shared by the active requests)

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;
    std::thread worker;

    // statistics
    uint64_t n_submitted = 0, n_completed = 0, n_rounds = 0, n_extra_passes = 0;
    uint64_t n_exact_certified = 0, n_exact_uncertified = 0;
    size_t peak_bytes = 0;
    double busy_ms = 0.0;
    Clock::time_point busy_since;

    // device side (worker thread only, after creation)
    int device = 0;
    hipStream_t streams[kBatchStreams] = {};
    char *arena = nullptr;
    Arena alloc;
    Slot slots[2];

    void run();
    void admit(std::vector<Request *> &newly);
    bool dispatchable() const;
    bool issue(Slot &slot, const std::vector<Request *> &newly, std::string *err);
    bool complete(Slot &slot, std::string *err);
};

void perm_server::admit(std::vector<Request *> &newly) {
    // in arrival order while the arena has room (no overtaking)
    while (!pending.empty()) {
        Request *r = pending.front();
        size_t off = 0;
        if (!alloc.alloc(r->bytes, &off)) break;
        r->arena_off = off;
        pending.pop_front();
        newly.push_back(r);
    }
    peak_bytes = std::max(peak_bytes, alloc.used());
}

bool perm_server::dispatchable() const {
    for (const Request *r : active)
        if (r->next_item < r->items_total) return true;
    return false;
}

#define SRV_HIP(call)                                                 \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) {                                       \
            *err = std::string(#call) + ": " + hipGetErrorString(e_); \
            return false;                                             \
        }                                                             \
    } while (0)

bool perm_server::issue(Slot &slot, const std::vector<Request *> &newly, std::string *err) {
    if (!slots[0].busy && !slots[1].busy) busy_since = Clock::now();
    // ---- shares of round_steps: small requests first, then oldest first ----
    // A request whose remaining work is at most a quarter of a round takes
    // all of it now (oldest first, within the round's budget), so short
    // requests finish in the next round whatever else is queued.  The rest of
    // the budget goes to the larger requests in arrival order, each as much
    // as it can use, so the oldest large request finishes as soon as the
    // device allows and the next ones fill what it leaves (equal shares among
    // all active requests slowed the largest ones most at high load).
    struct Take {
        Request *r;
        uint64_t items;
    };
    std::vector<Request *> cand;
    for (Request *r : active)
        if (r->next_item < r->items_total) cand.push_back(r);
    std::stable_sort(cand.begin(), cand.end(), [](const Request *x, const Request *y) { return x->ticket < y->ticket; });
    auto item_steps = [](const Request *r) { return std::ldexp(64.0, r->pm.kappa); };
    auto remaining = [&](const Request *r) { return (double)(r->items_total - r->next_item) * item_steps(r); };
    std::vector<Take> takes[kBatchStreams];
    double left = round_steps;
    bool any = false;
    for (int pass = 0; pass < 2; ++pass) {
        for (Request *r : cand) {
            const bool small = remaining(r) <= 0.25 * round_steps;
            if ((pass == 0) != small || left <= 0.0) continue;
            const uint64_t rem = r->items_total - r->next_item;
            uint64_t t = small ? rem : std::min<uint64_t>(rem, (uint64_t)(left / item_steps(r)));
            if (t == 0) continue;
            left -= (double)t * item_steps(r);
            takes[r->pm.ng % kBatchStreams].push_back(Take{r, t});
            any = true;
        }
    }
    if (!any && !cand.empty()) {  // a single item larger than the round: still progress
        Request *r = cand.front();
        takes[r->pm.ng % kBatchStreams].push_back(Take{r, 1});
    }
    // ---- per class stream: stage, upload, launch, finish ----
    const double *vals = reinterpret_cast<const double *>(arena);
    const int32_t *tops = reinterpret_cast<const int32_t *>(arena);
    double *parts = reinterpret_cast<double *>(arena);
    for (int c = 0; c < kBatchStreams; ++c) {
        ClassBuf &cb = slot.cls[c];
        cb.used = false;
        cb.finishing.clear();
        std::vector<Request *> up;
        for (Request *r : newly)
            if (r->pm.ng % kBatchStreams == c) up.push_back(r);
        if (takes[c].empty() && up.empty()) continue;
        // launches ordered by kernel instance, larger instances first
        std::stable_sort(takes[c].begin(), takes[c].end(), [](const Take &x, const Take &y) {
            if (x.r->pm.ng != y.r->pm.ng) return x.r->pm.ng > y.r->pm.ng;
            if (x.r->pm.zero_skip != y.r->pm.zero_skip) return x.r->pm.zero_skip;
            return x.r->pm.exact && !y.r->pm.exact;
        });
        std::vector<BatchMat> mats;
        std::vector<WavePlan> plans;
        std::vector<FinishDesc> fin;
        for (const Take &t : takes[c]) {
            Request *r = t.r;
            const PreparedMatrix &pm = r->pm;
            BatchMat d;
            d.n = pm.n;
            d.ng = pm.ng;
            d.kappa = pm.kappa;
            d.zero_skip = pm.zero_skip ? 1 : 0;
            d.chunk_top = pm.chunk_top;
            d.exact = pm.exact ? 1 : 0;
            d.nchunks = pm.nchunks;
            d.col_off = r->arena_off / sizeof(double);
            d.base_off = d.col_off + pm.base_index;
            d.top_off = (r->arena_off + r->vals_bytes) / sizeof(int32_t);
            d.pmod = pm.exact ? kExactPrimes[r->pass] : 0.0;
            d.pinv = pm.exact ? 1.0 / d.pmod : 0.0;
            const int32_t mi = (int32_t)mats.size();
            mats.push_back(d);
            const size_t tops_bytes = (pm.tops.size() * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign;
            const uint64_t part0 = (r->arena_off + r->vals_bytes + tops_bytes) / (kPartStride * sizeof(double));
            if (plans.empty() || plans.back().ng != pm.ng || plans.back().zero_skip != pm.zero_skip ||
                plans.back().exact != pm.exact) {
                plans.emplace_back();
                plans.back().ng = pm.ng;
                plans.back().zero_skip = pm.zero_skip;
                plans.back().exact = pm.exact;
            }
            plans.back().add(mi, r->next_item, t.items, part0 + r->next_item);
            r->next_item += t.items;
            if (r->next_item == r->items_total) {
                fin.push_back(FinishDesc{part0, r->items_total, pm.n, pm.exact ? 1 : 0, d.pmod, d.pinv});
                cb.finishing.push_back(r);
            }
        }
        size_t nranges = 0, nblk = 0, up_bytes = 0;
        for (const WavePlan &w : plans) {
            nranges += w.ranges.size();
            nblk += w.blk_first.size();
        }
        for (Request *r : up) up_bytes += r->vals_bytes + r->pm.tops.size() * sizeof(int32_t) + kAlign;
        const size_t nm = mats.size(), nf = fin.size();
        if (!grow_dev(&cb.d_mats, &cb.cap_mats, std::max<size_t>(nm, 1)) ||
            !grow_dev(&cb.d_ranges, &cb.cap_ranges, std::max<size_t>(nranges, 1)) ||
            !grow_dev(&cb.d_blk, &cb.cap_blk, std::max<size_t>(nblk, 1)) ||
            !grow_dev(&cb.d_fin, &cb.cap_fin, std::max<size_t>(nf, 1)) ||
            !grow_dev(&cb.d_out, &cb.cap_out, kPartStride * std::max<size_t>(nf, 1))) {
            *err = "device allocation for a round failed";
            return false;
        }
        const size_t bytes = nm * sizeof(BatchMat) + nranges * sizeof(BatchRange) + nblk * sizeof(int32_t) +
                             nf * sizeof(FinishDesc) + up_bytes + 256;
        if (!grow_host(&cb.h_stage, &cb.cap_stage, bytes) ||
            !grow_host(&cb.h_out, &cb.cap_hout, kPartStride * std::max<size_t>(nf, 1))) {
            *err = "pinned host allocation for a round failed";
            return false;
        }
        if (!cb.done) SRV_HIP(hipEventCreateWithFlags(&cb.done, hipEventDisableTiming));
        hipStream_t st = streams[c];
        // every host buffer goes through pinned staging so the copies are
        // truly asynchronous; the staging is reused only after `done`
        char *p = cb.h_stage;
        auto put = [&](const void *src, size_t n) {
            char *at = p;
            memcpy(p, src, n);
            p += (n + 15) / 16 * 16;
            return at;
        };
        for (Request *r : up) {
            const PreparedMatrix &pm = r->pm;
            char *sv = put(pm.vals.data(), pm.vals.size() * sizeof(double));
            SRV_HIP(hipMemcpyAsync(arena + r->arena_off, sv, pm.vals.size() * sizeof(double), hipMemcpyHostToDevice, st));
            char *stp = put(pm.tops.data(), pm.tops.size() * sizeof(int32_t));
            SRV_HIP(hipMemcpyAsync(arena + r->arena_off + r->vals_bytes, stp, pm.tops.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, st));
        }
        if (nm) {
            char *sm = put(mats.data(), nm * sizeof(BatchMat));
            SRV_HIP(hipMemcpyAsync(cb.d_mats, sm, nm * sizeof(BatchMat), hipMemcpyHostToDevice, st));
            char *sr = p;
            for (const WavePlan &w : plans) {
                memcpy(p, w.ranges.data(), w.ranges.size() * sizeof(BatchRange));
                p += w.ranges.size() * sizeof(BatchRange);
            }
            SRV_HIP(hipMemcpyAsync(cb.d_ranges, sr, nranges * sizeof(BatchRange), hipMemcpyHostToDevice, st));
            char *sb = p;
            for (const WavePlan &w : plans) {
                memcpy(p, w.blk_first.data(), w.blk_first.size() * sizeof(int32_t));
                p += w.blk_first.size() * sizeof(int32_t);
            }
            p = cb.h_stage + ((size_t)(p - cb.h_stage) + 15) / 16 * 16;
            SRV_HIP(hipMemcpyAsync(cb.d_blk, sb, nblk * sizeof(int32_t), hipMemcpyHostToDevice, st));
            if (nf) {
                char *sf = put(fin.data(), nf * sizeof(FinishDesc));
                SRV_HIP(hipMemcpyAsync(cb.d_fin, sf, nf * sizeof(FinishDesc), hipMemcpyHostToDevice, st));
            }
            size_t r0 = 0, b0 = 0;
            for (const WavePlan &w : plans) {
                BatchLaunchArgs la;
                la.ranges = cb.d_ranges + r0;
                la.nranges = (int)w.ranges.size();
                la.blk_first = cb.d_blk + b0;
                la.nwaves = (int64_t)w.nwaves;
                la.mats = cb.d_mats;
                la.vals = vals;
                la.tops = tops;
                la.partials = parts;
                SRV_HIP(launch_batch_ranges(w.ng, w.zero_skip, w.exact, la, 256, nullptr, 0, st));
                r0 += w.ranges.size();
                b0 += w.blk_first.size();
            }
            if (nf) {
                SRV_HIP(launch_batch_finish(cb.d_fin, (int)nf, parts, cb.d_out, st));
                SRV_HIP(hipMemcpyAsync(cb.h_out, cb.d_out, kPartStride * nf * sizeof(double), hipMemcpyDeviceToHost,
                                       st));
            }
        }
        SRV_HIP(hipEventRecord(cb.done, st));
        cb.used = true;
    }
    slot.busy = true;
    {
        std::lock_guard<std::mutex> g(mu);  // read by perm_server_get_stats
        ++n_rounds;
    }
    return true;
}

bool perm_server::complete(Slot &slot, std::string *err) {
    for (int c = 0; c < kBatchStreams; ++c)
        if (slot.cls[c].used) SRV_HIP(hipEventSynchronize(slot.cls[c].done));
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(mu);
    bool any = false;
    for (int c = 0; c < kBatchStreams; ++c) {
        ClassBuf &cb = slot.cls[c];
        if (!cb.used) continue;
        for (size_t i = 0; i < cb.finishing.size(); ++i) {
            Request *r = cb.finishing[i];
            const double *o = cb.h_out + kPartStride * i;
            if (r->pm.exact) {
                // exact mode: recover the integer; without a certificate the
                // request runs again with the next prime (same arena data)
                ExactSums &es = r->es;
                es.hi = o[0];
                es.lo = o[1];
                es.abs_sum = o[3];
                es.chunk_log2 = r->pm.kappa;
                es.resid[r->pass] = o[2];
                es.passes = r->pass + 1;
                const ExactOutcome eo = exact_recover(r->pm.n, es);
                r->result = eo.value;
                r->exact_state = eo.certified ? 1 : 0;
                const bool forced = es.passes < std::min(opts.exact_passes, kExactMaxPasses);
                if ((!eo.certified && eo.more) || forced) {
                    ++r->pass;
                    r->next_item = 0;
                    ++n_extra_passes;
                    continue;
                }
            } else {
                r->result = (o[0] + o[1]) * ((r->pm.n % 2 == 1) ? 2.0 : -2.0);  // 4 (n mod 2) - 2
            }
            if (r->exact_state == 1) ++n_exact_certified;
            if (r->exact_state == 0) ++n_exact_uncertified;
            r->state = State::Done;
            r->t_done = now;
            alloc.release(r->arena_off, r->bytes);
            active.erase(std::find(active.begin(), active.end(), r));
            ++n_completed;
            any = true;
        }
        cb.finishing.clear();
        cb.used = false;
    }
    slot.busy = false;
    if (!slots[0].busy && !slots[1].busy)
        busy_ms += std::chrono::duration<double, std::milli>(now - busy_since).count();
    if (any) cv_done.notify_all();
    return true;
}

#undef SRV_HIP

void perm_server::run() {
    std::string err;
    bool ok = hipSetDevice(device) == hipSuccess;
    if (!ok) err = "hipSetDevice failed in the server thread";
    int cur = 0;  // the slot the next round goes to; when both are busy it holds the older round
    while (ok) {
        std::vector<Request *> newly;
        bool work;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || !pending.empty() || dispatchable() || slots[0].busy || slots[1].busy;
            });
            if (stop && pending.empty() && active.empty() && !slots[0].busy && !slots[1].busy) break;
            admit(newly);
            for (Request *r : newly) {
                r->state = State::Active;
                active.push_back(r);
            }
            work = dispatchable();
        }
        const bool idle = !slots[0].busy && !slots[1].busy;
        if (work) {
            if (slots[cur].busy) ok = complete(slots[cur], &err);
            if (ok) {
                ok = issue(slots[cur], newly, &err);
                cur ^= 1;
            }
        } else if (!idle) {
            Slot &old = slots[cur].busy ? slots[cur] : slots[cur ^ 1];
            ok = complete(old, &err);
        }
    }
    // on a device error every unfinished request fails
    std::lock_guard<std::mutex> g(mu);
    if (!ok) {
        fatal = err;
        for (auto &kv : tickets)
            if (kv.second->state != State::Done) {
                kv.second->state = State::Done;
                kv.second->status = PERM_EDEVICE;
            }
        pending.clear();
        active.clear();
    }
    cv_done.notify_all();
}

namespace {
perm_status sfail(perm_status s, const std::string &m) {
    set_last_error(m);
    return s;
}
}  // namespace

extern "C" {

perm_server *perm_server_create(const perm_opts *opts, size_t device_mem_budget, int32_t max_inflight,
                                double round_steps) {
    std::unique_ptr<perm_server> s(new perm_server);
    memset(&s->opts, 0, sizeof s->opts);
    if (opts) s->opts = *opts;
    s->bo.zero_skip = s->opts.zero_skip;
    s->bo.kappa_shift = s->opts.batch_kappa_shift + kServerChunkShift;
    s->bo.exact = s->opts.exact;
    if (s->opts.exact < -1 || s->opts.exact > 1 || s->opts.exact_passes < 0 || s->opts.exact_passes > 3) {
        set_last_error("exact must be -1, 0 or 1 and exact_passes 0..3");
        return nullptr;
    }
    s->budget = device_mem_budget ? device_mem_budget : ((size_t)1 << 30);
    s->max_inflight = max_inflight > 0 ? max_inflight : 4096;
    if (!(round_steps >= 0.0)) {
        set_last_error("round_steps must be >= 0");
        return nullptr;
    }
    // default: about 20 ms of device work per round (measured best of 2e9 ..
    // 6.4e10 on the serving mix at 200, 300 and 400 requests/s)
    s->round_steps = round_steps > 0.0 ? round_steps : 1.6e10;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        set_last_error("no HIP device available");
        return nullptr;
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        set_last_error("hipGetDevice failed");
        return nullptr;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->device) != hipSuccess || std::string(prop.gcnArchName).compare(0, 6, "gfx950")) {
        set_last_error("device is not gfx950 (MI355X)");
        return nullptr;
    }
    for (int c = 0; c < kBatchStreams; ++c)
        if (hipStreamCreateWithFlags(&s->streams[c], hipStreamNonBlocking) != hipSuccess) {
            for (int d = 0; d < c; ++d) (void)hipStreamDestroy(s->streams[d]);
            set_last_error("stream creation failed");
            return nullptr;
        }
    if (hipMalloc(&s->arena, s->budget) != hipSuccess) {
        for (int c = 0; c < kBatchStreams; ++c) (void)hipStreamDestroy(s->streams[c]);
        set_last_error("device arena allocation of " + std::to_string(s->budget) + " bytes failed");
        return nullptr;
    }
    s->alloc.reset(s->budget);
    perm_server *raw = s.get();
    raw->worker = std::thread([raw] { raw->run(); });
    return s.release();
}

perm_status perm_submit(perm_server *s, const perm_csc *a, uint64_t *ticket) {
    if (!s || !ticket) return sfail(PERM_EINVAL, "null server or ticket");
    std::unique_ptr<Request> r(new Request);
    r->t_submit = Clock::now();
    std::string err;
    perm_status st = prepare_batch_matrix(a, s->bo, &r->pm, &err);
    if (st != PERM_OK) return sfail(st, err);
    if (!r->pm.singular) {
        r->items_total = (r->pm.nchunks + 63) / 64;
        r->bytes = request_bytes(r->pm, r->items_total, &r->vals_bytes);
        if (r->bytes > s->budget)
            return sfail(PERM_ETOOBIG, "request needs " + std::to_string(r->bytes) + " bytes, budget is " +
                                           std::to_string(s->budget));
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->fatal.empty()) return sfail(PERM_EDEVICE, s->fatal);
    if (s->stop) return sfail(PERM_EINVAL, "server is shutting down");
    if ((int)s->tickets.size() >= s->max_inflight)
        return sfail(PERM_EAGAIN, "max_inflight requests outstanding");
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    Request *raw = r.get();
    s->tickets.emplace(raw->ticket, std::move(r));
    ++s->n_submitted;
    if (raw->pm.singular) {
        raw->state = State::Done;  // no perfect matching: exactly 0, no device work
        raw->result = 0.0;
        raw->t_done = raw->t_submit;
        ++s->n_completed;
        s->cv_done.notify_all();
    } else {
        s->pending.push_back(raw);
        s->cv_work.notify_one();
    }
    return PERM_OK;
}

perm_status perm_poll(perm_server *s, uint64_t ticket, double *out) {
    if (!s || !out) return sfail(PERM_EINVAL, "null server or output");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return sfail(PERM_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    if (r->state != State::Done) return PERM_ENOTREADY;
    const perm_status st = r->status;
    *out = r->result;
    s->tickets.erase(it);
    if (st != PERM_OK) return sfail(st, s->fatal.empty() ? "request failed" : s->fatal);
    return PERM_OK;
}

perm_status perm_wait(perm_server *s, uint64_t ticket, double *out) {
    if (!s || !out) return sfail(PERM_EINVAL, "null server or output");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->tickets.find(ticket) == s->tickets.end()) return sfail(PERM_EINVAL, "unknown ticket");
    // The ticket is looked up again on every wake-up: while the lock is
    // released, a submit may rehash the map and another caller may collect
    // the request (then this wait reports an unknown ticket).
    Request *r = nullptr;
    s->cv_done.wait(lk, [&] {
        auto it = s->tickets.find(ticket);
        r = it == s->tickets.end() ? nullptr : it->second.get();
        return r == nullptr || r->state == State::Done;
    });
    if (!r) return sfail(PERM_EINVAL, "ticket collected by another caller");
    const perm_status st = r->status;
    *out = r->result;
    s->tickets.erase(ticket);
    if (st != PERM_OK) return sfail(st, s->fatal.empty() ? "request failed" : s->fatal);
    return PERM_OK;
}

perm_status perm_server_get_stats(perm_server *s, perm_server_stats *st) {
    if (!s || !st) return sfail(PERM_EINVAL, "null server or stats");
    std::lock_guard<std::mutex> g(s->mu);
    memset(st, 0, sizeof *st);
    st->submitted = s->n_submitted;
    st->completed = s->n_completed;
    st->rounds = s->n_rounds;
    st->pending = s->pending.size();
    st->active = s->active.size();
    st->arena_bytes = s->budget;
    st->arena_used = s->alloc.used();
    st->arena_peak = s->peak_bytes;
    st->busy_ms = s->busy_ms;
    st->exact_certified = s->n_exact_certified;
    st->exact_uncertified = s->n_exact_uncertified;
    st->extra_passes = s->n_extra_passes;
    return PERM_OK;
}

void perm_server_destroy(perm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (int c = 0; c < kBatchStreams; ++c) (void)hipStreamSynchronize(s->streams[c]);
    if (s->arena) (void)hipFree(s->arena);
    for (Slot &sl : s->slots)
        for (ClassBuf &cb : sl.cls) cb.release();
    for (int c = 0; c < kBatchStreams; ++c) (void)hipStreamDestroy(s->streams[c]);
    delete s;
}

}  // extern "C"
