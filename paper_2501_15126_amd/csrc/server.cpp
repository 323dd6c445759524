// server.cpp -- the submit/poll permanent server (continuous batching).
//
// Requests are validated and prepared for the precompiled batch kernels on
// the submitting thread.  A scheduler thread admits them in arrival order as
// device memory (one arena of `device_mem_budget` bytes) frees up, keeps each
// admitted request's matrix data and partial sums resident in the arena, and
// runs rounds: every round takes a share of 64-chunk work items from every
// active request (so a request that arrives while others run joins the next
// round instead of waiting for them to finish), launches the batch kernels on
// all of them together, and finishes the requests whose last items ran.  A
// request's result depends only on its own items and their fixed-order sum,
// so it is bitwise the same alone and in any mix.
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
#include "perm.h"
#include "perm_internal.h"

using namespace permx;

namespace {

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
};

size_t request_bytes(const PreparedMatrix &pm, uint64_t items, size_t *vals_bytes) {
    *vals_bytes = (pm.vals.size() * sizeof(double) + kAlign - 1) / kAlign * kAlign;
    const size_t tops = (pm.tops.size() * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign;
    const size_t parts = (items * 2 * sizeof(double) + kAlign - 1) / kAlign * kAlign;
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
    uint64_t n_submitted = 0, n_completed = 0, n_rounds = 0;
    size_t peak_bytes = 0;
    double busy_ms = 0.0;

    // device side (worker thread only, after creation)
    int device = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;
    Arena alloc;
    BatchMat *d_mats = nullptr;
    BatchItem *d_items = nullptr;
    FinishDesc *d_fin = nullptr;
    double *d_out = nullptr;
    size_t cap_mats = 0, cap_items = 0, cap_fin = 0, cap_out = 0;
    char *h_stage = nullptr;
    size_t cap_stage = 0;
    double *h_out = nullptr;
    size_t cap_hout = 0;

    void run();
    bool admit(std::vector<Request *> &newly, std::string *err);
    bool round(std::string *err);
};

bool perm_server::admit(std::vector<Request *> &newly, std::string *err) {
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
    (void)err;
    return true;
}

bool perm_server::round(std::string *err) {
    // ---- pick work items: an equal share per active request, oldest first ----
    std::vector<Request *> act = active;
    const double share_steps = round_steps / std::max<size_t>(1, act.size());
    std::vector<BatchMat> mats;
    std::vector<BatchItem> items;
    std::vector<FinishDesc> fin;
    std::vector<Request *> finishing;
    for (Request *r : act) {
        const PreparedMatrix &pm = r->pm;
        const double item_steps = std::ldexp(64.0, pm.kappa);
        const uint64_t share = std::max<uint64_t>(1, (uint64_t)(share_steps / item_steps));
        const uint64_t take = std::min<uint64_t>(share, r->items_total - r->next_item);
        if (take == 0) continue;
        BatchMat d;
        d.n = pm.n;
        d.ng = pm.ng;
        d.kappa = pm.kappa;
        d.zero_skip = pm.zero_skip ? 1 : 0;
        d.chunk_top = pm.chunk_top;
        d.pad = 0;
        d.nchunks = pm.nchunks;
        d.col_off = r->arena_off / sizeof(double);
        d.base_off = d.col_off + pm.base_index;
        d.top_off = (r->arena_off + r->vals_bytes) / sizeof(int32_t);
        const int mi = (int)mats.size();
        mats.push_back(d);
        const size_t tops_bytes = (pm.tops.size() * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign;
        const uint64_t part0 = (r->arena_off + r->vals_bytes + tops_bytes) / (2 * sizeof(double));
        for (uint64_t k = 0; k < take; ++k) {
            const uint64_t it = r->next_item + k;
            items.push_back(BatchItem{mi, 0, it * 64, part0 + it});
        }
        r->next_item += take;
        if (r->next_item == r->items_total) {
            fin.push_back(FinishDesc{part0, r->items_total, pm.n, 0});
            finishing.push_back(r);
        }
    }
    // items grouped by kernel instance (ng), stable within a group
    std::stable_sort(items.begin(), items.end(),
                     [&](const BatchItem &a, const BatchItem &b) { return mats[a.mat].ng < mats[b.mat].ng; });
    const size_t nm = mats.size(), ni = items.size(), nf = fin.size();
    if (!grow_dev(&d_mats, &cap_mats, std::max<size_t>(nm, 1)) ||
        !grow_dev(&d_items, &cap_items, std::max<size_t>(ni, 1)) ||
        !grow_dev(&d_fin, &cap_fin, std::max<size_t>(nf, 1)) || !grow_dev(&d_out, &cap_out, std::max<size_t>(nf, 1))) {
        *err = "device allocation for a round failed";
        return false;
    }
    const size_t bytes = nm * sizeof(BatchMat) + ni * sizeof(BatchItem) + nf * sizeof(FinishDesc) + 64;
    if (!grow_host(&h_stage, &cap_stage, bytes) || !grow_host(&h_out, &cap_hout, std::max<size_t>(nf, 1))) {
        *err = "pinned host allocation for a round failed";
        return false;
    }
    char *p = h_stage;
    memcpy(p, mats.data(), nm * sizeof(BatchMat));
    char *s_items = p + (nm * sizeof(BatchMat) + 15) / 16 * 16;
    memcpy(s_items, items.data(), ni * sizeof(BatchItem));
    char *s_fin = s_items + (ni * sizeof(BatchItem) + 15) / 16 * 16;
    memcpy(s_fin, fin.data(), nf * sizeof(FinishDesc));
#define SRV_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            *err = std::string(#call) + ": " + hipGetErrorString(e_);            \
            return false;                                                        \
        }                                                                        \
    } while (0)
    SRV_HIP(hipMemcpyAsync(d_mats, p, nm * sizeof(BatchMat), hipMemcpyHostToDevice, stream));
    SRV_HIP(hipMemcpyAsync(d_items, s_items, ni * sizeof(BatchItem), hipMemcpyHostToDevice, stream));
    if (nf) SRV_HIP(hipMemcpyAsync(d_fin, s_fin, nf * sizeof(FinishDesc), hipMemcpyHostToDevice, stream));
    const double *vals = reinterpret_cast<const double *>(arena);
    const int32_t *tops = reinterpret_cast<const int32_t *>(arena);
    double *parts = reinterpret_cast<double *>(arena);
    size_t i0 = 0;
    while (i0 < ni) {
        const int ng = mats[items[i0].mat].ng;
        size_t i1 = i0;
        while (i1 < ni && mats[items[i1].mat].ng == ng) ++i1;
        SRV_HIP(launch_batch_items(ng, d_items + i0, (int64_t)(i1 - i0), d_mats, vals, tops, parts, stream));
        i0 = i1;
    }
    if (nf) {
        SRV_HIP(launch_batch_finish(d_fin, (int)nf, parts, d_out, stream));
        SRV_HIP(hipMemcpyAsync(h_out, d_out, nf * sizeof(double), hipMemcpyDeviceToHost, stream));
    }
    SRV_HIP(hipStreamSynchronize(stream));
#undef SRV_HIP
    const auto now = Clock::now();
    std::lock_guard<std::mutex> g(mu);
    for (size_t i = 0; i < nf; ++i) {
        Request *r = finishing[i];
        r->result = h_out[i];
        r->state = State::Done;
        r->t_done = now;
        alloc.release(r->arena_off, r->bytes);
        active.erase(std::find(active.begin(), active.end(), r));
        ++n_completed;
    }
    ++n_rounds;
    if (nf) cv_done.notify_all();
    return true;
}

void perm_server::run() {
    std::string err;
    if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> g(mu);
        fatal = "hipSetDevice failed in the server thread";
    }
    for (;;) {
        std::vector<Request *> newly;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty() || !fatal.empty(); });
            if (!fatal.empty() || (stop && pending.empty() && active.empty())) break;
            admit(newly, &err);
        }
        // upload the newly admitted requests' data into the arena
        bool ok = true;
        for (Request *r : newly) {
            const PreparedMatrix &pm = r->pm;
            if (hipMemcpyAsync(arena + r->arena_off, pm.vals.data(), pm.vals.size() * sizeof(double),
                               hipMemcpyHostToDevice, stream) != hipSuccess ||
                hipMemcpyAsync(arena + r->arena_off + r->vals_bytes, pm.tops.data(), pm.tops.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, stream) != hipSuccess) {
                ok = false;
                err = "upload of an admitted request failed";
            }
        }
        {
            std::lock_guard<std::mutex> g(mu);
            for (Request *r : newly) {
                r->state = State::Active;
                active.push_back(r);
            }
        }
        const auto t0 = Clock::now();
        if (ok) ok = round(&err);
        busy_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
        if (!ok) {
            std::lock_guard<std::mutex> g(mu);
            fatal = err;
            break;
        }
    }
    // on a device error every unfinished request fails
    std::lock_guard<std::mutex> g(mu);
    if (!fatal.empty()) {
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

perm_server *perm_server_create(const perm_opts *opts, size_t device_mem_budget, int32_t max_inflight) {
    std::unique_ptr<perm_server> s(new perm_server);
    memset(&s->opts, 0, sizeof s->opts);
    if (opts) s->opts = *opts;
    s->bo.zero_skip = s->opts.zero_skip;
    s->bo.kappa_shift = s->opts.batch_kappa_shift;
    s->budget = device_mem_budget ? device_mem_budget : ((size_t)1 << 30);
    s->max_inflight = max_inflight > 0 ? max_inflight : 4096;
    s->round_steps = 4.0e9;  // a few milliseconds of device work per round
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
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        set_last_error("stream creation failed");
        return nullptr;
    }
    if (hipMalloc(&s->arena, s->budget) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
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
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return sfail(PERM_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    s->cv_done.wait(lk, [&] { return r->state == State::Done; });
    const perm_status st = r->status;
    *out = r->result;
    s->tickets.erase(it);
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
    (void)hipStreamSynchronize(s->stream);
    if (s->arena) (void)hipFree(s->arena);
    if (s->d_mats) (void)hipFree(s->d_mats);
    if (s->d_items) (void)hipFree(s->d_items);
    if (s->d_fin) (void)hipFree(s->d_fin);
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->h_stage) (void)hipHostFree(s->h_stage);
    if (s->h_out) (void)hipHostFree(s->h_out);
    (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
