// Continuous-batching request server over the persistent batched filter.
//
// Online interface (dctf_server_submit / dctf_server_poll):
//   - a submitted request is validated and queued at once (its mask is
//     copied, so the caller may free it);
//   - each poll reaps the batches that have finished, then admits queued
//     requests in submission order while their output fits in the server's
//     device arena (first-fit allocation; the arena size is the HBM budget)
//     and a launch slot is free; a request whose output alone exceeds the
//     arena completes with DCTF_EBUSY;
//   - the requests admitted together form one batch: their operators come
//     from a device-resident cache keyed by (mask bytes, kh, kw, N, border)
//     (LRU eviction of entries no batch in flight uses), the work table is
//     copied from pinned host memory on the slot's stream and one persistent
//     filter launch covers all of them;
//   - up to max_inflight batches run at once, one HIP stream each, so work of
//     requests that arrive while others are on the GPU overlaps on the device;
//   - completion is observed by polling each slot's event; the slot's arena
//     ranges and cache references are then released and its requests are
//     handed back by the poll.
// dctf_server_run replays a list of requests with known arrival times in real
// time on top of the same two calls.
// Each request's blocks go through the same per-block arithmetic as a
// single-operator call, so its result does not depend on the mix it ran in.
#include "dctf_internal.h"

#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <list>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

namespace dctf {
namespace {

double now_s()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
  public:
    void reset(size_t size)
    {
        free_.clear();
        if (size)
            free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t n, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest)
                    free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

  private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct CacheEntry {
    dctf_operator op = nullptr;
    int refs = 0;
    std::list<std::string>::iterator lru;
};

// A submitted request waiting for admission: the caller's record and the
// cache key (header + a copy of the mask).
struct Queued {
    dctf_request *req;
    std::string key;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *table_dev = nullptr;
    char *table_host = nullptr;
    size_t table_cap = 0;
    bool busy = false;
    std::vector<dctf_request *> reqs;
    std::vector<size_t> offs, sizes;
    std::vector<CacheEntry *> entries;
};

}  // namespace
}  // namespace dctf

using namespace dctf;

struct dctf_server_s {
    dctf_server_config cfg;
    void *arena_dev = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::unordered_map<std::string, CacheEntry> cache;
    std::list<std::string> lru;   // front = most recently used
    dctf_server_stats stats;
    double t0 = 0.0;              // origin of the server clock (absolute seconds)
    std::deque<Queued> queue;     // submitted, not yet admitted
    std::deque<dctf_request *> finished;   // completed, not yet returned by a poll
    int64_t outstanding = 0;      // submitted and not yet returned by a poll
    std::vector<dctf_job> jobs;   // scratch of the admission step
    std::vector<dctf_job> side;   // its jobs of N = 2, 4, 32 (launched one by one)
    std::vector<char> table;
    std::vector<dctf_operator> ops;
};

namespace {

// Checks one request: block size, mask shape and values (finite), border,
// pointers and alignment.  arrival_s is not read here.
bool request_valid(const dctf_request &r)
{
    if (r.B < 1 || (r.N != 2 && r.N != 4 && r.N != 8 && r.N != 16 && r.N != 32) || r.mask_host == nullptr ||
        r.kh < 1 || r.kw < 1 ||
        r.kh > 2 * r.N + 1 || r.kw > 2 * r.N + 1 ||
        (r.border != DCTF_BORDER_ZERO && r.border != DCTF_BORDER_REPLICATE) || r.in_dev == nullptr ||
        ((uintptr_t)r.in_dev & 15) || ((uintptr_t)r.out_dev & 15))
        return false;
    for (int i = 0; i < r.kh * r.kw; ++i)
        if (!std::isfinite(r.mask_host[i]))
            return false;
    return true;
}

std::string cache_key(const dctf_request &r)
{
    std::string k;
    const int hdr[4] = {r.kh, r.kw, r.N, r.border};
    k.append(reinterpret_cast<const char *>(hdr), sizeof(hdr));
    k.append(reinterpret_cast<const char *>(r.mask_host), sizeof(double) * r.kh * r.kw);
    return k;
}

// Operator of a cache key (built on `stream` on a miss); takes a reference.
dctf_status cache_get(dctf_server s, const std::string &key, hipStream_t stream, CacheEntry **out)
{
    auto it = s->cache.find(key);
    if (it != s->cache.end()) {
        s->lru.erase(it->second.lru);
        s->lru.push_front(key);
        it->second.lru = s->lru.begin();
        ++it->second.refs;
        ++s->stats.cache_hits;
        *out = &it->second;
        return DCTF_OK;
    }
    // Evict least recently used entries no batch in flight uses.
    for (auto l = s->lru.rbegin(); (int)s->cache.size() >= s->cfg.max_cached_ops && l != s->lru.rend();) {
        auto victim = s->cache.find(*l);
        if (victim->second.refs == 0) {
            dctf_operator_destroy(victim->second.op);
            auto fwd = std::next(l).base();
            l = std::list<std::string>::reverse_iterator(s->lru.erase(fwd));
            s->cache.erase(victim);
            ++s->stats.cache_evictions;
        } else {
            ++l;
        }
    }
    int hdr[4];
    memcpy(hdr, key.data(), sizeof(hdr));
    std::vector<double> m((size_t)hdr[0] * hdr[1]);   // aligned copy of the key's mask bytes
    memcpy(m.data(), key.data() + sizeof(hdr), sizeof(double) * m.size());
    dctf_operator op = nullptr;
    dctf_status st = dctf_build_operator(m.data(), hdr[0], hdr[1], hdr[2], hdr[3], stream, &op);
    if (st != DCTF_OK)
        return st;
    ++s->stats.cache_misses;
    CacheEntry &e = s->cache[key];
    e.op = op;
    e.refs = 1;
    s->lru.push_front(key);
    e.lru = s->lru.begin();
    *out = &e;
    return DCTF_OK;
}

double clock_s(dctf_server s) { return now_s() - s->t0; }

// A request leaves the server's hands: it waits in `finished` for a poll.
void complete(dctf_server s, dctf_request *r, int status, double t)
{
    r->status = status;
    r->done_s = t;
    if (r->admit_s < 0.0)
        r->admit_s = t;
    if (status == DCTF_EBUSY)
        ++s->stats.rejected;
    else if (status != DCTF_OK)
        ++s->stats.failed;
    s->finished.push_back(r);
}

void release_slot(dctf_server s, Slot &sl, int status, double t)
{
    for (dctf_request *r : sl.reqs)
        complete(s, r, status, t);
    for (size_t i = 0; i < sl.offs.size(); ++i)
        s->arena.release(sl.offs[i], sl.sizes[i]);
    for (CacheEntry *e : sl.entries)
        --e->refs;
    sl.reqs.clear();
    sl.offs.clear();
    sl.sizes.clear();
    sl.entries.clear();
    sl.busy = false;
}

// Reaps finished batches.  A device error fails the slot's requests and is
// returned (the other slots are still reaped).
dctf_status reap(dctf_server s)
{
    dctf_status err = DCTF_OK;
    for (Slot &sl : s->slots) {
        if (!sl.busy)
            continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) {
            release_slot(s, sl, DCTF_OK, clock_s(s));
        } else if (q != hipErrorNotReady) {
            release_slot(s, sl, DCTF_EHIP, clock_s(s));
            err = DCTF_EHIP;
        }
    }
    return err;
}

// Fills free slots from the queue and launches them.
dctf_status admit(dctf_server s)
{
    dctf_status err = DCTF_OK;
    for (Slot &sl : s->slots) {
        if (sl.busy || s->queue.empty())
            continue;
        const double t = clock_s(s);
        s->jobs.clear();
        while (!s->queue.empty() && (int)sl.reqs.size() < s->cfg.max_batch_jobs) {
            dctf_request *r = s->queue.front().req;
            const size_t bytes = align256((size_t)r->B * r->N * r->N * sizeof(float));
            if (bytes > (size_t)s->cfg.arena_bytes) {
                s->queue.pop_front();
                complete(s, r, DCTF_EBUSY, t);
                continue;
            }
            size_t off;
            if (!s->arena.alloc(bytes, &off))
                break;   // admit in submission order: wait for memory
            CacheEntry *e = nullptr;
            const dctf_status st = cache_get(s, s->queue.front().key, sl.stream, &e);
            s->queue.pop_front();
            if (st != DCTF_OK) {   // this request cannot run (e.g. no memory for its operator)
                s->arena.release(off, bytes);
                complete(s, r, st, t);
                continue;
            }
            r->admit_s = t;
            sl.reqs.push_back(r);
            sl.offs.push_back(off);
            sl.sizes.push_back(bytes);
            sl.entries.push_back(e);
            s->jobs.push_back({e->op, r->in_dev, reinterpret_cast<float *>(static_cast<char *>(s->arena_dev) + off),
                               r->B});
        }
        if (sl.reqs.empty()) {
            if (s->queue.empty())
                continue;   // every candidate completed without running
            break;          // the head request waits for arena space
        }
        BatchArgs a;
        dctf_status st = plan_batch(s->jobs.data(), (int)s->jobs.size(), s->cfg.prec, batch_config(s->cfg.prec),
                                    s->table, a, s->ops, &s->side);
        if (st == DCTF_OK && s->table.size() > sl.table_cap)
            st = DCTF_EINVAL;
        hipError_t e = hipSuccess;
        if (st == DCTF_OK) {
            memcpy(sl.table_host, s->table.data(), s->table.size());
            e = hipMemcpyAsync(sl.table_dev, sl.table_host, s->table.size(), hipMemcpyHostToDevice, sl.stream);
            rebase_batch(a, sl.table_dev);
            if (e == hipSuccess)
                e = launch_batch(a, sl.stream);
            if (e == hipSuccess && launch_side_jobs(s->side, s->cfg.prec, sl.stream) != DCTF_OK)
                e = hipErrorLaunchFailure;
            for (size_t k = 0; k < sl.reqs.size() && e == hipSuccess; ++k) {
                const dctf_request &r = *sl.reqs[k];
                if (r.out_dev)
                    e = hipMemcpyAsync(r.out_dev, s->jobs[k].out, (size_t)r.B * r.N * r.N * sizeof(float),
                                       hipMemcpyDeviceToDevice, sl.stream);
            }
            if (e == hipSuccess)
                e = hipEventRecord(sl.done, sl.stream);
        }
        if (st != DCTF_OK || e != hipSuccess) {
            // Nothing of this batch is known to have run: wait for whatever
            // was enqueued, then fail its requests.
            (void)hipStreamSynchronize(sl.stream);
            const dctf_status fail = st != DCTF_OK ? st : DCTF_EHIP;
            release_slot(s, sl, fail, clock_s(s));
            if (fail == DCTF_EHIP)
                err = DCTF_EHIP;
            continue;
        }
        const double tl = clock_s(s);
        for (dctf_request *r : sl.reqs) {
            r->launch_s = tl;
            r->batch = (int)s->stats.batches;
        }
        ++s->stats.batches;
        sl.busy = true;
        int inflight = 0;
        for (const Slot &o : s->slots)
            inflight += o.busy ? 1 : 0;
        s->stats.peak_inflight_batches = std::max<int64_t>(s->stats.peak_inflight_batches, inflight);
        s->stats.peak_arena_bytes = std::max<int64_t>(s->stats.peak_arena_bytes, (int64_t)s->arena.used());
    }
    return err;
}

// One round of progress: reap, then admit.
dctf_status step(dctf_server s)
{
    const dctf_status e1 = reap(s);
    const dctf_status e2 = admit(s);
    return e1 != DCTF_OK ? e1 : e2;
}

int take_finished(dctf_server s, dctf_request **done, int max_done)
{
    int n = 0;
    while (n < max_done && !s->finished.empty()) {
        done[n++] = s->finished.front();
        s->finished.pop_front();
    }
    s->outstanding -= n;
    return n;
}

}  // namespace

extern "C" dctf_status dctf_server_create(const dctf_server_config *cfg, dctf_server *out)
{
    if (cfg == nullptr || out == nullptr)
        return DCTF_EINVAL;
    if (cfg->arena_bytes < 256 || cfg->max_inflight < 1 || cfg->max_inflight > 16 || cfg->max_batch_jobs < 1 ||
        cfg->max_batch_jobs > 4096 || cfg->max_cached_ops < 1 ||
        (cfg->prec != DCTF_PREC_FP32 && cfg->prec != DCTF_PREC_SPLIT_BF16))
        return DCTF_EINVAL;
    dctf_server s = new (std::nothrow) dctf_server_s();
    if (!s)
        return DCTF_ENOMEM;
    s->cfg = *cfg;
    memset(&s->stats, 0, sizeof(s->stats));
    s->t0 = now_s();
    hipError_t e = hipMalloc(&s->arena_dev, (size_t)cfg->arena_bytes);
    if (e != hipSuccess) {
        delete s;
        return e == hipErrorOutOfMemory ? DCTF_ENOMEM : DCTF_EHIP;
    }
    s->arena.reset((size_t)cfg->arena_bytes);
    s->slots.resize(cfg->max_inflight);
    // Work table of one batch: jobs, fronts and operators (bounded by the jobs).
    const size_t cap = 1024 + (size_t)cfg->max_batch_jobs *
                                  (sizeof(JobDesc) + 2 * sizeof(SegDesc) + sizeof(OpDesc));
    for (Slot &sl : s->slots) {
        sl.table_cap = cap;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&sl.table_dev, cap) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.table_host), cap, hipHostMallocDefault) != hipSuccess) {
            dctf_server_destroy(s);
            return DCTF_EHIP;
        }
    }
    *out = s;
    return DCTF_OK;
}

extern "C" void dctf_server_destroy(dctf_server s)
{
    if (s == nullptr)
        return;
    for (Slot &sl : s->slots) {
        if (sl.stream)
            (void)hipStreamSynchronize(sl.stream);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
        if (sl.table_dev)
            (void)hipFree(sl.table_dev);
        if (sl.table_host)
            (void)hipHostFree(sl.table_host);
        if (sl.stream)
            (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : s->cache)
        dctf_operator_destroy(kv.second.op);
    if (s->arena_dev)
        (void)hipFree(s->arena_dev);
    delete s;
}

extern "C" dctf_status dctf_server_stats_get(dctf_server s, dctf_server_stats *out)
{
    if (s == nullptr || out == nullptr)
        return DCTF_EINVAL;
    *out = s->stats;
    return DCTF_OK;
}

extern "C" double dctf_server_clock(dctf_server s) { return s == nullptr ? -1.0 : clock_s(s); }

extern "C" dctf_status dctf_server_submit(dctf_server s, dctf_request *req)
{
    if (s == nullptr || req == nullptr || !request_valid(*req))
        return DCTF_EINVAL;
    req->admit_s = req->launch_s = req->done_s = -1.0;
    req->status = DCTF_EBUSY;
    req->batch = -1;
    try {
        s->queue.push_back({req, cache_key(*req)});
    } catch (...) {
        return DCTF_ENOMEM;
    }
    ++s->outstanding;
    return DCTF_OK;
}

extern "C" dctf_status dctf_server_poll(dctf_server s, double wait_s, dctf_request **done, int max_done,
                                        int *n_done)
{
    if (s == nullptr || n_done == nullptr || max_done < 0 || (max_done > 0 && done == nullptr) ||
        !(wait_s >= 0.0))
        return DCTF_EINVAL;
    *n_done = 0;
    const double until = clock_s(s) + wait_s;
    dctf_status err = step(s);
    // Wait (polling) until something completes, the time is up, or the
    // server holds nothing that could complete.
    while (err == DCTF_OK && s->finished.empty() && max_done > 0 && clock_s(s) < until &&
           (s->outstanding > 0))
        err = step(s);
    *n_done = take_finished(s, done, max_done);
    return err;
}

extern "C" dctf_status dctf_server_run(dctf_server s, dctf_request *reqs, int n)
{
    if (s == nullptr || n < 0 || (n > 0 && reqs == nullptr))
        return DCTF_EINVAL;
    for (int i = 0; i < n; ++i)
        if ((i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s) || !(reqs[i].arrival_s >= 0.0) ||
            !request_valid(reqs[i]))
            return DCTF_EINVAL;
    if (s->outstanding > 0)
        return DCTF_EBUSY;   // requests of the online interface are still in the server
    const double start = now_s();
    s->t0 = start;
    int next = 0, got = 0;
    dctf_status err = DCTF_OK;
    dctf_request *done[64];
    while (got < n) {
        const double t = clock_s(s);
        while (next < n && reqs[next].arrival_s <= t && err == DCTF_OK) {
            const dctf_status st = dctf_server_submit(s, &reqs[next]);
            if (st != DCTF_OK)
                err = st;
            else
                ++next;
        }
        if (err != DCTF_OK && next < n) {
            // A device error (or no host memory): the rest never runs.
            for (; next < n; ++next) {
                reqs[next].admit_s = reqs[next].launch_s = -1.0;
                reqs[next].done_s = clock_s(s);
                reqs[next].status = err;
                reqs[next].batch = -1;
                ++got;
            }
        }
        int k = 0;
        const dctf_status st = dctf_server_poll(s, 0.0, done, 64, &k);
        got += k;
        if (st != DCTF_OK && err == DCTF_OK)
            err = st;
        if (err != DCTF_OK && s->outstanding == 0)
            break;
    }
    s->stats.busy_s += now_s() - start;
    return err;
}
