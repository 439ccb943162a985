// Continuous-batching request server over the persistent batched filter.
//
// dctf_server_run replays a list of requests in real time on one host thread:
//   - a request becomes pending at its arrival time;
//   - pending requests are admitted in arrival order while their output fits
//     in the server's device arena (first-fit allocation; the arena size is
//     the HBM budget) and a launch slot is free; a request whose output alone
//     exceeds the arena is rejected with DCTF_EBUSY;
//   - the admitted requests of one slot form one batch: their operators come
//     from a device-resident cache keyed by (mask bytes, kh, kw, N, border)
//     (LRU eviction of entries no batch in flight uses), the work table is
//     copied from pinned host memory on the slot's stream and one persistent
//     filter launch covers all of them;
//   - up to max_inflight batches run at once, one HIP stream each, so work of
//     requests that arrive while others are on the GPU overlaps on the device;
//   - completion is observed by polling each slot's event; the slot's arena
//     ranges and cache references are then released.
// Each request's blocks go through the same per-block arithmetic as a
// single-operator call, so its result does not depend on the mix it ran in.
#include "dctf_internal.h"

#include <string.h>

#include <algorithm>
#include <chrono>
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

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *table_dev = nullptr;
    char *table_host = nullptr;
    size_t table_cap = 0;
    bool busy = false;
    std::vector<int> reqs;
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
};

namespace {

std::string cache_key(const dctf_request &r)
{
    std::string k;
    const int hdr[4] = {r.kh, r.kw, r.N, r.border};
    k.append(reinterpret_cast<const char *>(hdr), sizeof(hdr));
    k.append(reinterpret_cast<const char *>(r.mask_host), sizeof(double) * r.kh * r.kw);
    return k;
}

dctf_status cache_get(dctf_server s, const dctf_request &r, hipStream_t stream, CacheEntry **out)
{
    const std::string key = cache_key(r);
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
    dctf_operator op = nullptr;
    dctf_status st = dctf_build_operator(r.mask_host, r.kh, r.kw, r.N, r.border, stream, &op);
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

void release_slot(dctf_server s, Slot &sl, dctf_request *reqs, double t)
{
    for (int id : sl.reqs) {
        reqs[id].done_s = t;
        reqs[id].status = DCTF_OK;
    }
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

extern "C" dctf_status dctf_server_run(dctf_server s, dctf_request *reqs, int n)
{
    if (s == nullptr || n < 0 || (n > 0 && reqs == nullptr))
        return DCTF_EINVAL;
    for (int i = 0; i < n; ++i) {
        const dctf_request &r = reqs[i];
        if ((i > 0 && r.arrival_s < reqs[i - 1].arrival_s) || !(r.arrival_s >= 0.0) || r.B < 1 ||
            (r.N != 8 && r.N != 16) || r.mask_host == nullptr || r.kh < 1 || r.kw < 1 || r.kh > 2 * r.N + 1 ||
            r.kw > 2 * r.N + 1 || (r.border != DCTF_BORDER_ZERO && r.border != DCTF_BORDER_REPLICATE) ||
            r.in_dev == nullptr || ((uintptr_t)r.in_dev & 15) || ((uintptr_t)r.out_dev & 15))
            return DCTF_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        reqs[i].admit_s = reqs[i].launch_s = reqs[i].done_s = -1.0;
        reqs[i].status = DCTF_EBUSY;
        reqs[i].batch = -1;
    }
    const int J = s->cfg.max_batch_jobs;
    std::deque<int> pending;
    int next = 0, finished = 0;
    std::vector<dctf_job> jobs;
    std::vector<char> table;
    std::vector<dctf_operator> ops;
    dctf_status err = DCTF_OK;
    const double t0 = now_s();

    while (finished < n && err == DCTF_OK) {
        bool progress = false;
        double t = now_s() - t0;
        while (next < n && reqs[next].arrival_s <= t) {
            pending.push_back(next++);
            progress = true;
        }
        int inflight = 0;
        for (Slot &sl : s->slots) {
            if (!sl.busy)
                continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finished += (int)sl.reqs.size();
                release_slot(s, sl, reqs, now_s() - t0);
                progress = true;
            } else if (q != hipErrorNotReady) {
                err = DCTF_EHIP;
            } else {
                ++inflight;
            }
        }
        for (Slot &sl : s->slots) {
            if (sl.busy || pending.empty() || err != DCTF_OK)
                continue;
            t = now_s() - t0;
            jobs.clear();
            while (!pending.empty() && (int)sl.reqs.size() < J) {
                const int id = pending.front();
                dctf_request &r = reqs[id];
                const size_t bytes = align256((size_t)r.B * r.N * r.N * sizeof(float));
                if (bytes > (size_t)s->cfg.arena_bytes) {
                    pending.pop_front();
                    r.status = DCTF_EBUSY;
                    r.admit_s = r.done_s = t;
                    ++s->stats.rejected;
                    ++finished;
                    continue;
                }
                size_t off;
                if (!s->arena.alloc(bytes, &off))
                    break;   // admit in arrival order: wait for memory
                pending.pop_front();
                CacheEntry *e = nullptr;
                err = cache_get(s, r, sl.stream, &e);
                if (err != DCTF_OK) {
                    s->arena.release(off, bytes);
                    break;
                }
                r.admit_s = t;
                sl.reqs.push_back(id);
                sl.offs.push_back(off);
                sl.sizes.push_back(bytes);
                sl.entries.push_back(e);
                jobs.push_back({e->op, r.in_dev, reinterpret_cast<float *>(static_cast<char *>(s->arena_dev) + off),
                                r.B});
            }
            if (sl.reqs.empty())
                break;   // the head request waits for arena space
            BatchArgs a;
            err = plan_batch(jobs.data(), (int)jobs.size(), s->cfg.prec, table, a, ops);
            if (err == DCTF_OK && table.size() > sl.table_cap)
                err = DCTF_EINVAL;
            if (err == DCTF_OK) {
                memcpy(sl.table_host, table.data(), table.size());
                hipError_t e = hipMemcpyAsync(sl.table_dev, sl.table_host, table.size(), hipMemcpyHostToDevice,
                                              sl.stream);
                rebase_batch(a, sl.table_dev);
                if (e == hipSuccess)
                    e = launch_batch(a, sl.stream);
                for (size_t k = 0; k < sl.reqs.size() && e == hipSuccess; ++k) {
                    dctf_request &r = reqs[sl.reqs[k]];
                    if (r.out_dev)
                        e = hipMemcpyAsync(r.out_dev, jobs[k].out, (size_t)r.B * r.N * r.N * sizeof(float),
                                           hipMemcpyDeviceToDevice, sl.stream);
                }
                if (e == hipSuccess)
                    e = hipEventRecord(sl.done, sl.stream);
                if (e != hipSuccess)
                    err = DCTF_EHIP;
            }
            const double tl = now_s() - t0;
            for (int id : sl.reqs) {
                reqs[id].launch_s = tl;
                reqs[id].batch = (int)s->stats.batches;
            }
            ++s->stats.batches;
            sl.busy = true;
            ++inflight;
            progress = true;
            s->stats.peak_inflight_batches = std::max<int64_t>(s->stats.peak_inflight_batches, inflight);
            s->stats.peak_arena_bytes = std::max<int64_t>(s->stats.peak_arena_bytes, (int64_t)s->arena.used());
        }
        (void)progress;   // the loop polls: arrivals are due at wall-clock times
    }
    // Drain whatever is still in flight (also after an error).
    for (Slot &sl : s->slots) {
        if (!sl.busy)
            continue;
        const hipError_t e = hipEventSynchronize(sl.done);
        if (e != hipSuccess && err == DCTF_OK)
            err = DCTF_EHIP;
        release_slot(s, sl, reqs, now_s() - t0);
    }
    s->stats.busy_s += now_s() - t0;
    return err;
}
