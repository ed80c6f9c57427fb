// server.hip -- a serving loop for stochastic lookups: continuous batching of
// uneven requests against resident textures, memory-based admission, and
// per-request latency.
//
// A worker thread owns the device work.  Each round it
//   1. admits pending requests in arrival order while a resident slot and
//      room in the device arena (queries staged from host memory, results)
//      are free;
//   2. takes the next chunk (at most `chunk_queries`) of every resident
//      request, groups the chunks by (texture, filter) and serves each group
//      with one kernel launch over a chunk table;
//   3. copies the results of requests whose last chunk was launched to the
//      caller's buffer and records a completion event;
//   4. retires requests whose completion event has fired: latency = fire time
//      observed - arrival time, arena space freed.
// Up to two rounds are in flight on the stream, so admission and the next
// launch overlap the device work.  Requests arriving while others run join
// the next round.  A query's random draw depends only on (request seed,
// index within the request), so every result equals what stf_filter returns
// for the same request alone.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "device_common.h"
#include "stf_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class Arena {
public:
    void init(size_t size)
    {
        free_.clear();
        free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    void reset_peak() { peak_ = used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

enum ReqState { PENDING, RESIDENT, FINISHING, DONE, CANCELLED, FAILED };

struct Request {
    uint64_t ticket;
    const stf_texture* tex;
    const float* q_user;
    float* out_user;
    int32_t* idx_user;
    int64_t n;
    int filter;
    uint32_t key;
    uint32_t flags;
    double t_arrival;
    int dims, channels;
    size_t off = 0, bytes = 0;
    const float* q_dev = nullptr;
    float* out_dev = nullptr;
    int32_t* idx_dev = nullptr;
    int64_t next = 0;
    bool cancel = false;
    int state = PENDING;
    hipEvent_t done_ev = nullptr;
    int64_t round = -1;       // round whose launch carries the request's last chunk
    int64_t last_round = -1;  // latest round that launched any chunk of the request
    int32_t res_pos = -1;     // index in the server's resident list
};

constexpr int RING = 4;

}  // namespace

struct stf_server {
    stf_server_config cfg;
    int device;
    hipStream_t stream;
    char* arena_dev = nullptr;
    Arena arena;
    ServeChunk* desc_host = nullptr;   // RING * max_resident, pinned
    ServeChunk* desc_dev = nullptr;
    hipEvent_t round_ev[RING];
    int64_t round = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> resident;
    std::unordered_map<uint64_t, Request*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    // statistics since the last reset
    std::vector<double> lat_ms;
    int64_t completed = 0, cancelled = 0, queries = 0, launches = 0, peak_resident = 0;
    double t_first = 0.0, t_last = 0.0;
    int64_t n_rounds = 0;
    std::string error;
    // completion events of released requests, reused by later ones (creating
    // and destroying one per request costs runtime work under the lock at
    // tens of thousands of requests per second)
    std::vector<hipEvent_t> event_pool;
};

namespace {

void record_failure(stf_server* s, const char* what, hipError_t e)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    s->error = buf;
}

// Removes r from the resident list in O(1) (the list's order does not
// matter: a query's draw depends only on its request's seed and its index).
void unlist_resident(stf_server* s, Request* r)
{
    // caller holds s->mu
    const int32_t pos = r->res_pos;
    if (pos < 0) return;
    Request* last = s->resident.back();
    s->resident[pos] = last;
    last->res_pos = pos;
    s->resident.pop_back();
    r->res_pos = -1;
}

void retire(stf_server* s, Request* r, int state, double t)
{
    // caller holds s->mu
    if (r->bytes) s->arena.release(r->off, r->bytes);
    r->bytes = 0;
    r->state = state;
    // the event has served its purpose (the worker saw it complete, or the
    // request never reached it): back to the pool for later requests
    if (r->done_ev && s->event_pool.size() < 65536) {
        s->event_pool.push_back(r->done_ev);
        r->done_ev = nullptr;
    }
    if (state == DONE) {
        s->completed += 1;
        s->queries += r->n;
        s->lat_ms.push_back((t - r->t_arrival) * 1e3);
        if (s->t_first == 0.0 || r->t_arrival < s->t_first) s->t_first = r->t_arrival;
        s->t_last = std::max(s->t_last, t);
    } else if (state == CANCELLED) {
        s->cancelled += 1;
    }
    s->cv_done.notify_all();
}

void worker_main(stf_server* s)
{
    (void)hipSetDevice(s->device);
    const int qpb3 = serve3d_queries_per_block(), qpb2 = serve2d_queries_per_block();
    std::vector<Request*> finishing, still;
    for (;;) {
        std::vector<Request*> admitted;
        std::vector<Request*> round_reqs;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // retire cancelled residents once no copy or launch of theirs is in
            // flight (the stream is in order: a later event implies earlier work)
            for (size_t k = 0; k < s->resident.size();) {
                Request* r = s->resident[k];
                bool quiet = false;
                if (r->cancel && r->state == RESIDENT) {
                    if (r->last_round >= 0)   // launched: the event of its last round
                        quiet = s->round - r->last_round >= RING ||
                                hipEventQuery(s->round_ev[r->last_round % RING]) == hipSuccess;
                    else   // admitted, never launched: only the staging copy of host queries, which done_ev marks
                        quiet = (r->flags & STF_SERVE_QUERIES_ON_DEVICE) || hipEventQuery(r->done_ev) == hipSuccess;
                }
                if (quiet) {
                    unlist_resident(s, r);   // the last entry moves to k
                    retire(s, r, CANCELLED, now_s());
                } else {
                    ++k;
                }
            }
            while (!s->pending.empty() && (int)s->resident.size() < s->cfg.max_resident) {
                Request* r = s->pending.front();
                // the arena stages host queries and host results only: device
                // results are written in place by the kernels
                const bool dev_q = r->flags & STF_SERVE_QUERIES_ON_DEVICE;
                const bool dev_out = r->flags & STF_SERVE_RESULTS_ON_DEVICE;
                const size_t need = (dev_q ? 0 : (size_t)r->n * 4 * r->dims + 256) +
                                    (dev_out ? 0
                                             : (size_t)r->n * 4 * r->channels + 256 +
                                                   (r->idx_user ? (size_t)r->n * 4 * r->dims + 256 : 0));
                size_t off = 0;
                if (need && !s->arena.alloc(need, &off)) break;
                s->pending.pop_front();
                r->off = off;
                r->bytes = need;
                char* base = s->arena_dev + off;
                size_t o = 0;
                if (dev_q) {
                    r->q_dev = r->q_user;
                } else {
                    r->q_dev = (const float*)base;
                    o += ((size_t)r->n * 4 * r->dims + 255) & ~(size_t)255;
                }
                if (dev_out) {
                    r->out_dev = r->out_user;
                    r->idx_dev = r->idx_user;
                } else {
                    r->out_dev = (float*)(base + o);
                    o += ((size_t)r->n * 4 * r->channels + 255) & ~(size_t)255;
                    r->idx_dev = r->idx_user ? (int32_t*)(base + o) : nullptr;
                }
                r->state = RESIDENT;
                r->res_pos = (int32_t)s->resident.size();
                s->resident.push_back(r);
                admitted.push_back(r);
            }
            s->peak_resident = std::max<int64_t>(s->peak_resident, (int64_t)s->resident.size());
            for (Request* r : s->resident)
                if (r->state == RESIDENT && !r->cancel && r->next < r->n) round_reqs.push_back(r);
            if (round_reqs.empty() && finishing.empty() && admitted.empty()) {
                if (s->stop && s->pending.empty()) break;
                s->cv_work.wait_for(lk, std::chrono::microseconds(200));
                continue;
            }
        }
        hipError_t e = hipSuccess;
        for (Request* r : admitted)
            if (!(r->flags & STF_SERVE_QUERIES_ON_DEVICE) && e == hipSuccess) {
                e = hipMemcpyAsync((void*)r->q_dev, r->q_user, (size_t)r->n * 4 * r->dims, hipMemcpyHostToDevice,
                                   s->stream);
                // marks the copy, so that a request cancelled before its first
                // launch is retired (and its caller told) only once the copy
                // has read the caller's queries
                if (e == hipSuccess) e = hipEventRecord(r->done_ev, s->stream);
            }
        if (!round_reqs.empty() && e == hipSuccess) {
            // at most two rounds in flight; the descriptor slot of round - RING is free
            int slot = (int)(s->round % RING);
            if (s->round >= 2) e = hipEventSynchronize(s->round_ev[(s->round - 2) % RING]);
            if (s->round >= RING && e == hipSuccess) e = hipEventSynchronize(s->round_ev[slot]);
            ServeChunk* hd = s->desc_host + (size_t)slot * s->cfg.max_resident;
            ServeChunk* dd = s->desc_dev + (size_t)slot * s->cfg.max_resident;
            // group by (texture, filter); each group is contiguous in the table
            std::stable_sort(round_reqs.begin(), round_reqs.end(), [](const Request* a, const Request* b) {
                if (a->tex != b->tex) return a->tex < b->tex;
                return a->filter < b->filter;
            });
            struct Group {
                const stf_texture* tex;
                int filter, first, count, blocks;
            };
            std::vector<Group> groups;
            for (size_t k = 0; k < round_reqs.size(); ++k) {
                Request* r = round_reqs[k];
                bool is3d = r->tex->kind == STF_KIND_GRID3D;
                int qpb = is3d ? qpb3 : qpb2;
                if (groups.empty() || groups.back().tex != r->tex || groups.back().filter != r->filter)
                    groups.push_back({r->tex, r->filter, (int)k, 0, 0});
                Group& g = groups.back();
                int64_t cnt = std::min<int64_t>(s->cfg.chunk_queries, r->n - r->next);
                ServeChunk c;
                c.q = r->q_dev + r->next * r->dims;
                c.out = r->out_dev + r->next * r->channels;
                c.idx = r->idx_dev ? r->idx_dev + r->next * r->dims : nullptr;
                c.count = (int32_t)cnt;
                c.qid0 = (uint32_t)r->next;
                c.key = r->key;
                c.block0 = g.blocks;
                hd[k] = c;
                g.count += 1;
                g.blocks += (int)((cnt + qpb - 1) / qpb);
                r->next += cnt;
                r->last_round = s->round;
                if (r->next == r->n) r->round = s->round;
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(dd, hd, round_reqs.size() * sizeof(ServeChunk), hipMemcpyHostToDevice, s->stream);
            for (const Group& g : groups) {
                if (e != hipSuccess) break;
                e = g.tex->kind == STF_KIND_GRID3D
                        ? launch_serve3d(g.tex, g.filter, dd + g.first, g.count, g.blocks, s->stream)
                        : launch_serve2d(g.tex, g.filter, dd + g.first, g.count, g.blocks, s->stream);
                s->launches += 1;
            }
            // results of requests finished in this round go to the caller's
            // host buffers (device results are already in place)
            for (Request* r : round_reqs) {
                if (r->next != r->n || e != hipSuccess) continue;
                if (!(r->flags & STF_SERVE_RESULTS_ON_DEVICE)) {
                    e = hipMemcpyAsync(r->out_user, r->out_dev, (size_t)r->n * 4 * r->channels,
                                       hipMemcpyDeviceToHost, s->stream);
                    if (e == hipSuccess && r->idx_user)
                        e = hipMemcpyAsync(r->idx_user, r->idx_dev, (size_t)r->n * 4 * r->dims, hipMemcpyDeviceToHost,
                                           s->stream);
                }
                if (e == hipSuccess) e = hipEventRecord(r->done_ev, s->stream);
                {
                    std::lock_guard<std::mutex> lk(s->mu);   // poll, wait and cancel read the state under the lock
                    r->state = FINISHING;
                }
                finishing.push_back(r);
            }
            if (e == hipSuccess) e = hipEventRecord(s->round_ev[slot], s->stream);
            s->round += 1;
            s->n_rounds += 1;
        }
        if (e != hipSuccess) {
            // let whatever the failed round did enqueue drain first, so that no
            // launch or copy still writes into a caller's buffer after its
            // request has been reported as failed
            (void)hipStreamSynchronize(s->stream);
            (void)hipGetLastError();
            std::lock_guard<std::mutex> lk(s->mu);
            record_failure(s, "serving round failed", e);
            for (Request* r : s->resident) {
                r->res_pos = -1;
                retire(s, r, FAILED, now_s());
            }
            s->resident.clear();
            finishing.clear();
            continue;
        }
        // retire finished requests; block on the oldest one only when there is
        // nothing else to do
        bool idle = round_reqs.empty() && admitted.empty();
        still.clear();
        for (size_t k = 0; k < finishing.size(); ++k) {
            Request* r = finishing[k];
            hipError_t q = idle && k == 0 ? hipEventSynchronize(r->done_ev) : hipEventQuery(r->done_ev);
            if (q == hipErrorNotReady) {
                still.push_back(r);
                continue;
            }
            double t = now_s();
            std::lock_guard<std::mutex> lk(s->mu);
            unlist_resident(s, r);
            retire(s, r, q == hipSuccess ? DONE : FAILED, t);
        }
        finishing.swap(still);
    }
}

Request* find_req(stf_server* s, uint64_t ticket)
{
    auto it = s->all.find(ticket);
    return it == s->all.end() ? nullptr : it->second;
}

stf_status submit_locked(stf_server* s, const stf_texture* tex, const float* queries, int64_t n,
                         stf_filter_kind filter, uint64_t seed, float* out, int32_t* out_index, uint32_t flags,
                         double t_arrival, uint64_t* ticket)
{
    Request* r = new (std::nothrow) Request();
    if (!r) return stf_fail(STF_E_OOM, "host allocation failed");
    if (!s->event_pool.empty()) {
        r->done_ev = s->event_pool.back();
        s->event_pool.pop_back();
    } else if (hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) {
        delete r;
        return stf_fail(STF_E_DEVICE, "hipEventCreate failed");
    }
    r->ticket = s->next_ticket++;
    r->tex = tex;
    r->q_user = queries;
    r->out_user = out;
    r->idx_user = out_index;
    r->n = n;
    r->filter = filter;
    r->key = stf::seed_key(seed);
    r->flags = flags;
    r->t_arrival = t_arrival;
    r->dims = tex->kind == STF_KIND_GRID3D ? 3 : 2;
    r->channels = tex->channels;
    s->all[r->ticket] = r;
    s->pending.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return STF_OK;
}

// Device allocations (base, size) seen while validating one batch of
// requests: the requests of a replay, whose buffers must all stay valid
// until it returns, often share a few pools.  Nothing is remembered across
// calls, since an allocation may be freed and its addresses reused.
using RangeCache = std::vector<std::pair<uintptr_t, size_t>>;

// True if [p, p + bytes) lies in one device allocation.
bool device_range(const void* p, size_t bytes, RangeCache* cache)
{
    const uintptr_t a = (uintptr_t)p;
    if (cache)
        for (const auto& r : *cache)
            if (a >= r.first && a - r.first <= r.second && bytes <= r.second - (a - r.first)) return true;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess ||
        (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return false;
    }
    void* base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const uintptr_t b = (uintptr_t)base;
    if (a < b || a - b > size || bytes > size - (a - b)) return false;
    if (cache && cache->size() < 64) cache->push_back({b, size});
    return true;
}

stf_status validate_request(stf_server* s, const stf_texture* tex, const float* queries, int64_t n,
                            stf_filter_kind filter, float* out, const int32_t* out_index, uint32_t flags,
                            RangeCache* cache = nullptr)
{
    if (!tex || (tex->kind != STF_KIND_GRID3D && tex->kind != STF_KIND_TEX2D && tex->kind != STF_KIND_MATERIAL))
        return stf_fail(STF_E_INVALID, "requests need a 3D grid, a 2D texture or a material");
    if (n < 1 || n > 0x7fffffff) return stf_fail(STF_E_INVALID, "n = %lld out of range (1..2^31-1)", (long long)n);
    if (!valid_filter(filter)) return stf_fail(STF_E_INVALID, "unknown filter");
    if (filter != STF_LINEAR && filter != STF_CUBIC_BSPLINE)
        return stf_fail(STF_E_UNSUPPORTED, "serving supports the linear and B-spline filters only");
    if (!queries || !out) return stf_fail(STF_E_INVALID, "queries and out are required");
    if (flags & ~(uint32_t)(STF_SERVE_QUERIES_ON_DEVICE | STF_SERVE_RESULTS_ON_DEVICE))
        return stf_fail(STF_E_INVALID, "unknown flags 0x%x", flags);
    int dims = tex->kind == STF_KIND_GRID3D ? 3 : 2;
    const bool dev_q = flags & STF_SERVE_QUERIES_ON_DEVICE, dev_out = flags & STF_SERVE_RESULTS_ON_DEVICE;
    size_t need = (dev_q ? 0 : (size_t)n * 4 * dims) + (dev_out ? 0 : (size_t)n * 4 * tex->channels +
                                                                        (size_t)n * 4 * dims) + 1024;
    if (need > (size_t)s->cfg.memory_budget_bytes)
        return stf_fail(STF_E_OOM, "request of %lld queries needs %zu bytes, more than the budget", (long long)n, need);
    if ((uintptr_t)queries % (dev_q && dims == 2 ? 8 : 4)) return stf_fail(STF_E_INVALID, "queries are misaligned");
    if (dev_out && ((uintptr_t)out % 4 || (uintptr_t)out_index % 4))
        return stf_fail(STF_E_INVALID, "out or out_index is misaligned");
    if (dev_q && !device_range(queries, (size_t)n * 4 * dims, cache))
        return stf_fail(STF_E_INVALID, "STF_SERVE_QUERIES_ON_DEVICE: queries are not n x %d floats of device memory", dims);
    if (dev_out && (!device_range(out, (size_t)n * 4 * tex->channels, cache) ||
                    (out_index && !device_range(out_index, (size_t)n * 4 * dims, cache))))
        return stf_fail(STF_E_INVALID, "STF_SERVE_RESULTS_ON_DEVICE: out / out_index are not device memory of the "
                                       "request's size");
    return STF_OK;
}

}  // namespace

extern "C" {

stf_status stf_server_create(const stf_server_config* cfg, stf_server** out)
{
    stf_clear_error();
    if (!cfg || !out) return stf_fail(STF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (cfg->memory_budget_bytes < 4096 || cfg->max_resident < 1 || cfg->max_resident > 65536 ||
        cfg->chunk_queries < 1)
        return stf_fail(STF_E_INVALID, "bad server configuration");
    stf_server* s = new (std::nothrow) stf_server();
    if (!s) return stf_fail(STF_E_OOM, "host allocation failed");
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&s->arena_dev, (size_t)cfg->memory_budget_bytes);
    size_t dbytes = (size_t)RING * cfg->max_resident * sizeof(ServeChunk);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->desc_host, dbytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s->desc_dev, dbytes);
    for (int k = 0; k < RING && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->round_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (s->arena_dev) (void)hipFree(s->arena_dev);
        if (s->desc_host) (void)hipHostFree(s->desc_host);
        if (s->desc_dev) (void)hipFree(s->desc_dev);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return stf_fail(STF_E_OOM, "allocating the server's device state failed: %s", hipGetErrorString(e));
    }
    s->arena.init((size_t)cfg->memory_budget_bytes);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return STF_OK;
}

void stf_server_destroy(stf_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Request* r : s->pending) {
            r->state = CANCELLED;
            s->cancelled += 1;
        }
        s->pending.clear();
        for (Request* r : s->resident) r->cancel = true;
        s->stop = true;
        s->cv_work.notify_all();
    }
    s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) {
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        delete kv.second;
    }
    for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
    for (int k = 0; k < RING; ++k) (void)hipEventDestroy(s->round_ev[k]);
    (void)hipFree(s->arena_dev);
    (void)hipHostFree(s->desc_host);
    (void)hipFree(s->desc_dev);
    (void)hipStreamDestroy(s->stream);
    delete s;
}

stf_status stf_server_submit(stf_server* s, const stf_texture* tex, const float* queries, int64_t n,
                             stf_filter_kind filter, uint64_t seed, float* out, int32_t* out_index, uint32_t flags,
                             uint64_t* ticket)
{
    stf_clear_error();
    if (!s || !ticket) return stf_fail(STF_E_INVALID, "NULL argument");
    stf_status st = validate_request(s, tex, queries, n, filter, out, out_index, flags);
    if (st != STF_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    return submit_locked(s, tex, queries, n, filter, seed, out, out_index, flags, now_s(), ticket);
}

stf_status stf_server_poll(stf_server* s, uint64_t ticket, int32_t* done)
{
    stf_clear_error();
    if (!s || !done) return stf_fail(STF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = find_req(s, ticket);
    if (!r) return stf_fail(STF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    *done = r->state == DONE || r->state == CANCELLED || r->state == FAILED;
    if (r->state == CANCELLED) return stf_fail(STF_E_CANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
    if (r->state == FAILED) return stf_fail(STF_E_DEVICE, "request failed: %s", s->error.c_str());
    return STF_OK;
}

stf_status stf_server_wait(stf_server* s, uint64_t ticket, double timeout_s)
{
    stf_clear_error();
    if (!s) return stf_fail(STF_E_INVALID, "NULL argument");
    if (!(timeout_s >= 0.0)) return stf_fail(STF_E_INVALID, "timeout_s = %g must be >= 0", timeout_s);
    std::unique_lock<std::mutex> lk(s->mu);
    Request* r = find_req(s, ticket);
    if (!r) return stf_fail(STF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    bool ok;
    if (timeout_s > 1e6) {   // longer than any clock arithmetic needs: wait without a deadline
        s->cv_done.wait(lk, [&] { return r->state >= DONE; });
        ok = true;
    } else {
        auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(timeout_s));
        ok = s->cv_done.wait_until(lk, deadline, [&] { return r->state >= DONE; });
    }
    if (!ok) return stf_fail(STF_E_BUSY, "request %llu not finished after %.3f s", (unsigned long long)ticket, timeout_s);
    if (r->state == CANCELLED) return stf_fail(STF_E_CANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
    if (r->state == FAILED) return stf_fail(STF_E_DEVICE, "request failed: %s", s->error.c_str());
    return STF_OK;
}

stf_status stf_server_cancel(stf_server* s, uint64_t ticket)
{
    stf_clear_error();
    if (!s) return stf_fail(STF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = find_req(s, ticket);
    if (!r) return stf_fail(STF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (r->state == PENDING) {
        s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
        retire(s, r, CANCELLED, now_s());
    } else if (r->state == RESIDENT) {
        r->cancel = true;   // no further chunks; retired once its launches are done
        s->cv_work.notify_one();
    }
    return STF_OK;
}

stf_status stf_server_release(stf_server* s, uint64_t ticket)
{
    stf_clear_error();
    if (!s) return stf_fail(STF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    Request* r = find_req(s, ticket);
    if (!r) return stf_fail(STF_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (r->state < DONE) return stf_fail(STF_E_BUSY, "request %llu is still in flight", (unsigned long long)ticket);
    s->all.erase(ticket);
    if (r->done_ev) (void)hipEventDestroy(r->done_ev);   // retire returned it to the pool unless the pool was full
    delete r;
    return STF_OK;
}

stf_status stf_server_stats(stf_server* s, stf_serve_stats* st)
{
    stf_clear_error();
    if (!s || !st) return stf_fail(STF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof(*st));
    st->completed = s->completed;
    st->cancelled = s->cancelled;
    st->queries = s->queries;
    st->launches = s->launches;
    st->rounds = s->n_rounds;
    st->peak_resident = s->peak_resident;
    st->peak_arena_bytes = (int64_t)s->arena.peak();
    st->pending = (int64_t)s->pending.size();
    st->resident = (int64_t)s->resident.size();
    if (!s->lat_ms.empty()) {
        std::vector<double> v = s->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
        double sum = 0.0;
        for (double x : v) sum += x;
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = v.back();
        st->mean_ms = sum / v.size();
        double span = s->t_last - s->t_first;
        st->lookups_per_s = span > 0 ? s->queries / span : 0.0;
        st->span_s = span;
    }
    return STF_OK;
}

stf_status stf_server_reset_stats(stf_server* s)
{
    stf_clear_error();
    if (!s) return stf_fail(STF_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    s->lat_ms.clear();
    s->completed = s->cancelled = s->queries = s->launches = s->n_rounds = 0;
    s->peak_resident = (int64_t)s->resident.size();
    s->t_first = s->t_last = 0.0;
    s->arena.reset_peak();
    return STF_OK;
}

stf_status stf_server_replay(stf_server* s, const stf_serve_request* reqs, int64_t count, uint32_t flags,
                             double timeout_s)
{
    stf_clear_error();
    if (!s || (!reqs && count)) return stf_fail(STF_E_INVALID, "NULL argument");
    RangeCache ranges;
    for (int64_t k = 0; k < count; ++k) {
        stf_status st = validate_request(s, reqs[k].tex, reqs[k].queries, reqs[k].n, reqs[k].filter, reqs[k].out,
                                         reqs[k].out_index, flags, &ranges);
        if (st != STF_OK) return st;
        if (k && reqs[k].arrival_s < reqs[k - 1].arrival_s) return stf_fail(STF_E_INVALID, "arrivals must not decrease");
    }
    if (!(timeout_s >= 0.0)) return stf_fail(STF_E_INVALID, "timeout_s = %g must be >= 0", timeout_s);
    std::vector<uint64_t> tickets;
    tickets.reserve((size_t)count);
    {
        // grown ahead: a rehash of the ticket table or a reallocation of the
        // latency record while the requests stream in would stall submission
        // and the worker (both under the lock) for milliseconds
        std::lock_guard<std::mutex> lk(s->mu);
        s->all.reserve(s->all.size() + (size_t)count);
        s->lat_ms.reserve(s->lat_ms.size() + (size_t)count);
    }
    // On an error or a time-out the requests still outstanding are cancelled
    // and waited for without a deadline before the call returns, so no copy
    // into a caller's buffer can land after it (a cancelled request is
    // retired once its last launch is done; one already copying its results
    // finishes them).
    auto quiesce = [&]() {
        for (uint64_t t : tickets) (void)stf_server_cancel(s, t);
        for (uint64_t t : tickets) (void)stf_server_wait(s, t, HUGE_VAL);
        for (uint64_t t : tickets) (void)stf_server_release(s, t);
    };
    double t0 = now_s();
    stf_status result = STF_OK;
    std::string why;
    for (int64_t k = 0; k < count && result == STF_OK; ++k) {
        double due = t0 + reqs[k].arrival_s;
        for (;;) {   // open loop: submit at the scheduled time; latency counts from it
            double dt = due - now_s();
            if (dt <= 0) break;
            if (dt > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(dt - 100e-6));
        }
        std::lock_guard<std::mutex> lk(s->mu);
        uint64_t t = 0;
        result = submit_locked(s, reqs[k].tex, reqs[k].queries, reqs[k].n, reqs[k].filter, reqs[k].seed,
                               reqs[k].out, reqs[k].out_index, flags, due, &t);
        if (result == STF_OK) tickets.push_back(t);
        else why = stf_last_error();
    }
    double deadline = now_s() + timeout_s;
    for (size_t k = 0; k < tickets.size() && result == STF_OK; ++k) {
        result = stf_server_wait(s, tickets[k], std::max(0.0, deadline - now_s()));
        if (result != STF_OK) why = stf_last_error();
    }
    quiesce();
    if (result != STF_OK) return stf_fail(result, "replay: not every request completed (%s)", why.c_str());
    return STF_OK;
}

}  // extern "C"
