// Serving runtime: continuous batching of P-NDF requests over resident maps.
//
// Threads: callers submit / wait; one scheduler thread owns the streams.  The
// scheduler repeatedly (1) retires finished batches (event query), copying each
// piece's results from pinned staging to the caller's buffer, and completing a
// request (releasing its staging) once all its pieces are back, and (2) fills
// every idle slot with a new batch: the first waiting request fixes the map, then
// waiting requests of that map each give a piece of at most chunk_queries queries,
// in queue order, while the batch has room.  A request that still has queries left
// after giving a piece goes to the back of the queue, so requests share the device
// piece by piece (round robin) and a small request never waits for the whole of a
// large one.  A batch is H2D copies into the slot's contiguous query buffer, one
// evaluation (a plain per-batch launch or the slot's persistent plan), D2H copies
// into staging and an event, all on the slot's stream, so the batches of different
// slots overlap on the device: one batch's tail runs beside the next batch's bulk.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pndf_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds(Clock::time_point t) { return std::chrono::duration<double>(t.time_since_epoch()).count(); }

// First-fit allocator over one pinned host arena (offsets in bytes, 256-aligned).
class StagingPool {
  public:
    bool init(size_t bytes)
    {
        size_ = bytes;
        if (hipHostMalloc(&base_, bytes, hipHostMallocDefault) != hipSuccess) return false;
        free_[0] = bytes;
        return true;
    }
    ~StagingPool()
    {
        if (base_) (void)hipHostFree(base_);
    }
    void* alloc(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return (char*)base_ + off;
            }
        }
        return nullptr;
    }
    void release(void* p)
    {
        const size_t off = (size_t)((char*)p - (char*)base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }

  private:
    void* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
    std::map<size_t, size_t> used_;
};

struct Request {
    uint64_t ticket = 0;
    int map = 0;
    int64_t nq = 0;
    int64_t dispatched = 0;   // queries handed to batches
    int64_t returned = 0;     // queries whose results are in user_out
    pndf_query* q = nullptr;  // pinned staging: queries, then nq floats of results
    float* res = nullptr;
    float* user_out = nullptr;
    double t_arrive = 0, t_done = 0;
    int state = 0;  // 0 waiting (queries left to dispatch), 1 all dispatched, 2 done
};

struct Piece {
    Request* r;
    int64_t off, n;  // queries [off, off + n) of the request
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    pndf_query* d_q = nullptr;
    float* d_out = nullptr;
    std::vector<pndf_plan*> plans;  // one per map
    std::vector<Piece> pieces;
    bool busy = false;
};

}  // namespace

struct pndf_server {
    std::vector<const pndf_hier*> maps;
    pndf_server_opts opts{};
    std::vector<Slot> slots;
    StagingPool pool;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, Request*> live;
    uint64_t next_ticket = 1;
    int admitted = 0;
    bool stop = false;
    std::thread worker;
    hipError_t fault = hipSuccess;
    // statistics
    std::vector<double> lat_ms;
    uint64_t refused = 0, queries = 0, batches = 0, batch_reqs = 0;
    double t_first = -1, t_last = -1;
};

namespace {

void finish_slot(pndf_server* s, Slot& sl)
{
    const double now = seconds(Clock::now());
    std::lock_guard<std::mutex> g(s->mu);
    for (const Piece& p : sl.pieces) {
        Request* r = p.r;
        std::memcpy(r->user_out + p.off, r->res + p.off, sizeof(float) * (size_t)p.n);
        r->returned += p.n;
        if (r->returned < r->nq) continue;
        s->pool.release(r->q);
        r->q = nullptr;
        r->res = nullptr;
        r->t_done = now;
        r->state = 2;
        s->lat_ms.push_back(1e3 * (now - r->t_arrive));
        s->queries += (uint64_t)r->nq;
        --s->admitted;
    }
    s->t_last = now;
    sl.pieces.clear();
    sl.busy = false;
    s->cv_done.notify_all();
}

// Build a batch for `sl` from the waiting queue (caller holds the lock): requests of
// the first waiting request's map give pieces of at most chunk queries in queue
// order while the batch has room; those with queries left move to the back.
bool take_batch(pndf_server* s, Slot& sl)
{
    if (s->pending.empty()) return false;
    const int map = s->pending.front()->map;
    const int64_t chunk = s->opts.chunk_queries > 0 ? s->opts.chunk_queries : s->opts.max_batch_queries;
    int64_t total = 0;
    std::deque<Request*> kept, rotated;
    for (Request* r : s->pending) {
        const int64_t room = s->opts.max_batch_queries - total;
        if (r->map != map || room <= 0) {
            kept.push_back(r);
            continue;
        }
        const int64_t left = r->nq - r->dispatched;
        // a request is split only when it exceeds a chunk: a whole request that fits
        // the remaining room goes in one piece
        const int64_t n = left <= room && left <= chunk ? left : std::min(chunk, room);
        if (n < left && n < chunk && left <= chunk) {
            kept.push_back(r);  // would split a small request across batches: wait for a batch with room
            continue;
        }
        sl.pieces.push_back(Piece{r, r->dispatched, n});
        r->dispatched += n;
        total += n;
        if (r->dispatched < r->nq)
            rotated.push_back(r);
        else
            r->state = 1;
    }
    s->pending.swap(kept);
    for (Request* r : rotated) s->pending.push_back(r);
    return !sl.pieces.empty();
}

hipError_t launch_slot(pndf_server* s, Slot& sl)
{
    const int map = sl.pieces.front().r->map;
    int64_t off = 0;
    hipError_t e = hipSuccess;
    for (const Piece& p : sl.pieces) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.d_q + off, p.r->q + p.off, sizeof(pndf_query) * (size_t)p.n,
                               hipMemcpyHostToDevice, sl.stream);
        off += p.n;
    }
    if (e == hipSuccess) {
        pndf_status st;
        if (s->opts.algo == PNDF_ALGO_PERSISTENT) {
            st = pndf_plan_eval(sl.plans[map], sl.d_q, off, sl.d_out, sl.stream);
        } else {
            const pndf_eval_opts eo{s->opts.kernel, s->opts.tau, s->opts.sigma_to_r, PNDF_ALGO_PLAIN, 0};
            st = pndf_eval_batch(s->maps[map], sl.d_q, off, &eo, sl.d_out, sl.stream);
        }
        if (st != PNDF_OK) e = hipErrorLaunchFailure;
    }
    off = 0;
    for (const Piece& p : sl.pieces) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(p.r->res + p.off, sl.d_out + off, sizeof(float) * (size_t)p.n,
                               hipMemcpyDeviceToHost, sl.stream);
        off += p.n;
    }
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e;
}

void scheduler(pndf_server* s)
{
    while (true) {
        bool progress = false;
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finish_slot(s, sl);
                progress = true;
            } else if (q != hipErrorNotReady) {
                std::lock_guard<std::mutex> g(s->mu);
                s->fault = q;
                s->stop = true;
            }
        }
        for (Slot& sl : s->slots) {
            if (sl.busy) continue;
            bool got;
            {
                std::lock_guard<std::mutex> g(s->mu);
                got = take_batch(s, sl);
                if (got) {
                    ++s->batches;
                    s->batch_reqs += sl.pieces.size();
                }
            }
            if (!got) break;
            const hipError_t e = launch_slot(s, sl);
            sl.busy = true;
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> g(s->mu);
                s->fault = e;
                s->stop = true;
            }
            progress = true;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) {
            s->cv_done.notify_all();
            break;
        }
        if (!progress) {
            bool any_busy = false;
            for (Slot& sl : s->slots) any_busy |= sl.busy;
            if (any_busy || !s->pending.empty())
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

pndf_status fail(const char* msg, pndf_status st = PNDF_EINVAL)
{
    pndf::set_error(msg);
    return st;
}

void destroy_server(pndf_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        for (pndf_plan* p : sl.plans) pndf_plan_destroy(p);
        (void)hipFree(sl.d_q);
        (void)hipFree(sl.d_out);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto& kv : s->live) delete kv.second;
    delete s;
}

pndf_status submit_at(pndf_server* s, int32_t map, const pndf_query* h_q, int64_t nq, float* h_out,
                      double t_arrive, uint64_t* ticket)
{
    if (!s || !ticket) return fail("NULL argument");
    if (map < 0 || map >= (int)s->maps.size()) return fail("map index out of range");
    if (nq < 1 || nq > s->opts.max_batch_queries) return fail("request size out of range");
    if (!h_q || !h_out) return fail("NULL query or output pointer");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->fault != hipSuccess) return pndf::hip_fail(s->fault, "server device error");
    if (s->admitted >= s->opts.max_pending) {
        ++s->refused;
        pndf::set_error("pending limit reached");
        return PNDF_EAGAIN;
    }
    const size_t bytes = (sizeof(pndf_query) + sizeof(float)) * (size_t)nq + 256;
    void* stage = s->pool.alloc(bytes);
    if (!stage) {
        ++s->refused;
        pndf::set_error("memory budget exhausted");
        return PNDF_EAGAIN;
    }
    Request* r = new Request;
    r->ticket = s->next_ticket++;
    r->map = map;
    r->nq = nq;
    r->q = (pndf_query*)stage;
    r->res = (float*)((char*)stage + (((sizeof(pndf_query) * (size_t)nq) + 255) & ~(size_t)255));
    r->user_out = h_out;
    r->t_arrive = t_arrive;
    std::memcpy(r->q, h_q, sizeof(pndf_query) * (size_t)nq);
    s->live[r->ticket] = r;
    s->pending.push_back(r);
    ++s->admitted;
    if (s->t_first < 0) s->t_first = seconds(Clock::now());
    *ticket = r->ticket;
    lk.unlock();
    s->cv_work.notify_one();
    return PNDF_OK;
}

}  // namespace

extern "C" {

pndf_status pndf_server_create(const pndf_hier* const* maps, int32_t nmaps, const pndf_server_opts* opts,
                               pndf_server** out)
{
    if (!out) return fail("out is NULL");
    *out = nullptr;
    if (!maps || nmaps < 1 || !opts) return fail("need at least one map and options");
    for (int k = 0; k < nmaps; ++k)
        if (!maps[k]) return fail("NULL map");
    const pndf_server_opts& o = *opts;
    if (o.slots < 1 || o.slots > 16) return fail("slots must be in [1, 16]");
    if (o.max_batch_queries < 1 || o.max_batch_queries >= ((int64_t)1 << 31)) return fail("bad max_batch_queries");
    if (o.max_pending < 1) return fail("max_pending must be >= 1");
    if (o.chunk_queries < 0) return fail("chunk_queries must be >= 0");
    if (o.memory_budget < (int64_t)(28 * o.max_batch_queries + 512)) return fail("memory budget below one batch");
    if (o.algo != PNDF_ALGO_AUTO && o.algo != PNDF_ALGO_PLAIN && o.algo != PNDF_ALGO_PERSISTENT)
        return fail("algo must be AUTO, PLAIN or PERSISTENT");
    if (o.kernel < PNDF_KERNEL_GAUSSIAN || o.kernel > PNDF_KERNEL_BOX) return fail("unknown kernel");
    if (o.tau > 0.f)
        for (int k = 0; k < nmaps; ++k)
            if (!maps[k]->cluster) return fail("tau > 0 needs hierarchies built with clusters");
    pndf_server* s = new (std::nothrow) pndf_server;
    if (!s) return PNDF_ENOMEM;
    s->maps.assign(maps, maps + nmaps);
    s->opts = o;
    if (s->opts.sigma_to_r <= 0.f) s->opts.sigma_to_r = 3.f;
    if (!s->pool.init((size_t)o.memory_budget)) {
        delete s;
        return fail("pinned staging allocation failed", PNDF_ENOMEM);
    }
    pndf_eval_opts eo{o.kernel, o.tau, o.sigma_to_r > 0.f ? o.sigma_to_r : 3.f,
                      PNDF_ALGO_PERSISTENT, 0};
    s->slots.resize((size_t)o.slots);
    pndf_status st = PNDF_OK;
    for (Slot& sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.d_q, sizeof(pndf_query) * (size_t)o.max_batch_queries);
        if (e == hipSuccess) e = hipMalloc(&sl.d_out, sizeof(float) * (size_t)o.max_batch_queries);
        if (e != hipSuccess) {
            st = pndf::hip_fail(e, "pndf_server_create");
            break;
        }
        for (int k = 0; k < nmaps && st == PNDF_OK && o.algo == PNDF_ALGO_PERSISTENT; ++k) {
            pndf_plan* p = nullptr;
            st = pndf_plan_create(maps[k], o.max_batch_queries, &eo, o.tuning.blocks_per_cu > 0 ? &o.tuning : nullptr,
                                  sl.stream, &p);
            if (st == PNDF_OK) sl.plans.push_back(p);
        }
        if (st != PNDF_OK) break;
    }
    if (st != PNDF_OK) {
        destroy_server(s);
        return st;
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return PNDF_OK;
}

pndf_status pndf_server_submit(pndf_server* srv, int32_t map, const pndf_query* h_q, int64_t nq,
                               float* h_out, uint64_t* ticket)
{
    return submit_at(srv, map, h_q, nq, h_out, seconds(Clock::now()), ticket);
}

pndf_status pndf_server_wait(pndf_server* srv, uint64_t ticket, double timeout_s, double* latency_ms)
{
    if (!srv) return fail("server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->live.find(ticket);
    if (it == srv->live.end()) return fail("unknown or already collected ticket");
    Request* r = it->second;
    auto ready = [&] { return r->state == 2 || srv->fault != hipSuccess; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        pndf::set_error("timed out");
        return PNDF_EAGAIN;
    }
    if (r->state != 2) return pndf::hip_fail(srv->fault, "server device error");
    if (latency_ms) *latency_ms = 1e3 * (r->t_done - r->t_arrive);
    srv->live.erase(it);
    delete r;
    return PNDF_OK;
}

pndf_status pndf_server_drain(pndf_server* srv)
{
    if (!srv) return fail("server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->admitted == 0 || srv->fault != hipSuccess; });
    if (srv->fault != hipSuccess) return pndf::hip_fail(srv->fault, "server device error");
    return PNDF_OK;
}

pndf_status pndf_server_get_stats(pndf_server* srv, pndf_server_stats* out)
{
    if (!srv || !out) return fail("NULL argument");
    std::lock_guard<std::mutex> g(srv->mu);
    std::vector<double> v = srv->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
        return v[k];
    };
    out->completed = v.size();
    out->refused = srv->refused;
    out->queries = srv->queries;
    out->batches = srv->batches;
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    out->max_ms = v.empty() ? 0.0 : v.back();
    out->mean_batch_requests = srv->batches ? (double)srv->batch_reqs / (double)srv->batches : 0.0;
    out->busy_s = (srv->t_first >= 0 && srv->t_last >= 0) ? srv->t_last - srv->t_first : 0.0;
    return PNDF_OK;
}

pndf_status pndf_server_reset_stats(pndf_server* srv)
{
    if (!srv) return fail("server is NULL");
    std::lock_guard<std::mutex> g(srv->mu);
    srv->lat_ms.clear();
    srv->refused = srv->queries = srv->batches = srv->batch_reqs = 0;
    srv->t_first = srv->t_last = -1;
    return PNDF_OK;
}

pndf_status pndf_server_replay(pndf_server* srv, int64_t nreq, const int32_t* map_ids,
                               const double* arrival_s, const pndf_query* const* h_q,
                               const int64_t* nq, float* const* h_out, double* latency_ms)
{
    if (!srv || nreq < 0 || (nreq > 0 && (!map_ids || !arrival_s || !h_q || !nq || !h_out)))
        return fail("bad replay arguments");
    // the whole trace is checked before anything is submitted
    for (int64_t k = 0; k < nreq; ++k) {
        if (!(arrival_s[k] >= 0.0) || (k > 0 && arrival_s[k] < arrival_s[k - 1]))
            return fail("arrival times must be finite, >= 0 and non-decreasing");
        if (map_ids[k] < 0 || map_ids[k] >= (int32_t)srv->maps.size()) return fail("map index out of range");
        if (nq[k] < 1 || nq[k] > srv->opts.max_batch_queries) return fail("request size out of range");
        if (!h_q[k] || !h_out[k]) return fail("NULL query or output pointer");
    }
    std::vector<uint64_t> tickets((size_t)nreq, 0);
    pndf_status failed = PNDF_OK;
    int64_t submitted = 0;
    const Clock::time_point t0 = Clock::now();
    for (int64_t k = 0; k < nreq && failed == PNDF_OK; ++k) {
        const Clock::time_point due =
            t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[k]));
        std::this_thread::sleep_until(due);
        const double t_arr = seconds(due);
        while (true) {
            const pndf_status st = submit_at(srv, map_ids[k], h_q[k], nq[k], h_out[k], t_arr, &tickets[k]);
            if (st == PNDF_OK) {
                ++submitted;
                break;
            }
            if (st != PNDF_EAGAIN) {
                failed = st;
                break;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }
    // every submitted request is waited for, also after a failure: their results go
    // to the caller's buffers, which must not be released before
    const std::string first_error = failed != PNDF_OK ? std::string(pndf_last_error()) : std::string();
    for (int64_t k = 0; k < submitted; ++k) {
        double ms = 0;
        const pndf_status st = pndf_server_wait(srv, tickets[k], -1.0, &ms);
        if (st != PNDF_OK && failed == PNDF_OK) failed = st;
        if (latency_ms) latency_ms[k] = ms;
    }
    if (!first_error.empty()) pndf::set_error(first_error);
    return failed;
}

void pndf_server_destroy(pndf_server* srv) { destroy_server(srv); }

}  // extern "C"
