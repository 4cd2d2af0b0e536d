// Continuous-batching bake server (fipt_server_*).
//
// A scheduler thread admits queued requests first come first served while
// their output fits in the server's device pool and the in-flight limit
// allows, then fills each launch of the persistent tile-bake kernel with
// tiles (contiguous runs of one request's points): first every request
// whose remaining work fits in one launch, whole, then the other requests
// in admission order.  Small requests thus finish within a launch or two
// even while large ones run, and large ones keep first-come-first-served
// order.  Two launches are kept in flight, each on its own stream, so the
// GPU never waits for the host and one launch's last wavefronts overlap
// the next launch's first; a request that arrives meanwhile joins the next
// launch that is built.  Completion is detected from each launch's event;
// a request is done when all its points' tiles have completed.
//
// A tile's points carry their index within the request into the random
// number counter, so every point's result is bitwise identical to
// fipt_bake over the request alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "fipt_internal.hpp"

namespace fipt {
int check_bake_params(const fipt_bake_params* p);
BakeLaunch make_bake_launch(fipt_scene s, const fipt_points* pts, const fipt_bake_params* p,
                            const fipt_shading* out);
}  // namespace fipt

using namespace fipt;

namespace {

enum State { QUEUED, ADMITTED, DONE, CANCELED };

struct Request {
    uint64_t ticket = 0;
    fipt_scene scene = nullptr;
    fipt_points pts{};
    fipt_bake_params params{};
    int64_t n = 0;
    int64_t planes = 0;
    int64_t bytes = 0;
    int64_t pool_off = -1;
    int64_t next_point = 0;
    int64_t done_points = 0;
    State state = QUEUED;
    int64_t t_submit = 0, t_admit = -1, t_done = -1;
    int64_t samples_per_point() const { return params.spp_d + (int64_t)params.n_levels * params.spp_s; }
};

struct TileRec {
    uint64_t ticket;
    int64_t count;
};

struct Slot {
    TileDesc* host = nullptr;   // pinned
    TileDesc* dev = nullptr;
    int32_t* counter = nullptr;   // kXcdCount point counters
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<TileRec> recs;
};

constexpr int kSlots = 2;
constexpr int64_t kAlign = 256;

}  // namespace

struct fipt_server_s {
    int32_t device = 0;
    char* pool = nullptr;
    int64_t pool_bytes = 0;
    int32_t max_inflight = 0;
    int64_t samples_per_launch = 0;
    int32_t grid = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;          // submitted, not admitted (FIFO)
    std::vector<uint64_t> active;        // admitted, some points unassigned or in flight
    std::map<uint64_t, Request> reqs;
    std::map<int64_t, int64_t> free_list;   // offset -> size
    uint64_t next_ticket = 1;
    bool stop = false;
    int64_t pool_in_use = 0;
    fipt_server_stats stats{};
    Slot slots[kSlots];
    std::thread worker;
    std::string worker_error;

    int64_t now_us() const {
        return std::chrono::duration_cast<std::chrono::microseconds>(
                   std::chrono::steady_clock::now() - t0)
            .count();
    }

    // first-fit allocation in the pool
    int64_t pool_alloc(int64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first;
                const int64_t rest = it->second - bytes;
                free_list.erase(it);
                if (rest > 0) free_list[off + bytes] = rest;
                pool_in_use += bytes;
                return off;
            }
        }
        return -1;
    }
    void pool_free(int64_t off, int64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        pool_in_use -= bytes;
        auto it = free_list.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_list.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_list.erase(next);
        }
        if (it != free_list.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_list.erase(it);
            }
        }
    }

    // caller holds mu
    void admit() {
        while (!queue.empty() && (int32_t)active.size() < max_inflight) {
            Request& r = reqs[queue.front()];
            const int64_t off = pool_alloc(r.bytes);
            if (off < 0) break;   // wait for pool space (FIFO: no overtaking)
            r.pool_off = off;
            r.state = ADMITTED;
            r.t_admit = now_us();
            active.push_back(r.ticket);
            queue.pop_front();
        }
    }

    // caller holds mu; fills slot s, returns number of tiles.
    // A launch carries up to samples_per_launch lobe samples.  Requests whose
    // unassigned work fits in one launch ("small") go first, in admission
    // order, each taken whole; the rest of the budget goes to the other
    // requests in admission order.  Small requests (and the last launch of a
    // large one) so finish within the next launch, while large requests
    // keep first-come-first-served order and are not slowed by sharing.
    int build(Slot& s) {
        s.recs.clear();
        std::vector<Request*> work;
        for (uint64_t t : active) {
            Request& r = reqs[t];
            if (r.next_point < r.n) work.push_back(&r);
        }
        if (work.empty()) return 0;
        int64_t budget = samples_per_launch;
        std::vector<int64_t> take(work.size(), 0);
        auto left = [&](size_t i) { return work[i]->n - work[i]->next_point - take[i]; };
        for (size_t i = 0; i < work.size(); ++i) {
            const int64_t need = left(i) * work[i]->samples_per_point();
            if (need <= samples_per_launch && need <= budget) {
                take[i] = left(i);
                budget -= need;
            }
        }
        for (size_t i = 0; i < work.size() && budget > 0; ++i) {
            const int64_t spp = work[i]->samples_per_point();
            const int64_t pts = std::min(left(i), budget / spp);
            take[i] += pts;
            budget -= pts * spp;
        }
        if (std::all_of(take.begin(), take.end(), [](int64_t x) { return x == 0; }))
            take[0] = 1;   // one point can exceed a tiny launch budget: make progress
        int nt = 0;
        for (size_t i = 0; i < work.size(); ++i) {
            if (take[i] == 0) continue;
            Request* r = work[i];
            fipt_shading out;
            out.planes = reinterpret_cast<float*>(pool + r->pool_off);
            out.stride = r->n;
            BakeLaunch b = make_bake_launch(r->scene, &r->pts, &r->params, &out);
            const int64_t p0 = r->next_point;
            b.pts += p0;
            b.ptri += p0;
            b.out += p0;
            b.n = take[i];
            b.p_offset = p0;
            s.host[nt].job = b;
            s.host[nt].first = 0;
            s.recs.push_back({r->ticket, take[i]});
            r->next_point += take[i];
            ++nt;
        }
        int64_t acc = 0;
        for (int i = 0; i < nt; ++i) {
            s.host[i].first = acc;
            acc += s.host[i].job.n;
        }
        stats.tiles += nt;
        for (int i = 0; i < nt; ++i) {
            const Request& r = reqs[s.recs[i].ticket];
            stats.samples += s.recs[i].count * r.samples_per_point();
        }
        return nt;
    }

    void complete(Slot& s) {
        const int64_t t = now_us();
        for (const TileRec& tr : s.recs) {
            Request& r = reqs[tr.ticket];
            r.done_points += tr.count;
            if (r.done_points == r.n && r.state == ADMITTED) {
                r.state = DONE;
                r.t_done = t;
                ++stats.completed;
                active.erase(std::find(active.begin(), active.end(), r.ticket));
            }
        }
        s.recs.clear();
        s.busy = false;
    }

    void run() {
        (void)hipSetDevice(device);
        while (true) {
            bool progressed = false;
            // retire finished launches
            for (Slot& s : slots) {
                if (!s.busy) continue;
                hipError_t q = hipEventQuery(s.done);
                if (q == hipSuccess) {
                    std::lock_guard<std::mutex> lk(mu);
                    complete(s);
                    progressed = true;
                    cv.notify_all();
                } else if (q != hipErrorNotReady) {
                    std::lock_guard<std::mutex> lk(mu);
                    worker_error = hipGetErrorString(q);
                    stop = true;
                    cv.notify_all();
                    return;
                }
            }
            // admit and launch into free slots
            for (Slot& s : slots) {
                if (s.busy) continue;
                int nt;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    admit();
                    nt = build(s);
                    if (nt > 0) {
                        s.busy = true;
                        ++stats.launches;
                    }
                }
                if (nt == 0) break;
                hipError_t e = hipMemcpyAsync(s.dev, s.host, sizeof(TileDesc) * nt,
                                              hipMemcpyHostToDevice, s.stream);
                if (e == hipSuccess)
                    e = hipMemsetAsync(s.counter, 0, sizeof(int32_t) * kXcdCount, s.stream);
                int rc = e == hipSuccess ? launch_bake_tiles(s.dev, nt, s.counter, grid, s.stream)
                                         : FIPT_EHIP;
                if (rc == FIPT_OK) e = hipEventRecord(s.done, s.stream);
                if (e != hipSuccess || rc != FIPT_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    worker_error = e != hipSuccess ? hipGetErrorString(e) : "tile launch failed";
                    stop = true;
                    cv.notify_all();
                    return;
                }
                progressed = true;
            }
            {
                std::unique_lock<std::mutex> lk(mu);
                const bool idle = !slots[0].busy && !slots[1].busy;
                if (stop && idle && active.empty()) return;
                if (!progressed) {
                    if (idle && active.empty() && queue.empty())
                        cv.wait_for(lk, std::chrono::milliseconds(5));
                    else
                        cv.wait_for(lk, std::chrono::microseconds(100));
                }
            }
        }
    }
};

namespace {

void server_free(fipt_server s) {
    for (Slot& sl : s->slots) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.counter) (void)hipFree(sl.counter);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->pool) (void)hipFree(s->pool);
    delete s;
}

}  // namespace

extern "C" {

int fipt_server_create(int32_t device, int64_t pool_bytes, int32_t max_inflight,
                       int64_t samples_per_launch, fipt_server* out) {
    clear_error();
    if (!out) return fail(FIPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (pool_bytes < (1 << 20)) return fail(FIPT_EINVAL, "pool_bytes must be >= 1 MiB");
    if (max_inflight < 1 || max_inflight > 4096) return fail(FIPT_EINVAL, "max_inflight must be in [1, 4096]");
    if (samples_per_launch < 64) return fail(FIPT_EINVAL, "samples_per_launch must be >= 64");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(FIPT_EINVAL, "device %d not available", device);
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) return fail(FIPT_EHIP, "hipSetDevice failed");
    fipt_server s = new fipt_server_s();
    s->device = device;
    s->pool_bytes = pool_bytes;
    s->max_inflight = max_inflight;
    s->samples_per_launch = samples_per_launch;
    s->grid = bake_tiles_grid_hint();
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&s->pool), pool_bytes);
    for (int i = 0; i < kSlots && e == hipSuccess; ++i) {
        Slot& sl = s->slots[i];
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&sl.host), sizeof(TileDesc) * max_inflight, 0);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.dev), sizeof(TileDesc) * max_inflight);
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void**>(&sl.counter), sizeof(int32_t) * kXcdCount);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        server_free(s);
        if (prev >= 0) (void)hipSetDevice(prev);
        return fail(e == hipErrorOutOfMemory ? FIPT_ENOMEM : FIPT_EHIP, "server set-up: %s",
                    hipGetErrorString(e));
    }
    s->free_list[0] = pool_bytes / kAlign * kAlign;
    s->worker = std::thread([s] { s->run(); });
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = s;
    return FIPT_OK;
}

int fipt_server_submit(fipt_server srv, fipt_scene sc, const fipt_points* pts,
                       const fipt_bake_params* p, uint64_t* ticket) {
    clear_error();
    if (!srv || !sc || !pts || !ticket) return fail(FIPT_EINVAL, "NULL argument");
    if (!pts->planes || !pts->tri || pts->n < 1 || pts->stride < pts->n)
        return fail(FIPT_EINVAL, "invalid points");
    int rc = check_bake_params(p);
    if (rc) return rc;
    if (sc->device != srv->device) return fail(FIPT_EINVAL, "scene and server are on different devices");
    if (sc->cache_kind == FIPT_CACHE_VOXEL)
        return fail(FIPT_EINVAL, "serving bakes scenes with a per-triangle or per-vertex cache");
    Request r;
    r.scene = sc;
    r.pts = *pts;
    r.params = *p;
    r.n = pts->n;
    r.planes = 3 + 6 * (int64_t)p->n_levels;
    r.bytes = r.planes * r.n * (int64_t)sizeof(float);
    if (r.bytes > srv->pool_bytes)
        return fail(FIPT_EINVAL, "request needs %lld bytes, pool has %lld", (long long)r.bytes,
                    (long long)srv->pool_bytes);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(FIPT_ECANCELED, "server is stopping");
    r.ticket = srv->next_ticket++;
    r.t_submit = srv->now_us();
    sc->refs.fetch_add(1);
    srv->reqs[r.ticket] = r;
    srv->queue.push_back(r.ticket);
    *ticket = r.ticket;
    srv->cv.notify_all();
    return FIPT_OK;
}

int fipt_server_poll(fipt_server srv, uint64_t ticket) {
    clear_error();
    if (!srv) return fail(FIPT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(FIPT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!srv->worker_error.empty()) return fail(FIPT_EHIP, "server worker failed: %s", srv->worker_error.c_str());
    if (it->second.state == DONE) return FIPT_OK;
    if (it->second.state == CANCELED) return FIPT_ECANCELED;
    return FIPT_EAGAIN;
}

int fipt_server_wait(fipt_server srv, uint64_t ticket, int64_t timeout_us) {
    clear_error();
    if (!srv) return fail(FIPT_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us);
    while (true) {
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return fail(FIPT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        if (!srv->worker_error.empty()) return fail(FIPT_EHIP, "server worker failed: %s", srv->worker_error.c_str());
        if (it->second.state == DONE) return FIPT_OK;
        if (it->second.state == CANCELED) return FIPT_ECANCELED;
        if (timeout_us < 0) {
            srv->cv.wait_for(lk, std::chrono::milliseconds(50));
        } else {
            if (std::chrono::steady_clock::now() >= deadline) return FIPT_EAGAIN;
            srv->cv.wait_until(lk, deadline);
        }
    }
}

int fipt_server_result(fipt_server srv, uint64_t ticket, fipt_shading* out, int64_t* t_submit_us,
                       int64_t* t_admit_us, int64_t* t_done_us) {
    clear_error();
    if (!srv || !out) return fail(FIPT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(FIPT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Request& r = it->second;
    if (r.state != DONE) return r.state == CANCELED ? FIPT_ECANCELED : FIPT_EAGAIN;
    out->planes = reinterpret_cast<float*>(srv->pool + r.pool_off);
    out->stride = r.n;
    if (t_submit_us) *t_submit_us = r.t_submit;
    if (t_admit_us) *t_admit_us = r.t_admit;
    if (t_done_us) *t_done_us = r.t_done;
    return FIPT_OK;
}

int fipt_server_release(fipt_server srv, uint64_t ticket) {
    clear_error();
    if (!srv) return fail(FIPT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(FIPT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = it->second;
    if (r.state == QUEUED || r.state == ADMITTED)
        return fail(FIPT_EBUSY, "request %llu has not completed", (unsigned long long)ticket);
    if (r.state == DONE) srv->pool_free(r.pool_off, r.bytes);
    r.scene->refs.fetch_sub(1);
    srv->reqs.erase(it);
    srv->cv.notify_all();
    return FIPT_OK;
}

int fipt_server_cancel(fipt_server srv, uint64_t ticket) {
    clear_error();
    if (!srv) return fail(FIPT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(FIPT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request& r = it->second;
    if (r.state != QUEUED) return fail(FIPT_EBUSY, "request %llu already admitted", (unsigned long long)ticket);
    r.state = CANCELED;
    srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), ticket));
    srv->cv.notify_all();
    return FIPT_OK;
}

int fipt_server_stats_get(fipt_server srv, fipt_server_stats* out) {
    clear_error();
    if (!srv || !out) return fail(FIPT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->pool_in_use = srv->pool_in_use;
    out->queued = (int64_t)srv->queue.size();
    out->inflight = (int64_t)srv->active.size();
    return FIPT_OK;
}

int fipt_server_destroy(fipt_server srv) {
    clear_error();
    if (!srv) return FIPT_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (uint64_t t : srv->queue) srv->reqs[t].state = CANCELED;
        srv->queue.clear();
        srv->cv.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (Slot& sl : srv->slots) (void)hipStreamSynchronize(sl.stream);
    for (auto& kv : srv->reqs) kv.second.scene->refs.fetch_sub(1);
    server_free(srv);
    if (prev >= 0) (void)hipSetDevice(prev);
    return FIPT_OK;
}

}  // extern "C"
