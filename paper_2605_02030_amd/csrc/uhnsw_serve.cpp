// Serving form: continuous batching over the resident index.
//
// Queries are admitted into slots as they arrive (uhnsw_serve_submit copies
// the query; no slot free -> UHNSW_EBUSY). A dispatcher thread launches the
// pending queries as a micro-batch on the first idle stream, so a batch that
// arrives while others run goes to the device at once and overlaps with
// them; it polls the batches' completion events and moves finished rows to
// the result queue, freeing their slots. Each batch is one fused launch
// (walk + verification per wave), so a query's result does not depend on
// the batch it rode in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "uhnsw.h"
#include "uhnsw_guard.h"
#include "uhnsw_internal.h"

namespace {

double now_us(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
}

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    double t_launch = 0;
    std::vector<int> slots;
    // pinned host staging
    float *h_q = nullptr, *h_p = nullptr, *h_dist = nullptr;
    int32_t *h_k = nullptr, *h_ef = nullptr;
    int64_t *h_ids = nullptr;
    uhnsw_stats *h_st = nullptr;
    // device buffers
    float *d_q = nullptr, *d_p = nullptr, *d_dist = nullptr;
    int32_t *d_k = nullptr, *d_ef = nullptr;
    int64_t *d_ids = nullptr;
    uhnsw_stats *d_st = nullptr;
};

struct Slot {
    uint64_t tag;
    float p;
    int32_t k, ef;
    double t_submit;
};

}  // namespace

struct uhnsw_server {
    uhnsw_ctx *ctx = nullptr;
    uhnsw_serve_config cfg{};
    int d = 0, device = 0, max_batch = 0, slots_total = 0;
    int variant = 0;  // of the context's index (its p range)
    std::chrono::steady_clock::time_point t0;
    std::vector<float> slot_q;  // slots_total x d
    std::vector<Slot> slot;
    std::vector<int> free_slots;
    std::deque<int> pending;
    std::deque<uhnsw_serve_result> done;
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    std::atomic<bool> stop{false};
    std::atomic<int> error{0};
    std::string err;
    int64_t launched_batches = 0, completed = 0, max_overlap = 0;
    int waves_per_cu = 0, cus = 0;  // the fused kernel's residency under the LDS plan
};

namespace {

void free_lane(Lane &L) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.done) (void)hipEventDestroy(L.done);
    void *hp[] = {L.h_q, L.h_p, L.h_dist, L.h_k, L.h_ef, L.h_ids, L.h_st};
    for (void *p : hp)
        if (p) (void)hipHostFree(p);
    void *dp[] = {L.d_q, L.d_p, L.d_dist, L.d_k, L.d_ef, L.d_ids, L.d_st};
    for (void *p : dp)
        if (p) (void)hipFree(p);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L = Lane();
}

hipError_t alloc_lane(Lane &L, int B, int d, int kmax) {
    hipError_t e;
#define A_(call)                          \
    if ((e = (call)) != hipSuccess) return e;
    A_(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    A_(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    A_(hipHostMalloc((void **)&L.h_q, sizeof(float) * B * d, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_p, sizeof(float) * B, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_k, sizeof(int32_t) * B, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_ef, sizeof(int32_t) * B, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_ids, sizeof(int64_t) * B * kmax, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_dist, sizeof(float) * B * kmax, hipHostMallocDefault));
    A_(hipHostMalloc((void **)&L.h_st, sizeof(uhnsw_stats) * B, hipHostMallocDefault));
    A_(hipMalloc((void **)&L.d_q, sizeof(float) * B * d));
    A_(hipMalloc((void **)&L.d_p, sizeof(float) * B));
    A_(hipMalloc((void **)&L.d_k, sizeof(int32_t) * B));
    A_(hipMalloc((void **)&L.d_ef, sizeof(int32_t) * B));
    A_(hipMalloc((void **)&L.d_ids, sizeof(int64_t) * B * kmax));
    A_(hipMalloc((void **)&L.d_dist, sizeof(float) * B * kmax));
    A_(hipMalloc((void **)&L.d_st, sizeof(uhnsw_stats) * B));
#undef A_
    return hipSuccess;
}

size_t lane_device_bytes(int B, int d, int kmax) {
    return (size_t)B * (d * 4 + 12 + kmax * 12 + sizeof(uhnsw_stats));
}

// Harvest finished batches (under the lock). Returns how many finished.
int harvest(uhnsw_server *S) {
    int n = 0;
    for (auto &L : S->lanes) {
        if (!L.busy) continue;
        hipError_t q = hipEventQuery(L.done);
        if (q == hipErrorNotReady) continue;
        const double t = now_us(S->t0);
        const int kmax = S->cfg.k_max;
        for (size_t r = 0; r < L.slots.size(); ++r) {
            const int sl = L.slots[r];
            uhnsw_serve_result res;
            std::memset(&res, 0, sizeof res);
            res.tag = S->slot[sl].tag;
            res.submit_us = S->slot[sl].t_submit;
            res.launch_us = L.t_launch;
            res.done_us = t;
            if (q != hipSuccess) {
                res.status = UHNSW_EDEVICE;
            } else {
                res.stats = L.h_st[r];
                res.status = (res.stats.flags & UHNSW_QBAD) ? UHNSW_EINVAL : UHNSW_OK;
                const int k = S->slot[sl].k;
                int nr = 0;
                for (int j = 0; j < k; ++j) {
                    res.ids[j] = L.h_ids[r * kmax + j];
                    res.dists[j] = L.h_dist[r * kmax + j];
                    nr += res.ids[j] >= 0;
                }
                for (int j = k; j < UHNSW_KMAX; ++j) {
                    res.ids[j] = -1;
                    res.dists[j] = INFINITY;
                }
                res.nres = nr;
            }
            S->done.push_back(res);
            S->free_slots.push_back(sl);
        }
        S->completed += (int64_t)L.slots.size();
        L.slots.clear();
        L.busy = false;
        if (q != hipSuccess && q != hipErrorNotReady) S->error = UHNSW_EDEVICE;
        ++n;
    }
    return n;
}

// Launch pending queries on an idle lane (under the lock, HIP calls made
// with the lock held are asynchronous enqueues only).
bool launch_pending(uhnsw_server *S) {
    if (S->pending.empty()) return false;
    Lane *L = nullptr;
    for (auto &l : S->lanes)
        if (!l.busy) {
            L = &l;
            break;
        }
    if (!L) return false;
    const int d = S->d, kmax = S->cfg.k_max;
    int B = 0;
    while (!S->pending.empty() && B < S->max_batch) {
        const int sl = S->pending.front();
        S->pending.pop_front();
        std::memcpy(L->h_q + (size_t)B * d, &S->slot_q[(size_t)sl * d], sizeof(float) * d);
        L->h_p[B] = S->slot[sl].p;
        L->h_k[B] = S->slot[sl].k;
        L->h_ef[B] = S->slot[sl].ef;
        L->slots.push_back(sl);
        ++B;
    }
    hipStream_t s = L->stream;
    hipError_t e = hipSuccess;
    if ((e = hipMemcpyAsync(L->d_q, L->h_q, sizeof(float) * B * d, hipMemcpyHostToDevice, s)) == hipSuccess &&
        (e = hipMemcpyAsync(L->d_p, L->h_p, sizeof(float) * B, hipMemcpyHostToDevice, s)) == hipSuccess &&
        (e = hipMemcpyAsync(L->d_k, L->h_k, sizeof(int32_t) * B, hipMemcpyHostToDevice, s)) == hipSuccess &&
        (e = hipMemcpyAsync(L->d_ef, L->h_ef, sizeof(int32_t) * B, hipMemcpyHostToDevice, s)) == hipSuccess) {
        uhnsw_params prm = S->cfg.params;
        prm.fused = 1;
        prm.persistent = 0;  // each batch is one wave per query; no shared work counter
        prm.graph = 0;
        prm.timing = 0;
        int rc = uhnsw_search_device(S->ctx, L->d_q, B, L->d_p, L->d_k, L->d_ef, kmax, S->cfg.ef_max, &prm, kmax,
                                     L->d_ids, L->d_dist, L->d_st, nullptr, nullptr, 0, s);
        if (rc != UHNSW_OK) {
            S->error = rc;
            S->err = uhnsw_last_error(S->ctx);
        }
        if (rc == UHNSW_OK &&
            (e = hipMemcpyAsync(L->h_ids, L->d_ids, sizeof(int64_t) * B * kmax, hipMemcpyDeviceToHost, s)) ==
                hipSuccess &&
            (e = hipMemcpyAsync(L->h_dist, L->d_dist, sizeof(float) * B * kmax, hipMemcpyDeviceToHost, s)) ==
                hipSuccess &&
            (e = hipMemcpyAsync(L->h_st, L->d_st, sizeof(uhnsw_stats) * B, hipMemcpyDeviceToHost, s)) ==
                hipSuccess)
            e = hipEventRecord(L->done, s);
    }
    if (e != hipSuccess && !S->error) {
        S->error = UHNSW_EDEVICE;
        S->err = std::string("serving launch: ") + hipGetErrorString(e);
    }
    L->busy = true;
    L->t_launch = now_us(S->t0);
    ++S->launched_batches;
    int64_t ov = 0;
    for (auto &l : S->lanes) ov += l.busy;
    S->max_overlap = std::max(S->max_overlap, ov);
    return true;
}

void dispatch_loop(uhnsw_server *S, std::unique_lock<std::mutex> &lk);

// The server's thread. A C++ exception in its loop (a result queue that
// cannot grow) stops dispatching and is reported as UHNSW_ENOMEM by the
// next submit or poll; batches already launched are synchronised by stop.
void dispatcher(uhnsw_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    try {
        dispatch_loop(S, lk);
    } catch (const std::exception &e) {
        S->error = UHNSW_ENOMEM;
        try {
            S->err = std::string("serving dispatcher: ") + e.what();
        } catch (...) {
        }
    } catch (...) {
        S->error = UHNSW_ENOMEM;
    }
}

void dispatch_loop(uhnsw_server *S, std::unique_lock<std::mutex> &lk) {
    for (;;) {
        bool any_busy = false;
        for (auto &l : S->lanes) any_busy |= l.busy;
        if (S->stop && S->pending.empty() && !any_busy) break;
        const int fin = harvest(S);
        bool launched = false;
        while (launch_pending(S)) launched = true;
        if (fin) S->cv.notify_all();
        if (launched || fin) continue;
        any_busy = false;
        for (auto &l : S->lanes) any_busy |= l.busy;
        if (any_busy) {
            // Batches in flight: check their events again after a short wait.
            // The wait releases the lock, so submitters and pollers are not
            // starved by this loop; a submit that finds an idle lane ends it.
            S->cv.wait_for(lk, std::chrono::microseconds(20), [&] {
                if (S->stop.load()) return true;
                if (S->pending.empty()) return false;
                for (auto &l : S->lanes)
                    if (!l.busy) return true;
                return false;
            });
        } else {
            S->cv.wait(lk, [&] { return S->stop.load() || !S->pending.empty(); });
        }
    }
}

// A failure message from the caller's thread: kept with the server (the
// dispatcher may be using the context) and handed to the context by stop.
void note_error(uhnsw_server *S, const char *msg) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = msg;
}

}  // namespace

extern "C" {

void uhnsw_serve_default_config(uhnsw_serve_config *c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->k_max = 100;
    c->ef_max = 256;
    uhnsw_default_params(&c->params);
}

static int serve_start_body(uhnsw_ctx *ctx, const uhnsw_serve_config *cfg, uhnsw_server **out) {
    if (!ctx || !cfg || !out) return UHNSW_EINVAL;
    *out = nullptr;
    int32_t g, v;
    if (uhnsw_get_layout(ctx, &g, &v) != UHNSW_OK) return UHNSW_ESTATE;
    if (cfg->k_max < 1 || cfg->k_max > UHNSW_KMAX || cfg->ef_max < cfg->k_max || cfg->ef_max > UHNSW_EFMAX)
        return UHNSW_EINVAL;
    if (cfg->streams < 0 || cfg->streams > 16 || cfg->max_batch < 0 || cfg->max_inflight < 0 || cfg->hbm_budget < 0)
        return UHNSW_EINVAL;
    int32_t cus = 0, khz = 0;
    if (uhnsw_device_info(ctx, &cus, &khz) != UHNSW_OK) return UHNSW_EDEVICE;
    auto *S = new (std::nothrow) uhnsw_server();
    if (!S) return UHNSW_ENOMEM;
    S->ctx = ctx;
    S->cfg = *cfg;
    S->d = uhnsw::ctx_dim(ctx);
    S->variant = uhnsw::ctx_variant(ctx);
    S->device = uhnsw::ctx_device(ctx);
    // Two lanes by default: one batch runs while the next one gathers
    // arrivals. HIP gives a process four hardware queues by default and the
    // context's own streams hold some of them; more lanes than free queues
    // serialise behind each other and measured slower.
    const int streams = cfg->streams ? cfg->streams : 2;
    // LDS budget: a query occupies one wave of the fused kernel; admit at
    // most as many queries as the device keeps resident under the launch's
    // LDS plan (W, visited cache and scratch per wave, from k_max, ef_max and
    // the cache size) and register use, as the occupancy query reports
    int wpc = 0;
    {
        uhnsw_params prm = cfg->params;
        prm.persistent = 0;
        const int rc = uhnsw::ctx_resident_waves(ctx, cfg->k_max, cfg->ef_max, &prm, &wpc);
        if (rc != UHNSW_OK) {
            delete S;
            return rc;
        }
    }
    S->waves_per_cu = wpc;
    S->cus = cus;
    const int wave_capacity = std::max(1, cus * wpc);
    int slots = cfg->max_inflight ? cfg->max_inflight : wave_capacity;
    int B = cfg->max_batch ? cfg->max_batch : std::max(64, wave_capacity / streams);
    // HBM budget: the per-lane device buffers must fit; shrink the batch
    // until they do, refuse when even one query per lane does not
    if (cfg->hbm_budget > 0) {
        while (B > 1 && lane_device_bytes(B, S->d, cfg->k_max) * (size_t)streams > (size_t)cfg->hbm_budget) B /= 2;
        if (lane_device_bytes(B, S->d, cfg->k_max) * (size_t)streams > (size_t)cfg->hbm_budget) {
            delete S;
            return UHNSW_EBUSY;
        }
    }
    S->max_batch = B;
    S->slots_total = slots;
    try {  // host containers and the dispatcher thread; on failure nothing is kept
        S->slot_q.assign((size_t)slots * S->d, 0.f);
        S->slot.resize(slots);
        for (int i = slots - 1; i >= 0; --i) S->free_slots.push_back(i);
        S->lanes.resize(streams);
        (void)hipSetDevice(S->device);
        for (auto &L : S->lanes)
            if (alloc_lane(L, B, S->d, cfg->k_max) != hipSuccess) {
                for (auto &l : S->lanes) free_lane(l);
                delete S;
                return UHNSW_ENOMEM;
            }
        S->t0 = std::chrono::steady_clock::now();
        uhnsw::ctx_servers(ctx, +1);  // the index may not be replaced while this server runs
        try {
            S->th = std::thread(dispatcher, S);
        } catch (...) {
            uhnsw::ctx_servers(ctx, -1);
            throw;
        }
    } catch (...) {
        for (auto &l : S->lanes) free_lane(l);
        delete S;
        throw;
    }
    *out = S;
    return UHNSW_OK;
}

int uhnsw_serve_start(uhnsw_ctx *ctx, const uhnsw_serve_config *cfg, uhnsw_server **out) {
    const auto body = [&] { return serve_start_body(ctx, cfg, out); };
    return uhnsw::no_throw("uhnsw_serve_start", body, [&](const char *w) {
        if (ctx) uhnsw::ctx_set_error(ctx, w);
    });
}

static int serve_submit_body(uhnsw_server *S, const float *q, float p, int32_t k, int32_t ef, uint64_t tag) {
    if (!S || !q) return UHNSW_EINVAL;
    if (!uhnsw::p_in_range(S->variant, p) || k < 1 || k > S->cfg.k_max || ef < k || ef > S->cfg.ef_max)
        return UHNSW_EINVAL;
    for (int j = 0; j < S->d; ++j)
        if (!std::isfinite(q[j])) return UHNSW_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        const int e = S->error.load();
        if (e) return e;
        if (S->stop) return UHNSW_ESTATE;
        if (S->free_slots.empty()) return UHNSW_EBUSY;
        const int sl = S->free_slots.back();
        S->free_slots.pop_back();
        std::memcpy(&S->slot_q[(size_t)sl * S->d], q, sizeof(float) * S->d);
        S->slot[sl] = Slot{tag, p, k, ef, now_us(S->t0)};
        S->pending.push_back(sl);
    }
    S->cv.notify_all();
    return UHNSW_OK;
}

int uhnsw_serve_submit(uhnsw_server *S, const float *q, float p, int32_t k, int32_t ef, uint64_t tag) {
    const auto body = [&] { return serve_submit_body(S, q, p, k, ef, tag); };
    return uhnsw::no_throw("uhnsw_serve_submit", body, [&](const char *w) { if (S) note_error(S, w); });
}

static int serve_poll_body(uhnsw_server *S, uhnsw_serve_result *out, int32_t max, int32_t *n_out) {
    if (!S || !n_out || (max > 0 && !out)) return UHNSW_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    int n = 0;
    while (n < max && !S->done.empty()) {
        out[n++] = S->done.front();
        S->done.pop_front();
    }
    *n_out = n;
    const int e = S->error.load();
    return e ? e : UHNSW_OK;
}

int uhnsw_serve_poll(uhnsw_server *S, uhnsw_serve_result *out, int32_t max, int32_t *n_out) {
    const auto body = [&] { return serve_poll_body(S, out, max, n_out); };
    return uhnsw::no_throw("uhnsw_serve_poll", body, [&](const char *w) { if (S) note_error(S, w); });
}

int uhnsw_serve_info(uhnsw_server *S, int64_t *info) {
    if (!S || !info) return UHNSW_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    info[0] = S->slots_total;
    info[1] = (int64_t)S->free_slots.size();
    info[2] = (int64_t)S->pending.size();
    info[3] = S->launched_batches;
    info[4] = S->completed;
    info[5] = S->max_overlap;
    info[6] = S->max_batch;
    info[7] = (int64_t)S->lanes.size();
    info[8] = S->waves_per_cu;
    info[9] = S->cus;
    return UHNSW_OK;
}

int uhnsw_serve_stop(uhnsw_server *S) {
    if (!S) return UHNSW_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    const int rc = S->error.load();
    for (auto &L : S->lanes) free_lane(L);
    if (!S->err.empty()) {  // the dispatcher has ended: the context is the caller's again
        try {
            uhnsw::ctx_set_error(S->ctx, S->err.c_str());
        } catch (...) {
        }
    }
    uhnsw::ctx_servers(S->ctx, -1);
    delete S;
    return rc;
}

static int serve_drive_body(uhnsw_server *S, int64_t n, const float *queries, const int32_t *qidx, const float *p,
                            const int32_t *k, const int32_t *ef, const double *arrival_us, int32_t out_k, int64_t *ids,
                            float *dists, uhnsw_stats *stats, double *times, int32_t *status) {
    if (!S || n < 0 || out_k < 1 || out_k > UHNSW_KMAX ||
        (n > 0 && (!queries || !p || !k || !ef || !arrival_us || !ids || !dists || !times || !status)))
        return UHNSW_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    const double off = now_us(S->t0);  // server clock at this call's time zero
    int64_t next = 0, got = 0;
    std::vector<uhnsw_serve_result> buf(256);
    while (got < n) {
        const double t = now_us(t0);
        while (next < n && arrival_us[next] <= t) {
            const int64_t row = qidx ? qidx[next] : next;
            const int rc = uhnsw_serve_submit(S, queries + (size_t)row * S->d, p[next], k[next], ef[next],
                                              (uint64_t)next);
            if (rc == UHNSW_EBUSY) break;  // wait for a slot; the arrival time still counts
            if (rc != UHNSW_OK) return rc;
            ++next;
        }
        int32_t m = 0;
        const int rc = uhnsw_serve_poll(S, buf.data(), (int32_t)buf.size(), &m);
        if (rc != UHNSW_OK) return rc;
        for (int i = 0; i < m; ++i) {
            const uhnsw_serve_result &r = buf[i];
            const int64_t id = (int64_t)r.tag;
            std::memcpy(ids + id * out_k, r.ids, sizeof(int64_t) * out_k);
            std::memcpy(dists + id * out_k, r.dists, sizeof(float) * out_k);
            if (stats) stats[id] = r.stats;
            // times in the driver's clock; latency counts from the scheduled arrival
            times[3 * id] = arrival_us[id];
            times[3 * id + 1] = r.launch_us - off;
            times[3 * id + 2] = r.done_us - off;
            status[id] = r.status;
            ++got;
        }
        if (m == 0) std::this_thread::yield();
    }
    return UHNSW_OK;
}

int uhnsw_serve_drive(uhnsw_server *S, int64_t n, const float *queries, const int32_t *qidx, const float *p,
                      const int32_t *k, const int32_t *ef, const double *arrival_us, int32_t out_k, int64_t *ids,
                      float *dists, uhnsw_stats *stats, double *times, int32_t *status) {
    const auto body = [&] {
        return serve_drive_body(S, n, queries, qidx, p, k, ef, arrival_us, out_k, ids, dists, stats, times, status);
    };
    return uhnsw::no_throw("uhnsw_serve_drive", body, [&](const char *w) { if (S) note_error(S, w); });
}

}  // extern "C"
