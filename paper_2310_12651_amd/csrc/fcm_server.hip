// Request server for fast-FCM mobility evaluations (include/fcm_server.h).
//
// A worker thread owns the device work: it admits queued requests whenever one
// of its stream slots is free and the plan the request needs fits the
// device-byte budget, launches the request's evaluation on that slot's stream
// (each fcm_mobility call is stream-ordered and allocation-free), records a
// completion event, and retires the slot when the event has fired.  Requests
// are taken in arrival order, but one that has to wait for memory held by
// running requests is passed by later ones that fit (at most kMaxBypass times;
// then admission holds for it, so large requests are not starved).
// Plans are cached and re-bound to later requests with the same grid (all three
// axes: a request may name a rectangular box), support and precision, so grids,
// twiddles and sort/cell buffers stay resident;
// idle plans are freed least-recently-used first when room is needed.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include <string.h>

#include "../../include/fcm_server.h"
#include "fcm_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct CachedPlan {
    fcm_plan_impl* P = nullptr;
    int64_t bytes = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

// later requests admitted ahead of one that waits for memory, at most
constexpr int kMaxBypass = 32;

struct Req {
    fcm_request r;
    double L3[3] = {0.0, 0.0, 0.0};   // box sides (all r.L for a cubic request)
    int g3[3] = {0, 0, 0};            // grid points per axis
    int64_t ticket = 0;
    int state = 0;   // 0 queued, 1 running, 2 done
    int status = FCM_OK;
    int bypassed = 0;            // later requests admitted ahead of this one
    bool waited = false;         // a thread is in (or has been through) fcm_server_wait
    hipEvent_t after = nullptr;  // recorded on the caller's stream at submit, or null
    Clock::time_point t_submit, t_launch, t_done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int* nonfinite = nullptr;    // pinned host word: the plan's non-finite flag after the call
    Req* req = nullptr;
    CachedPlan* plan = nullptr;
    int64_t points = 0;          // grid points of the running request
};

}  // namespace

struct fcm_server_impl {
    fcm_server_options opt;
    int device = 0;
    std::mutex mu;
    std::condition_variable work_cv;   // wakes the worker
    std::condition_variable done_cv;   // wakes waiters
    std::deque<Req*> queue;
    std::unordered_map<int64_t, Req*> reqs;
    std::vector<Slot> slots;
    std::vector<CachedPlan*> cache;
    std::vector<hipEvent_t> free_events;   // for the caller-stream dependencies
    int64_t next_ticket = 1;
    int64_t budget = 0;
    uint64_t use_clock = 0;
    bool stopping = false;
    int inflight = 0;
    int64_t inflight_points = 0;   // grid points of the requests in flight
    fcm_server_stats stats;
    std::thread worker;

    void run();
    bool retire_locked();
    void release_event_locked(Req* r);
    bool admit_locked();
    CachedPlan* plan_for_locked(const fcm_plan_impl& d, int* status);
    void evict_one_locked();
};

namespace {

int64_t round_up_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// derive the plan scalars of a request on the box L3 with grid g3 (validation
// included, as fcm_plan_box)
int derive_request(const fcm_server_options& o, const fcm_request& r, const double L3[3], const int g3[3],
                   fcm_plan_impl* d) {
    fcm_options opt;
    fcm_options_default(&opt);
    opt.eta = r.eta > 0.0 ? r.eta : 1.0;
    opt.support = r.support;
    opt.precision = o.precision;
    opt.kahan = o.kahan;
    memset(d, 0, sizeof(*d));
    return fcm::plan_derive(d, r.N, L3, r.a, r.sigma_delta, g3, r.r_cut, &opt);
}

}  // namespace

void fcm_server_impl::evict_one_locked() {
    CachedPlan* victim = nullptr;
    size_t vi = 0;
    for (size_t i = 0; i < cache.size(); ++i) {
        CachedPlan* c = cache[i];
        if (!c->busy && (!victim || c->last_use < victim->last_use)) {
            victim = c;
            vi = i;
        }
    }
    if (!victim) return;
    cache.erase(cache.begin() + vi);
    stats.bytes_in_use -= victim->bytes;
    stats.plans_evicted++;
    fcm::plan_free(victim->P);
    delete victim;
}

CachedPlan* fcm_server_impl::plan_for_locked(const fcm_plan_impl& d, int* status) {
    *status = FCM_OK;
    CachedPlan* best = nullptr;
    for (CachedPlan* c : cache) {
        const fcm_plan_impl* P = c->P;
        if (c->busy || P->M != d.M || P->My != d.My || P->Mz != d.Mz || P->MG != d.MG ||
            P->precision != d.precision ||
            P->kahan != d.kahan || P->Ncap < d.N || P->cells_cap < d.ncells)
            continue;
        if (!best || P->Ncap < best->P->Ncap) best = c;
    }
    if (best) {
        *status = fcm::plan_rebind(best->P, &d);
        if (*status != FCM_OK) return nullptr;
        stats.plans_rebound++;
        return best;
    }
    const int64_t ncap = round_up_pow2(d.N);
    const int cellcap = (int)std::min<int64_t>(round_up_pow2(d.ncells), (int64_t)fcm::kMaxCellsPerAxis *
                                                                            fcm::kMaxCellsPerAxis *
                                                                            fcm::kMaxCellsPerAxis);
    const int g3[3] = {d.M, d.My, d.Mz};
    const int64_t bytes = fcm::plan_bytes(ncap, g3, d.precision, cellcap, d.nbins);
    if (bytes > budget) {
        *status = FCM_ENOMEM;
        return nullptr;
    }
    while (stats.bytes_in_use + bytes > budget) {
        const size_t before = cache.size();
        evict_one_locked();
        if (cache.size() == before) return nullptr;   // everything busy: wait for a slot
    }
    fcm_plan_impl* P = new (std::nothrow) fcm_plan_impl;
    if (!P) {
        *status = FCM_ENOMEM;
        return nullptr;
    }
    *P = d;
    P->grid = nullptr;   // plan_allocate fills every buffer pointer
    int st = fcm::plan_allocate(P, ncap, cellcap);
    if (st != FCM_OK) {
        fcm::plan_free(P);
        // device memory may be held by running requests: retry after they retire
        if (st == FCM_ENOMEM && inflight > 0) return nullptr;
        *status = st;
        return nullptr;
    }
    CachedPlan* c = new CachedPlan;
    c->P = P;
    c->bytes = bytes;
    cache.push_back(c);
    stats.plans_built++;
    stats.bytes_in_use += bytes;
    if (stats.bytes_in_use > stats.bytes_peak) stats.bytes_peak = stats.bytes_in_use;
    return c;
}

// retire every slot whose completion event has fired; true if any did
bool fcm_server_impl::retire_locked() {
    bool any = false;
    for (Slot& s : slots) {
        if (!s.req) continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        Req* r = s.req;
        r->t_done = Clock::now();
        if (q != hipSuccess)
            r->status = FCM_EDEVICE;
        else if (*s.nonfinite)
            r->status = FCM_ENONFINITE;   // a position was NaN or infinite
        release_event_locked(r);
        r->state = 2;
        if (r->status == FCM_OK)
            stats.completed++;
        else
            stats.failed++;
        s.plan->busy = false;
        s.plan->last_use = ++use_clock;
        s.req = nullptr;
        s.plan = nullptr;
        --inflight;
        inflight_points -= s.points;
        s.points = 0;
        any = true;
    }
    if (any) done_cv.notify_all();
    return any;
}

void fcm_server_impl::release_event_locked(Req* r) {
    if (r->after) {
        free_events.push_back(r->after);
        r->after = nullptr;
    }
}

// launch queued requests while slots and memory allow: in arrival order, past
// the ones that wait for memory held by running requests (each may be passed
// kMaxBypass times)
bool fcm_server_impl::admit_locked() {
    bool any = false;
    size_t i = 0;
    while (i < queue.size()) {
        Slot* free_slot = nullptr;
        for (Slot& s : slots)
            if (!s.req) {
                free_slot = &s;
                break;
            }
        if (!free_slot) break;
        Req* r = queue[i];
        fcm_plan_impl d;
        int st = derive_request(opt, r->r, r->L3, r->g3, &d);
        CachedPlan* c = nullptr;
        const int64_t pts = st == FCM_OK ? (int64_t)d.M * d.My * d.Mz : 0;
        // the grid points in flight stay within max_points (one request always runs)
        const bool crowded = st == FCM_OK && opt.max_points > 0 && inflight > 0 &&
                             inflight_points + pts > opt.max_points;
        if (st == FCM_OK && !crowded) c = plan_for_locked(d, &st);
        if (!c && st == FCM_OK) {        // needs room held by running requests
            if (r->bypassed >= kMaxBypass) break;   // admit nothing past it
            ++i;
            continue;
        }
        for (size_t j = 0; j < i; ++j) queue[j]->bypassed++;
        queue.erase(queue.begin() + (std::ptrdiff_t)i);
        if (!c) {
            r->status = st;
            r->state = 2;
            r->t_launch = r->t_done = Clock::now();
            release_event_locked(r);
            stats.failed++;
            done_cv.notify_all();
            any = true;
            continue;
        }
        c->busy = true;
        r->state = 1;
        r->t_launch = Clock::now();
        *free_slot->nonfinite = 0;
        hipStream_t ss = free_slot->stream;
        st = FCM_OK;
        if (r->after && hipStreamWaitEvent(ss, r->after, 0) != hipSuccess) st = FCM_EDEVICE;
        if (st == FCM_OK) st = fcm_mobility(c->P, r->r.pos, r->r.F, r->r.T, r->r.V, r->r.Omega, ss);
        // the plan's non-finite flag (raised by the hash of this call) to the
        // slot's host word, then cleared for the plan's next request
        if (st == FCM_OK &&
            (hipMemcpyAsync(free_slot->nonfinite, c->P->flag, sizeof(int), hipMemcpyDeviceToHost, ss) !=
                 hipSuccess ||
             fcm::launch_fill(c->P->flag, 1, 0, ss) != hipSuccess))
            st = FCM_EDEVICE;
        if (st == FCM_OK && hipEventRecord(free_slot->done, ss) != hipSuccess) st = FCM_EDEVICE;
        if (st != FCM_OK) {
            c->busy = false;
            r->status = st;
            r->state = 2;
            r->t_done = Clock::now();
            release_event_locked(r);
            stats.failed++;
            done_cv.notify_all();
        } else {
            free_slot->req = r;
            free_slot->plan = c;
            free_slot->points = pts;
            inflight_points += pts;
            ++inflight;
            if (inflight > stats.inflight_peak) stats.inflight_peak = inflight;
        }
        any = true;
    }
    return any;
}

void fcm_server_impl::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progress = retire_locked();
        progress = admit_locked() || progress;
        if (stopping && queue.empty() && inflight == 0) break;
        if (progress) continue;
        if (inflight > 0)
            work_cv.wait_for(lk, std::chrono::microseconds(20));
        else
            work_cv.wait(lk, [&] { return stopping || !queue.empty(); });
    }
}

namespace {

// validate a request on the box L3 with grid g3 and queue it
int submit_request(fcm_server_t s, const fcm_request* req, const double L3[3], const int g3[3],
                   int64_t* ticket) {
    if (!s || !req || !ticket || !req->pos || !req->F || !req->V) return FCM_EINVAL;
    fcm_plan_impl d;
    const int st = derive_request(s->opt, *req, L3, g3, &d);
    if (st != FCM_OK) return st;
    Req* r = new (std::nothrow) Req;
    if (!r) return FCM_ENOMEM;
    r->r = *req;
    for (int k = 0; k < 3; ++k) {
        r->L3[k] = L3[k];
        r->g3[k] = g3[k];
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete r;
            return FCM_EINVAL;
        }
        if ((int)s->queue.size() >= s->opt.max_queue) {
            delete r;
            return FCM_EBUSY;
        }
        if (req->after_stream) {
            // the request runs after the work the caller's stream holds now
            hipEvent_t ev = nullptr;
            if (!s->free_events.empty()) {
                ev = s->free_events.back();
                s->free_events.pop_back();
            } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                delete r;
                return FCM_EDEVICE;
            }
            if (hipEventRecord(ev, (hipStream_t)req->after_stream) != hipSuccess) {
                s->free_events.push_back(ev);
                delete r;
                return FCM_EDEVICE;
            }
            r->after = ev;
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
        s->stats.submitted++;
        *ticket = r->ticket;
    }
    s->work_cv.notify_one();
    return FCM_OK;
}

}  // namespace

extern "C" {

int fcm_server_options_default(fcm_server_options* o) {
    if (!o) return FCM_EINVAL;
    o->max_bytes = 0;
    o->slots = 8;
    o->precision = FCM_FP32_BULK;
    o->kahan = 0;
    o->max_queue = 4096;
    o->max_points = 0;
    return FCM_OK;
}

int fcm_server_create(fcm_server_t* out, const fcm_server_options* opt_in) {
    if (!out) return FCM_EINVAL;
    *out = nullptr;
    fcm_server_options o;
    fcm_server_options_default(&o);
    if (opt_in) o = *opt_in;
    if (o.slots < 1 || o.slots > 64 || o.max_queue < 1 || o.max_bytes < 0 || o.max_points < 0)
        return FCM_EINVAL;
    if (o.precision != FCM_FP64 && o.precision != FCM_FP32_BULK) return FCM_EINVAL;
    if (o.kahan < 0 || o.kahan > 2) return FCM_EINVAL;
    fcm_server_impl* s = new (std::nothrow) fcm_server_impl;
    if (!s) return FCM_ENOMEM;
    s->opt = o;
    memset(&s->stats, 0, sizeof(s->stats));
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FCM_EDEVICE;
    }
    s->budget = o.max_bytes;
    if (s->budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return FCM_EDEVICE;
        }
        s->budget = (int64_t)(0.8 * (double)fr);
    }
    s->slots.resize(o.slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.nonfinite, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            for (Slot& x : s->slots) {
                if (x.stream) (void)hipStreamDestroy(x.stream);
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.nonfinite) (void)hipHostFree(x.nonfinite);
            }
            delete s;
            return FCM_EDEVICE;
        }
        *sl.nonfinite = 0;
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return FCM_OK;
}

int fcm_server_submit(fcm_server_t s, const fcm_request* req, int64_t* ticket) {
    if (!req) return FCM_EINVAL;
    const double L3[3] = {req->L, req->L, req->L};
    const int g3[3] = {req->grid, req->grid, req->grid};
    return submit_request(s, req, L3, g3, ticket);
}

int fcm_server_submit_box(fcm_server_t s, const fcm_request* req, const double L[3], const int grid[3],
                          int64_t* ticket) {
    if (!L || !grid) return FCM_EINVAL;
    return submit_request(s, req, L, grid, ticket);
}

int fcm_server_poll(fcm_server_t s, int64_t ticket, int* state) {
    if (!s || !state) return FCM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FCM_EINVAL;
    *state = it->second->state;
    return it->second->state == 2 ? it->second->status : FCM_OK;
}

int fcm_server_wait(fcm_server_t s, int64_t ticket, double* queue_ms, double* run_ms) {
    if (!s) return FCM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return FCM_EINVAL;
    Req* r = it->second;
    if (r->waited) return FCM_EINVAL;   // another thread waits for this ticket
    r->waited = true;
    s->work_cv.notify_one();
    s->done_cv.wait(lk, [&] { return r->state == 2; });
    if (queue_ms) *queue_ms = ms_between(r->t_submit, r->t_launch);
    if (run_ms) *run_ms = ms_between(r->t_launch, r->t_done);
    const int st = r->status;
    s->reqs.erase(it);
    delete r;
    return st;
}

int fcm_server_get_stats(fcm_server_t s, fcm_server_stats* out) {
    if (!s || !out) return FCM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return FCM_OK;
}

int fcm_server_destroy(fcm_server_t s) {
    if (!s) return FCM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->work_cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.nonfinite) (void)hipHostFree(sl.nonfinite);
    }
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    for (CachedPlan* c : s->cache) {
        fcm::plan_free(c->P);
        delete c;
    }
    for (auto& kv : s->reqs) {
        if (kv.second->after) (void)hipEventDestroy(kv.second->after);
        delete kv.second;
    }
    delete s;
    return FCM_OK;
}

}  // extern "C"
