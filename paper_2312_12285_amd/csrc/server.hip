// Request server: continuous batching of transforms on one device.
//
// Requests (a catalog already resident in device memory, its lmax and
// precision, and where to write a_lm and optionally C_l) are queued by
// ptalm_server_submit from any host thread.  A scheduler thread admits them
// into the server's device arena (their scratch block) and runs each as work
// items (server_core.h): launches of the transform over consecutive groups of
// its point slices, then one finishing launch (the second pass and the
// spectrum) once every chunk has completed.  Items go to execution slots (HIP
// streams of default priority) as they free up, shortest remaining work first,
// so a small request does not wait behind a large one, and requests that have
// waited long go first, so none starves.  Completion of an item is seen by
// polling an event.  Every request uses the work plan of the same call made
// alone; a chunk computes exactly the slice partials that call computes, so the
// result is bitwise the solo result.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ptalm.h"
#include "ptalm_internal.h"
#include "server_core.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// terms of work per chunk aimed at (~35 ms of the whole device in FP64)
constexpr double kChunkTerms = 2e11;
// a request waiting longer than this (from submission) goes before shorter work
constexpr double kAgeSeconds = 30.0;

struct Req {
    ptalm_request r;
    ptalm_request_stats st;
    ptalm::SlicedCall call{};
    int chunks = 0, slices_per_chunk = 1;
    bool planned = false, failed = false, done = false;
    std::string err;
};

struct InFlight {
    ptalm::serve::Item it;
    hipEvent_t ev;
};

}  // namespace

struct ptalm_server {
    int device = 0;
    void *arena = nullptr;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    ptalm::serve::Scheduler sched;
    std::unordered_map<int64_t, Req> reqs;
    std::vector<InFlight> inflight;
    std::vector<hipEvent_t> spare_events;
    int64_t next_ticket = 1;
    bool stop = false;
    std::thread th;

    ptalm_server(size_t bytes, int slots) : sched(bytes, slots, kAgeSeconds) {}
};

namespace {

thread_local std::string g_server_error;

int sfail(int code, const std::string &msg) {
    g_server_error = msg;
    return code;
}

// Scratch bytes of the call the server makes for this request (0 on bad arguments).
size_t footprint(const ptalm_request &r) {
    ptalm_opts o;
    memset(&o, 0, sizeof o);
    o.precision = r.precision;
    o.n_weights = 1;
    return ptalm_workspace_bytes(r.n, r.lmax, &o);
}

// Enqueues one work item on its slot's stream (scheduler thread, no lock held).
// Returns the HIP or ptalm error, with the message in q.err.
int launch(ptalm_server *s, Req &q, const ptalm::serve::Item &it) {
    hipStream_t st = s->streams[it.slot];
    hipError_t e = hipSuccess;
    if (it.chunk != ptalm::serve::kFinish) {
        const int s0 = it.chunk * q.slices_per_chunk;
        const int s1 = std::min(q.call.a.n_slices, s0 + q.slices_per_chunk);
        e = ptalm::launch_sliced(q.call, s0, s1, st);
    } else if (q.r.n == 0) {
        e = ptalm::launch_zero(q.r.alm, 2 * ptalm::tri_size(q.r.lmax), st);
    } else {
        e = ptalm::launch_sliced_finish(q.call, q.r.alm, st);
    }
    if (e == hipSuccess && it.chunk == ptalm::serve::kFinish && q.r.cl != nullptr)
        e = ptalm::launch_cl(q.r.alm, nullptr, q.r.lmax, q.r.cl, st);
    if (e != hipSuccess) {
        q.err = std::string("launch: ") + hipGetErrorString(e);
        return PTALM_EDEVICE;
    }
    return PTALM_OK;
}

void scheduler(ptalm_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        const double t = now_s();
        // 1. memory admission; plan each admitted request (tables built on first use)
        for (const ptalm::serve::Admitted &a : s->sched.admit(t)) {
            progress = true;
            Req &q = s->reqs[a.ticket];
            q.st.admit_s = t;
            q.st.footprint_bytes = a.bytes;
            if (q.r.n > 0) {
                lk.unlock();
                const int rc = ptalm::plan_sliced(q.r.theta, q.r.phi, q.r.w, q.r.n, q.r.lmax, q.r.precision,
                                                  (double *)((char *)s->arena + a.offset), &q.call);
                lk.lock();
                if (rc != PTALM_OK) {
                    q.failed = true;
                    q.st.status = rc;
                    q.err = ptalm_last_error();
                }
            }
        }
        // 2. work items onto free slots
        ptalm::serve::Item it;
        while (s->sched.next_item(t, &it)) {
            progress = true;
            Req &q = s->reqs[it.ticket];
            if (it.chunk == 0 || (it.chunk == ptalm::serve::kFinish && q.st.slot < 0)) q.st.slot = it.slot;
            hipEvent_t ev = nullptr;
            if (!q.failed) {
                lk.unlock();
                int rc = launch(s, q, it);
                if (rc == PTALM_OK) {
                    hipError_t e = hipSuccess;
                    if (s->spare_events.empty()) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                    else {
                        ev = s->spare_events.back();
                        s->spare_events.pop_back();
                    }
                    if (e == hipSuccess) e = hipEventRecord(ev, s->streams[it.slot]);
                    if (e != hipSuccess) {
                        rc = PTALM_EDEVICE;
                        q.err = std::string("completion event: ") + hipGetErrorString(e);
                    }
                }
                lk.lock();
                if (rc != PTALM_OK) {
                    q.failed = true;
                    q.st.status = rc;
                }
            }
            s->inflight.push_back({it, q.failed ? nullptr : ev});
            if (q.failed && ev) s->spare_events.push_back(ev);
        }
        // 3. completions
        for (size_t i = 0; i < s->inflight.size();) {
            InFlight &f = s->inflight[i];
            Req &q = s->reqs[f.it.ticket];
            bool finished = f.ev == nullptr;   // never launched (the request failed)
            if (!finished) {
                const hipError_t e = hipEventQuery(f.ev);
                if (e == hipSuccess) {
                    finished = true;
                } else if (e != hipErrorNotReady) {
                    finished = true;
                    q.failed = true;
                    q.st.status = PTALM_EDEVICE;
                    q.err = std::string("device error: ") + hipGetErrorString(e);
                }
            }
            if (!finished) {
                ++i;
                continue;
            }
            if (f.ev) s->spare_events.push_back(f.ev);
            if (s->sched.item_done(f.it)) {
                q.st.done_s = now_s();
                q.done = true;
            }
            s->inflight[i] = s->inflight.back();
            s->inflight.pop_back();
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        if (s->stop && s->sched.waiting() == 0 && s->sched.active() == 0 && s->inflight.empty()) break;
        if (!progress) {
            // idle or waiting on the device: short sleep, woken early by a submission
            s->cv_work.wait_for(lk, std::chrono::microseconds(s->inflight.empty() ? 2000 : 50));
        }
    }
}

}  // namespace

extern "C" {

int ptalm_server_create(int device, size_t arena_bytes, int slots, ptalm_server **out) {
    g_server_error.clear();
    if (out == nullptr) return sfail(PTALM_EINVAL, "out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64) return sfail(PTALM_EINVAL, "slots must be in [1, 64]");
    if (arena_bytes < ptalm::serve::kArenaAlign) return sfail(PTALM_EINVAL, "arena smaller than 256 bytes");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return sfail(PTALM_EDEVICE, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    if (device < 0 || device >= count) return sfail(PTALM_EINVAL, "no such device");
    int prev = 0;
    (void)hipGetDevice(&prev);
    if ((e = hipSetDevice(device)) != hipSuccess) return sfail(PTALM_EDEVICE, "hipSetDevice failed");
    ptalm_server *s = new ptalm_server(arena_bytes, slots);
    s->device = device;
    int rc = PTALM_OK;
    if ((e = hipMalloc(&s->arena, s->sched.arena().size())) != hipSuccess)
        rc = sfail(e == hipErrorOutOfMemory ? PTALM_ENOMEM : PTALM_EDEVICE, "arena allocation failed");
    for (int i = 0; i < slots && rc == PTALM_OK; ++i) {
        hipStream_t st;
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
            rc = sfail(PTALM_EDEVICE, "hipStreamCreate failed");
        else
            s->streams.push_back(st);
    }
    (void)hipSetDevice(prev);
    if (rc != PTALM_OK) {
        // clean-up after a failed creation: the first error is the one reported
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->arena) (void)hipFree(s->arena);
        delete s;
        return rc;
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return PTALM_OK;
}

int ptalm_server_submit(ptalm_server *s, const ptalm_request *req, int64_t *ticket) {
    g_server_error.clear();
    if (s == nullptr || req == nullptr || ticket == nullptr) return sfail(PTALM_EINVAL, "NULL argument");
    if (req->precision != PTALM_FP64 && req->precision != PTALM_MIXED && req->precision != PTALM_FP32)
        return sfail(PTALM_EINVAL, "served requests take PTALM_FP64, PTALM_MIXED or PTALM_FP32");
    if (req->n < 0 || req->lmax < 0 || req->lmax > PTALM_LMAX_MAX) return sfail(PTALM_EINVAL, "bad n or lmax");
    if (req->alm == nullptr || (req->n > 0 && (req->theta == nullptr || req->phi == nullptr || req->w == nullptr)))
        return sfail(PTALM_EINVAL, "NULL pointer in request");
    const size_t bytes = req->n > 0 ? footprint(*req) : ptalm::serve::kArenaAlign;
    if (bytes == 0) return sfail(PTALM_EINVAL, ptalm_last_error());
    // work items: chunks of about kChunkTerms terms, whole slices of the call's plan
    int chunks = 0, per_chunk = 1;
    double chunk_work = 0.0;
    if (req->n > 0) {
        const int S = ptalm::sliced_slice_count(req->n, req->lmax, req->precision);
        if (S < 1) return sfail(PTALM_EINVAL, ptalm_last_error());
        const double work = (double)req->n * (double)ptalm::tri_size(req->lmax);
        per_chunk = (int)std::min<double>(S, std::max(1.0, std::ceil(S * kChunkTerms / work)));
        chunks = (S + per_chunk - 1) / per_chunk;
        chunk_work = work * per_chunk / S;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(PTALM_EINVAL, "server is shutting down");
    const int64_t t = s->next_ticket;
    if (!s->sched.push(t, bytes, chunks, chunk_work, now_s()))
        return sfail(PTALM_EBUSY, "request footprint exceeds the server arena");
    ++s->next_ticket;
    Req &q = s->reqs[t];
    q.r = *req;
    q.chunks = chunks;
    q.slices_per_chunk = per_chunk;
    memset(&q.st, 0, sizeof q.st);
    q.st.status = PTALM_OK;
    q.st.slot = -1;
    q.st.footprint_bytes = bytes;
    q.st.submit_s = now_s();
    *ticket = t;
    s->cv_work.notify_one();
    return PTALM_OK;
}

int ptalm_server_poll(ptalm_server *s, int64_t ticket, int *done, ptalm_request_stats *stats) {
    g_server_error.clear();
    if (s == nullptr || done == nullptr) return sfail(PTALM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(PTALM_EINVAL, "unknown ticket");
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return PTALM_OK;
    if (stats) *stats = it->second.st;
    const int rc = it->second.st.status;
    if (rc != PTALM_OK) g_server_error = it->second.err;
    s->reqs.erase(it);
    return rc;
}

int ptalm_server_wait(ptalm_server *s, int64_t ticket, ptalm_request_stats *stats) {
    g_server_error.clear();
    if (s == nullptr) return sfail(PTALM_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(PTALM_EINVAL, "unknown ticket");
    s->cv_done.wait(lk, [&] {
        auto j = s->reqs.find(ticket);
        return j == s->reqs.end() || j->second.done;
    });
    it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(PTALM_EINVAL, "ticket collected by another caller");
    if (stats) *stats = it->second.st;
    const int rc = it->second.st.status;
    if (rc != PTALM_OK) g_server_error = it->second.err;
    s->reqs.erase(it);
    return rc;
}

int ptalm_server_query(ptalm_server *s, ptalm_server_state *info) {
    g_server_error.clear();
    if (s == nullptr || info == nullptr) return sfail(PTALM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    info->arena_bytes = s->sched.arena().size();
    info->arena_in_use = s->sched.arena().in_use();
    info->slots = s->sched.slots();
    info->running = (int)s->sched.active();
    info->waiting = (int64_t)s->sched.waiting();
    return PTALM_OK;
}

int ptalm_server_destroy(ptalm_server *s) {
    g_server_error.clear();
    if (s == nullptr) return PTALM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    // teardown: nothing pending remains, and errors here have no caller to report to
    for (hipEvent_t ev : s->spare_events) (void)hipEventDestroy(ev);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->arena);
    (void)hipSetDevice(prev);
    delete s;
    return PTALM_OK;
}

const char *ptalm_server_last_error(void) { return g_server_error.c_str(); }

}  // extern "C"
