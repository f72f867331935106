// Request server: continuous batching of transforms on one device.
//
// Requests (a catalog already resident in device memory, its lmax and
// precision, and where to write a_lm and optionally C_l) are queued by
// ptalm_server_submit from any host thread.  A scheduler thread admits them in
// arrival order as soon as an execution slot (a HIP stream of default
// priority) is free and their scratch footprint fits in the server's device
// arena (server_core.h), enqueues the transform (and spectrum) on the slot's
// stream with its arena block as workspace, and detects completion by polling
// an event per request; completion frees the slot and the block and wakes the
// waiters.  Requests admitted while others run execute concurrently on the
// device.  Every request is computed with the same work plan as the same call
// made alone, so its result is bitwise the solo result.
#include <string.h>

#include <chrono>
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

struct Req {
    ptalm_request r;
    ptalm_request_stats st;
    ptalm::serve::Admitted adm{};
    hipEvent_t done_ev = nullptr;
    bool done = false;
    std::string err;
};

}  // namespace

struct ptalm_server {
    int device = 0;
    void *arena = nullptr;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    ptalm::serve::Admission adm;
    std::unordered_map<int64_t, Req> reqs;
    std::vector<int64_t> inflight;
    int64_t next_ticket = 1;
    bool stop = false;
    std::thread th;

    ptalm_server(size_t bytes, int slots) : adm(bytes, slots) {}
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

// Enqueues one admitted request on its slot's stream (scheduler thread, no lock held).
void launch(ptalm_server *s, Req &q) {
    hipStream_t st = s->streams[q.adm.slot];
    ptalm_opts o;
    memset(&o, 0, sizeof o);
    o.precision = q.r.precision;
    o.n_weights = 1;
    void *ws = (char *)s->arena + q.adm.offset;
    int rc = ptalm_alm_from_points_ex(q.r.theta, q.r.phi, q.r.w, q.r.n, q.r.lmax, q.r.alm, &o, ws, q.adm.bytes, st);
    if (rc == PTALM_OK && q.r.cl != nullptr) rc = ptalm_cl_from_alm(q.r.alm, q.r.lmax, q.r.cl, st);
    if (rc == PTALM_OK) {
        hipError_t e = hipEventCreateWithFlags(&q.done_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(q.done_ev, st);
        if (e != hipSuccess) {
            rc = PTALM_EDEVICE;
            q.err = std::string("completion event: ") + hipGetErrorString(e);
        }
    } else {
        q.err = ptalm_last_error();
    }
    q.st.status = rc;
}

void scheduler(ptalm_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = false;
        // 1. admissions, in arrival order
        std::vector<ptalm::serve::Admitted> adm = s->adm.admit();
        if (!adm.empty()) {
            progress = true;
            const double t = now_s();
            std::vector<Req *> batch;
            for (const auto &a : adm) {
                Req &q = s->reqs[a.ticket];
                q.adm = a;
                q.st.admit_s = t;
                q.st.slot = a.slot;
                q.st.footprint_bytes = a.bytes;
                batch.push_back(&q);
            }
            lk.unlock();
            for (Req *q : batch) launch(s, *q);   // map entries are stable while in flight
            lk.lock();
            for (Req *q : batch) s->inflight.push_back(q->adm.ticket);
        }
        // 2. completions
        for (size_t i = 0; i < s->inflight.size();) {
            Req &q = s->reqs[s->inflight[i]];
            bool finished = q.st.status != PTALM_OK;   // failed at launch
            if (!finished) {
                const hipError_t e = hipEventQuery(q.done_ev);
                if (e == hipSuccess) {
                    finished = true;
                } else if (e != hipErrorNotReady) {
                    finished = true;
                    q.st.status = PTALM_EDEVICE;
                    q.err = std::string("device error: ") + hipGetErrorString(e);
                }
            }
            if (!finished) {
                ++i;
                continue;
            }
            if (q.done_ev) {
                hipEventDestroy(q.done_ev);
                q.done_ev = nullptr;
            }
            q.st.done_s = now_s();
            q.done = true;
            s->adm.complete(q.adm);
            s->inflight[i] = s->inflight.back();
            s->inflight.pop_back();
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        if (s->stop && s->adm.waiting() == 0 && s->inflight.empty()) break;
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
    if ((e = hipMalloc(&s->arena, s->adm.arena().size())) != hipSuccess)
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
        for (hipStream_t st : s->streams) hipStreamDestroy(st);
        if (s->arena) hipFree(s->arena);
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
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return sfail(PTALM_EINVAL, "server is shutting down");
    const int64_t t = s->next_ticket;
    if (!s->adm.push(t, bytes)) return sfail(PTALM_EBUSY, "request footprint exceeds the server arena");
    ++s->next_ticket;
    Req &q = s->reqs[t];
    q.r = *req;
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
    info->arena_bytes = s->adm.arena().size();
    info->arena_in_use = s->adm.arena().in_use();
    info->slots = s->adm.slots();
    info->running = s->adm.running();
    info->waiting = (int64_t)s->adm.waiting();
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
    for (hipStream_t st : s->streams) hipStreamDestroy(st);
    hipFree(s->arena);
    (void)hipSetDevice(prev);
    delete s;
    return PTALM_OK;
}

const char *ptalm_server_last_error(void) { return g_server_error.c_str(); }

}  // extern "C"
