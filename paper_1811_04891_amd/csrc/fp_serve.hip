// Serving layer: continuous batching of findpts + findpts_eval requests over
// resident meshes.  One host worker thread admits queued requests when a slot
// (HIP stream) is free and the request's workspace fits in the device arena,
// enqueues its kernels on the slot's stream, and a host callback at the end
// of that stream's work completes the request, releases slot and workspace,
// and wakes the worker to admit the next ones.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fp_internal.h"

namespace fp {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxSlots = 16;
constexpr int kMaxPass = 1 << 20;  // points per findpts pass of a request
constexpr int kMinPass = 256;
constexpr int kMaxBypass = 8;      // later requests admitted past a waiting one
constexpr size_t kWindow = 64;     // queued requests examined per admission

// First-fit allocator over [0, size) (offsets and lengths are multiples of
// 256 bytes), coalescing on release.
struct Arena {
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;  // offset -> length

    void init(size_t n)
    {
        size = n;
        used = peak = 0;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest) free_[o + n] = rest;
            *off = o;
            used += n;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
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
        used -= n;
    }
};

struct Mesh {
    fp_handle *h = nullptr;
    std::vector<const double *> fields;
};

enum State { kQueued, kRunning, kDone };

struct Request {
    fps *owner = nullptr;
    long long id = 0;
    int mesh = 0, npts = 0;
    // the mesh as sized at submit: the workspace is laid out with these, and
    // launch refuses a handle whose candidate lists have since grown
    fp_handle *h = nullptr;
    int E = 0, MC = 1;
    bool delta = false;
    const double *pts = nullptr;
    const int *psess = nullptr;
    std::vector<const double *> fields;
    int *code = nullptr, *el = nullptr;
    double *rst = nullptr, *dist2 = nullptr, *out = nullptr;
    int pass = 0;       // points per findpts pass
    size_t bytes = 0;   // workspace bytes
    size_t off = 0;     // workspace offset in the arena
    int slot = -1;
    bool waited = false;
    State state = kQueued;
    int rc = FP_OK;
    std::string err;
    Clock::time_point t_submit, t_done;
};

}  // namespace
}  // namespace fp

struct fps {
    int device = 0;
    char *arena_mem = nullptr;
    fp::Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<long long> slot_req;  // running request per slot, 0 = free
    std::vector<fp::Mesh> meshes;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<long long> queue;
    std::map<long long, std::unique_ptr<fp::Request>> reqs;
    long long next_id = 1;
    int running = 0, peak_running = 0, bypass = 0;
    long long waited_admissions = 0;
    bool stop = false;
    std::thread worker;

    // latency window (since the last reset)
    std::vector<double> lat;
    long long pts_done = 0;
    bool have_window = false;
    fp::Clock::time_point win_first, win_last;
};

namespace fp {
namespace {

int free_slot(const fps *s)
{
    for (size_t i = 0; i < s->slot_req.size(); ++i)
        if (s->slot_req[i] == 0) return (int)i;
    return -1;
}

// Mark a request finished (caller holds the lock).
void finish_locked(fps *s, Request *r, Clock::time_point t)
{
    r->t_done = t;
    r->state = kDone;
    s->arena.release(r->off, r->bytes);
    s->slot_req[r->slot] = 0;
    --s->running;
    if (r->rc == FP_OK) {
        s->lat.push_back(std::chrono::duration<double>(t - r->t_submit).count());
        s->pts_done += r->npts;
        if (!s->have_window || r->t_submit < s->win_first) s->win_first = r->t_submit;
        if (!s->have_window || t > s->win_last) s->win_last = t;
        s->have_window = true;
    }
}

// Host callback at the end of a request's stream work: no HIP calls here.
void on_done(void *p)
{
    Request *r = static_cast<Request *>(p);
    fps *s = r->owner;
    const Clock::time_point t = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        finish_locked(s, r, t);
    }
    s->cv.notify_all();
}

// Enqueue one admitted request on its slot's stream (no lock held).
int launch(fps *s, Request *r)
{
    hipStream_t st = s->streams[r->slot];
    fp_handle *h = r->h;
    // findpts_update between submit and admission may have lengthened the
    // longest hash-cell list: the reserved workspace would then be too small
    if (h->E != r->E || h->MC > r->MC || (h->delta != nullptr) != r->delta) {
        set_error("fps: the mesh changed (findpts_update) while the request was queued");
        return FP_ESTATE;
    }
    Work w;
    work_carve(w, s->arena_mem + r->off, r->E, r->MC, r->pass, r->delta);
    int rc = run_findpts(h, w, r->npts, r->pts, r->psess, r->code, r->el, r->rst, r->dist2, st,
                         false);
    if (rc == FP_OK && !r->fields.empty())
        rc = run_eval(h, w, r->npts, r->code, r->el, r->rst, (int)r->fields.size(),
                      r->fields.data(), r->out, st, false);
    if (rc == FP_OK) {
        const hipError_t e = hipLaunchHostFunc(st, on_done, r);
        if (e != hipSuccess) rc = hip_fail(e, "hipLaunchHostFunc");
    }
    return rc;
}

void worker_main(fps *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        for (;;) {
            const int slot = free_slot(s);
            if (slot < 0 || s->queue.empty()) break;
            const size_t window =
                (s->bypass >= kMaxBypass) ? 1 : std::min(s->queue.size(), kWindow);
            Request *pick = nullptr;
            size_t pos = 0, off = 0;
            for (size_t i = 0; i < window; ++i) {
                Request *r = s->reqs[s->queue[i]].get();
                if (s->arena.alloc(r->bytes, &off)) {
                    pick = r;
                    pos = i;
                    break;
                }
            }
            if (!pick) break;
            s->bypass = (pos > 0) ? s->bypass + 1 : 0;
            s->queue.erase(s->queue.begin() + (long)pos);
            if (pick->waited) ++s->waited_admissions;
            pick->state = kRunning;
            pick->slot = slot;
            pick->off = off;
            s->slot_req[slot] = pick->id;
            ++s->running;
            s->peak_running = std::max(s->peak_running, s->running);
            lk.unlock();
            const int rc = launch(s, pick);
            std::string msg = (rc == FP_OK) ? std::string() : std::string(fp_last_error());
            if (rc != FP_OK) (void)hipStreamSynchronize(s->streams[slot]);
            lk.lock();
            if (rc != FP_OK) {
                pick->rc = rc;
                pick->err = msg;
                finish_locked(s, pick, Clock::now());
                s->cv.notify_all();
            }
        }
        for (long long id : s->queue) s->reqs[id]->waited = true;
        if (s->stop && s->queue.empty() && s->running == 0) break;
        s->cv.wait(lk);
    }
}

}  // namespace
}  // namespace fp

using namespace fp;

extern "C" int fps_create(fps **out, size_t hbm_budget_bytes, int slots)
{
    if (!out) {
        set_error("fps_create: NULL argument");
        return FP_EINVAL;
    }
    *out = nullptr;
    if (hbm_budget_bytes == 0 || slots < 1 || slots > kMaxSlots) {
        set_error("fps_create: need a budget > 0 and 1 <= slots <= 16");
        return FP_EINVAL;
    }
    std::unique_ptr<fps> s(new fps());
    FP_HIP(hipGetDevice(&s->device));
    const size_t budget = (hbm_budget_bytes / 256) * 256;
    if (budget == 0) {
        set_error("fps_create: budget below 256 bytes");
        return FP_EINVAL;
    }
    const hipError_t e = hipMalloc((void **)&s->arena_mem, budget);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("fps_create: cannot reserve the device arena");
        return FP_ENOMEM;
    }
    s->arena.init(budget);
    for (int i = 0; i < slots; ++i) {
        hipStream_t st = nullptr;
        const hipError_t es = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (es != hipSuccess) {
            for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
            (void)hipFree(s->arena_mem);
            return hip_fail(es, "hipStreamCreateWithFlags");
        }
        s->streams.push_back(st);
    }
    s->slot_req.assign(slots, 0);
    fps *raw = s.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return FP_OK;
}

extern "C" int fps_add_mesh(fps *s, fp_handle *h, const double *const *h_fields, int nfields,
                            int *h_mesh_id)
{
    if (!s || !h || !h_mesh_id || nfields < 0 || (nfields > 0 && !h_fields)) {
        set_error("fps_add_mesh: NULL argument or nfields < 0");
        return FP_EINVAL;
    }
    if (h->device != s->device) {
        set_error("fps_add_mesh: handle lives on another device");
        return FP_EINVAL;
    }
    Mesh m;
    m.h = h;
    for (int f = 0; f < nfields; ++f) {
        if (!h_fields[f]) {
            set_error("fps_add_mesh: NULL field pointer");
            return FP_EINVAL;
        }
        m.fields.push_back(h_fields[f]);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->meshes.push_back(std::move(m));
    *h_mesh_id = (int)s->meshes.size() - 1;
    return FP_OK;
}

extern "C" int fps_submit(fps *s, int mesh_id, int npts, const double *pts,
                          const int *pt_session, int nfields, const int *h_field_ids, int *code,
                          int *el, double *rst, double *dist2, double *out, long long *h_ticket)
{
    const Clock::time_point t0 = Clock::now();
    if (!s || !h_ticket || npts < 0 || nfields < 0) {
        set_error("fps_submit: NULL argument or negative size");
        return FP_EINVAL;
    }
    std::unique_ptr<Request> r(new Request());
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (mesh_id < 0 || mesh_id >= (int)s->meshes.size()) {
            set_error("fps_submit: unknown mesh id");
            return FP_EINVAL;
        }
        const Mesh &m = s->meshes[mesh_id];
        if (nfields > 0 && !h_field_ids) {
            set_error("fps_submit: NULL field id list");
            return FP_EINVAL;
        }
        for (int f = 0; f < nfields; ++f) {
            const int id = h_field_ids[f];
            if (id < 0 || id >= (int)m.fields.size()) {
                set_error("fps_submit: unknown field id");
                return FP_EINVAL;
            }
            r->fields.push_back(m.fields[id]);
        }
        if (npts > 0 && (!pts || !code || !el || !rst || !dist2 || (nfields > 0 && !out))) {
            set_error("fps_submit: NULL buffer");
            return FP_EINVAL;
        }
        // workspace: one pass of up to 2^20 points, halved until it fits
        const fp_handle *h = m.h;
        int pass = std::max(1, std::min(npts, kMaxPass));
        while ((double)pass * h->MC >= 2147483647.0) pass /= 2;
        size_t bytes = work_bytes(h->E, h->MC, pass, h->delta != nullptr);
        while (bytes > s->arena.size && pass > kMinPass) {
            pass = std::max(kMinPass, pass / 2);
            bytes = work_bytes(h->E, h->MC, pass, h->delta != nullptr);
        }
        if (bytes > s->arena.size) {
            set_error("fps_submit: the request's workspace exceeds the serving budget");
            return FP_ENOMEM;
        }
        r->owner = s;
        r->id = s->next_id++;
        r->mesh = mesh_id;
        r->h = m.h;
        r->E = h->E;
        r->MC = h->MC;
        r->delta = h->delta != nullptr;
        r->npts = npts;
        r->pts = pts;
        r->psess = pt_session;
        r->code = code;
        r->el = el;
        r->rst = rst;
        r->dist2 = dist2;
        r->out = out;
        r->pass = pass;
        r->bytes = bytes;
        r->t_submit = t0;
        *h_ticket = r->id;
        if (npts == 0) {
            r->state = kDone;
            r->t_done = t0;
            s->reqs[r->id] = std::move(r);
            return FP_OK;
        }
        s->queue.push_back(r->id);
        s->reqs[r->id] = std::move(r);
    }
    s->cv.notify_all();
    return FP_OK;
}

extern "C" int fps_wait(fps *s, long long ticket, double timeout_s)
{
    if (!s) {
        set_error("fps_wait: NULL serving object");
        return FP_EINVAL;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        set_error("fps_wait: unknown ticket (or already waited for)");
        return FP_EINVAL;
    }
    Request *r = it->second.get();
    auto done = [r] { return r->state == kDone; };
    if (timeout_s < 0) {
        s->cv.wait(lk, done);
    } else if (!s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        set_error("fps_wait: timed out");
        return FP_EBUSY;
    }
    const int rc = r->rc;
    if (rc != FP_OK) set_error(r->err);
    s->reqs.erase(it);
    return rc;
}

extern "C" int fps_latency(fps *s, double *h_p50_s, double *h_p99_s, double *h_pts_per_s,
                           long long *h_info, int reset)
{
    if (!s || !h_p50_s || !h_p99_s || !h_pts_per_s) {
        set_error("fps_latency: NULL argument");
        return FP_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto rank = [&v](double q) {
        if (v.empty()) return 0.0;
        const size_t k = (size_t)std::ceil(q * (double)v.size());
        return v[std::min(v.size(), std::max<size_t>(k, 1)) - 1];
    };
    *h_p50_s = rank(0.50);
    *h_p99_s = rank(0.99);
    const double span = s->have_window
                            ? std::chrono::duration<double>(s->win_last - s->win_first).count()
                            : 0.0;
    *h_pts_per_s = span > 0.0 ? (double)s->pts_done / span : 0.0;
    if (h_info) {
        h_info[0] = (long long)s->lat.size();
        h_info[1] = (long long)s->queue.size();
        h_info[2] = s->running;
        h_info[3] = s->peak_running;
        h_info[4] = (long long)s->arena.peak;
        h_info[5] = s->waited_admissions;
    }
    if (reset) {
        s->lat.clear();
        s->pts_done = 0;
        s->have_window = false;
        s->peak_running = s->running;
        s->arena.peak = s->arena.used;
        s->waited_admissions = 0;
    }
    return FP_OK;
}

extern "C" int fps_destroy(fps *s)
{
    if (!s) return FP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    // the last host callbacks may still be returning: drain the streams
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    (void)hipFree(s->arena_mem);
    delete s;
    return FP_OK;
}
