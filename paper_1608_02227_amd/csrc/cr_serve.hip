// Serving: continuous batching of convex-regression fits on one device.
//
// Requests enter a FIFO queue.  An admission step moves the head of the queue onto a free slot
// as soon as one is free and the device bytes of its state (its whole workspace, including the
// FP64 copy a mixed-precision promotion would take) fit in the context's budget.  Each slot has
// its own worker thread, HIP stream, pinned scalar buffer and device arena; a fit runs inside its
// slot's arena (the solver's workspace mode), which grows to the largest fit the slot has run and
// is then reused, so fits do not allocate or free device memory (hipFree would synchronize the
// device under every other slot's work).  Admitted fits run concurrently on the GPU and a new fit
// starts the moment one retires.  A fit's arithmetic does not depend on what else is running (same
// kernels, tiling and fixed-order reductions), so its result is bitwise the same alone and in a
// mix.  Strict FIFO: a head request that does not fit waits for memory rather than being
// overtaken.

#include "cr_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int64_t id = 0;
    int64_t N = 0, n = 0;
    std::vector<double> x, ybar;
    double delta = 1e-3, tol = 1e-4;
    cr_options opt{};
    size_t bytes = 0;
    double t_submit = 0.0, t_done = 0.0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int status = CR_OK;
    std::vector<double> y, xi;
    std::vector<double> lam0;    // warm start (opt.lambda0, copied at submission)
    std::vector<double> lam;     // final multipliers (opt.keep_lambda)
    cr_report rep{};
};

// One slot's resources, created with the context and reused by every fit the slot runs.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr;   // orders the slot's grouped trial rounds behind its stream
    double *h_scal = nullptr;     // pinned, 32 doubles (trial scalars and the sequence word)
    char *arena = nullptr;        // device workspace of the current capacity
    size_t cap = 0;
};



}  // namespace

struct cr_ctx {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    std::mutex mu;
    std::condition_variable cv_work;   // slot threads wait for assignments
    std::condition_variable cv_done;   // waiters for results / admission changes
    std::condition_variable cv_idle;   // destroy waits for the callers inside cr_wait to leave
    std::deque<int64_t> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::vector<int64_t> assigned;     // per slot: request id or -1
    std::vector<std::thread> workers;
    std::vector<Slot> slots;
    size_t resident = 0;
    int64_t next_id = 1;
    int64_t finished = 0, running = 0;
    int waiters = 0;
    bool stop = false;
    // grouped iterations (cr_ctx_set_grouping): fits with N <= group_max_n hand their adaptive-step
    // rounds to `batch`; off (0) by default
    cr_batcher *batch = nullptr;
    int64_t group_max_n = 0;

    void admit_locked() {
        while (!stop && !queue.empty()) {
            Request *r = reqs[queue.front()].get();
            int slot = -1;
            for (int q = 0; q < max_slots; ++q)
                if (assigned[q] < 0) { slot = q; break; }
            if (slot < 0 || resident + r->bytes > budget) return;
            queue.pop_front();
            assigned[slot] = r->id;
            resident += r->bytes;
            r->state = 1;
            ++running;
        }
        cv_work.notify_all();
    }

    void worker(int slot) {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv_work.wait(lk, [&] { return stop || assigned[slot] >= 0; });
            if (assigned[slot] < 0) return;   // stopping and nothing assigned
            Request *r = reqs[assigned[slot]].get();
            cr_batcher *b = (batch && r->N <= group_max_n && r->opt.step_rule == 1) ? batch : nullptr;
            lk.unlock();
            run(r, slots[slot], b);
            lk.lock();
            r->state = 2;
            resident -= r->bytes;
            assigned[slot] = -1;
            --running;
            ++finished;
            admit_locked();
            cv_done.notify_all();
            if (stop) return;
        }
    }

    // Grows the slot's arena to `need` bytes (freeing the smaller one first).
    int reserve(Slot &sl, size_t need) {
        if (need <= sl.cap) return CR_OK;
        if (sl.arena) (void)hipFree(sl.arena);
        sl.arena = nullptr;
        sl.cap = 0;
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? CR_ENOMEM : CR_EDEVICE;
        }
        sl.arena = static_cast<char *>(p);
        sl.cap = need;
        return CR_OK;
    }

    void run(Request *r, Slot &sl, cr_batcher *b) {
        cr_options o = r->opt;
        o.device = device;
        o.stream = sl.stream;
        o.lambda0 = r->lam0.empty() ? nullptr : r->lam0.data();
        r->y.assign((size_t)r->N, 0.0);
        r->xi.assign((size_t)(r->N * r->n), 0.0);
        double *lam_out = nullptr;
        if (r->opt.keep_lambda) {
            r->lam.assign((size_t)(r->N * r->N), 0.0);
            lam_out = r->lam.data();
        }
        if (r->N == 1) {
            r->status = cr_fit(r->N, r->n, r->x.data(), r->ybar.data(), r->delta, r->tol, &o, r->y.data(),
                               r->xi.data(), lam_out, &r->rep);
        } else {
            r->status = reserve(sl, r->bytes);
            if (r->status == CR_OK) {
                cr_workspace ws;
                ws.base = sl.arena;
                ws.size = sl.cap;
                r->status = cr_fit_impl(r->N, r->n, r->x.data(), r->ybar.data(), r->delta, r->tol, &o, r->y.data(),
                                        r->xi.data(), lam_out, &r->rep, false, &ws, sl.h_scal, b,
                                        b ? sl.ready : nullptr);
            }
        }
        r->t_done = now_s();
        r->x.clear();
        r->x.shrink_to_fit();
        r->lam0.clear();
        r->lam0.shrink_to_fit();
    }
};

// Device bytes of one fit's whole state in a slot arena (0 for invalid arguments; N = 1 needs none).
static size_t request_bytes(int64_t N, int64_t n, const cr_options &opt, int device) {
    if (N == 1) return 0;
    return cr_workspace_bytes(N, n, &opt, device, true);
}

extern "C" size_t cr_fit_state_bytes(int64_t N, int64_t n, int32_t precision) {
    if (N < 1 || n < 1 || n + 1 > 16 * cr::kMaxMB || precision < CR_FP64 || precision > CR_MIXED_BF16) return 0;
    cr_options o;
    cr_default_options(&o);
    o.precision = precision;
    return request_bytes(N, n, o, 0);
}

extern "C" int cr_ctx_create(int device, size_t byte_budget, int32_t max_slots, cr_ctx **out) {
    if (!out || max_slots < 1 || max_slots > 64) return CR_EINVAL;
    *out = nullptr;
    if (cr_device_check(device) != CR_OK) return CR_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return CR_EDEVICE;
    cr_ctx *c = new cr_ctx();
    c->device = device;
    c->max_slots = max_slots;
    if (byte_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete c; return CR_EDEVICE; }
        byte_budget = (size_t)(0.8 * (double)fr);
    }
    c->budget = byte_budget;
    c->assigned.assign((size_t)max_slots, -1);
    c->slots.resize((size_t)max_slots);
    bool ok = true;
    for (int q = 0; ok && q < max_slots; ++q) {
        Slot &sl = c->slots[q];
        ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc((void **)&sl.h_scal, 32 * sizeof(double), hipHostMallocDefault) == hipSuccess;
        if (ok) std::memset(sl.h_scal, 0, 32 * sizeof(double));
    }
    if (!ok) {
        for (auto &o : c->slots) {
            if (o.stream) (void)hipStreamDestroy(o.stream);
            if (o.ready) (void)hipEventDestroy(o.ready);
            if (o.h_scal) (void)hipHostFree(o.h_scal);
        }
        cr_batcher_destroy(c->batch);
        delete c;
        return CR_EDEVICE;
    }
    for (int q = 0; q < max_slots; ++q) c->workers.emplace_back([c, q] { c->worker(q); });
    *out = c;
    return CR_OK;
}

extern "C" int cr_ctx_destroy(cr_ctx *c) {
    if (!c) return CR_EINVAL;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->stop = true;
        // queued requests are dropped: their waiters wake with CR_ECANCELED
        for (int64_t id : c->queue) {
            Request *r = c->reqs[id].get();
            r->state = 2;
            r->status = CR_ECANCELED;
            r->t_done = now_s();
        }
        c->queue.clear();
    }
    c->cv_work.notify_all();
    c->cv_done.notify_all();
    // running fits finish their current solve before the threads exit
    for (auto &t : c->workers) t.join();
    {
        // every request is done now; wait until the callers blocked in cr_wait have taken their
        // results and left (they hold references into the context)
        std::unique_lock<std::mutex> lk(c->mu);
        c->cv_done.notify_all();
        c->cv_idle.wait(lk, [&] { return c->waiters == 0; });
    }
    cr_batcher_destroy(c->batch);   // no fit is running: its thread has nothing left to launch
    for (auto &sl : c->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.arena) (void)hipFree(sl.arena);
        if (sl.h_scal) (void)hipHostFree(sl.h_scal);
        if (sl.ready) (void)hipEventDestroy(sl.ready);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete c;
    return CR_OK;
}

extern "C" int cr_submit(cr_ctx *c, int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
                         const cr_options *opt, int64_t *req_id) {
    if (!c || !x || !ybar || !req_id || N < 1 || n < 1 || n + 1 > 16 * cr::kMaxMB || !(delta > 0.0) || !(tol > 0.0))
        return CR_EINVAL;
    auto r = std::make_unique<Request>();
    r->N = N;
    r->n = n;
    r->x.assign(x, x + (size_t)(N * n));
    r->ybar.assign(ybar, ybar + (size_t)N);
    r->delta = delta;
    r->tol = tol;
    if (opt) r->opt = *opt; else cr_default_options(&r->opt);
    if (r->opt.precision < CR_FP64 || r->opt.precision > CR_MIXED_BF16) return CR_EINVAL;
    if (r->opt.keep_lambda < 0 || r->opt.keep_lambda > 1) return CR_EINVAL;
    // sized with the warm start still set (its staging), which then lives in the request
    r->bytes = request_bytes(N, n, r->opt, c->device);
    if (r->opt.lambda0) r->lam0.assign(r->opt.lambda0, r->opt.lambda0 + (size_t)(N * N));
    r->opt.lambda0 = nullptr;
    if (N > 1 && r->bytes == 0) return CR_EINVAL;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->stop) return CR_ECANCELED;
    if (r->bytes > c->budget) return CR_ENOMEM;
    r->id = c->next_id++;
    *req_id = r->id;
    c->queue.push_back(r->id);
    c->reqs[r->id] = std::move(r);
    c->admit_locked();
    return CR_OK;
}

static int collect(cr_ctx *c, Request *r, int64_t id, double *y, double *xi, double *lambda, cr_report *rep,
                   double *lat) {
    if (r->status != CR_ECANCELED) {
        if (y) std::memcpy(y, r->y.data(), r->y.size() * 8);
        if (xi) std::memcpy(xi, r->xi.data(), r->xi.size() * 8);
        if (lambda) std::memcpy(lambda, r->lam.data(), r->lam.size() * 8);
        if (rep) *rep = r->rep;
    }
    if (lat) *lat = r->t_done - r->t_submit;
    const int st = r->status;
    c->reqs.erase(id);
    return st;
}

extern "C" int cr_poll(cr_ctx *c, int64_t id, double *y, double *xi, double *lambda, cr_report *rep,
                       double *latency_s) {
    if (!c) return CR_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->reqs.find(id);
    if (it == c->reqs.end()) return CR_ENOTFOUND;
    if (lambda && !it->second->opt.keep_lambda) return CR_EINVAL;
    if (it->second->state != 2) return CR_EAGAIN;
    return collect(c, it->second.get(), id, y, xi, lambda, rep, latency_s);
}

extern "C" int cr_wait(cr_ctx *c, int64_t id, double *y, double *xi, double *lambda, cr_report *rep,
                       double *latency_s) {
    if (!c) return CR_EINVAL;
    std::unique_lock<std::mutex> lk(c->mu);
    auto it = c->reqs.find(id);
    if (it == c->reqs.end()) return CR_ENOTFOUND;
    Request *r = it->second.get();
    if (lambda && !r->opt.keep_lambda) return CR_EINVAL;
    ++c->waiters;
    c->cv_done.wait(lk, [&] { return r->state == 2; });
    const int st = collect(c, r, id, y, xi, lambda, rep, latency_s);
    if (--c->waiters == 0) c->cv_idle.notify_all();
    return st;
}

extern "C" int cr_ctx_stats(cr_ctx *c, int64_t *queued, int64_t *running, int64_t *finished, size_t *resident) {
    if (!c) return CR_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (queued) *queued = (int64_t)c->queue.size();
    if (running) *running = c->running;
    if (finished) *finished = c->finished;
    if (resident) *resident = c->resident;
    return CR_OK;
}

extern "C" int cr_ctx_set_grouping(cr_ctx *c, int64_t max_n) {
    if (!c || max_n < 0) return CR_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (max_n > 0 && !c->batch) {
        c->batch = cr_batcher_create(c->device);
        if (!c->batch) return CR_EDEVICE;
    }
    c->group_max_n = max_n;
    return CR_OK;
}

extern "C" int cr_ctx_group_stats(cr_ctx *c, double *rounds, double *pass_launches, double *fit_rounds) {
    if (!c) return CR_EINVAL;
    if (rounds) *rounds = 0.0;
    if (pass_launches) *pass_launches = 0.0;
    if (fit_rounds) *fit_rounds = 0.0;
    if (c->batch) cr_batcher_stats(c->batch, rounds, pass_launches, fit_rounds);
    return CR_OK;
}
