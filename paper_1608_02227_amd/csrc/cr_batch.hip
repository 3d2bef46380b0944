// Grouped trial rounds for serving: the same step of several small fits in one launch per kernel.
//
// Each fit of the serving context runs its own driver loop (cr_solver::solve on its slot thread).
// Under the adaptive step an iteration is a trial round: the pair sweep (re-forming or retry
// trial pass), the trial finalize, the reduction that takes the step decision, and the queued
// update of the primal point.  A fit attached to a batcher hands that round over instead of
// launching it.  The rounds of the fits that are iterating are gathered -- until every active fit
// has handed over its round, or at most kGatherUs -- and launched as grouped kernels on the
// batcher's stream: one pass launch per kernel variant (mode, arithmetic, representation, feature
// blocks), one trial finalize per (arithmetic, feature blocks), one reduction and one update
// launch for the whole round.  There is no batcher thread: the first fit thread of a round gathers
// and launches it (cr_batcher_run).  Each fit's workgroups compute exactly what its own launches
// would (same tiles and fixed-order sums), so results do not depend on the grouping.  Events order
// a round behind its fit's earlier work and the fit's later work behind the round; the fit then
// reads its decision from pinned memory as usual.

#include "cr_internal.h"

#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

using namespace cr;

namespace {
constexpr int kGatherUs = 30;      // longest wait for the other active fits of a round
constexpr int kDoneRing = 32;      // events marking the ends of rounds (reused round-robin)
}  // namespace

struct cr_batcher {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done[kDoneRing] = {};
    int done_pos = 0;
    std::mutex mu;                       // guards pending, leader, active and the counters
    std::vector<TrialPlan *> pending;
    bool leader = false;                 // a fit thread is gathering / launching a round
    int active = 0;
    double rounds = 0.0, pass_launches = 0.0, fit_rounds = 0.0;

    // Launches one round; returns a HIP error code (hipSuccess on success).
    hipError_t launch(std::vector<TrialPlan *> &batch) {
        hipError_t e = hipSuccess;
        auto H = [&](hipError_t x) { if (e == hipSuccess && x != hipSuccess) e = x; };
        // a fit whose earlier work has already finished needs no wait (the common case: between
        // two of its rounds the fit's stream only waits for the previous round)
        for (TrialPlan *p : batch)
            if (hipEventQuery(p->ready) != hipSuccess) H(hipStreamWaitEvent(stream, p->ready, 0));
        // grouped passes, one launch per kernel variant (kGroupMax fits at most)
        std::map<int, std::vector<TrialPlan *>> by_key;
        for (TrialPlan *p : batch) by_key[pass_group_key(p->g, p->mode, p->fp32, p->rep)].push_back(p);
        for (auto &kv : by_key) {
            auto &v = kv.second;
            for (size_t b0 = 0; b0 < v.size(); b0 += kGroupMax) {
                PassGroup G{};
                G.nfit = (int)std::min<size_t>(kGroupMax, v.size() - b0);
                G.off[0] = 0;
                for (int f = 0; f < G.nfit; ++f) {
                    const TrialPlan *p = v[b0 + f];
                    G.g[f] = p->g;
                    G.a[f] = p->pass;
                    G.off[f + 1] = G.off[f] + p->g.grid();
                }
                H(launch_pass_group(v[b0]->mode, v[b0]->fp32, v[b0]->rep, G, stream));
                pass_launches += 1.0;
            }
        }
        // trial finalize per (arithmetic, feature blocks)
        std::map<int, std::vector<TrialPlan *>> by_fin;
        for (TrialPlan *p : batch) by_fin[(p->fp32 ? 16 : 0) + p->g.MB].push_back(p);
        for (auto &kv : by_fin) {
            auto &v = kv.second;
            for (size_t b0 = 0; b0 < v.size(); b0 += kGroupMax) {
                TrialFinalizeGroup G{};
                G.nfit = (int)std::min<size_t>(kGroupMax, v.size() - b0);
                G.off[0] = 0;
                for (int f = 0; f < G.nfit; ++f) {
                    const TrialPlan *p = v[b0 + f];
                    G.g[f] = p->g;
                    G.a[f] = p->fin;
                    G.off[f + 1] = G.off[f] + p->g.Nr / 16;
                }
                H(launch_trial_finalize_group(v[b0]->fp32, v[b0]->g.MB, G, stream));
            }
        }
        // the step decisions, then the queued updates
        for (size_t b0 = 0; b0 < batch.size(); b0 += kGroupMax) {
            TrialReduceGroup R{};
            R.nfit = (int)std::min<size_t>(kGroupMax, batch.size() - b0);
            for (int f = 0; f < R.nfit; ++f) R.a[f] = batch[b0 + f]->red;
            H(launch_trial_reduce_group(R, stream));
        }
        for (size_t b0 = 0; b0 < batch.size(); b0 += kGroupMax) {
            AcceptGroup A{};
            A.nfit = (int)std::min<size_t>(kGroupMax, batch.size() - b0);
            A.off[0] = 0;
            for (int f = 0; f < A.nfit; ++f) {
                const TrialPlan *p = batch[b0 + f];
                A.a[f] = p->acc;
                A.off[f + 1] = A.off[f] + p->g.Nr / 16;
            }
            H(launch_accept_group(A, stream));
        }
        hipEvent_t ev = done[done_pos];
        done_pos = (done_pos + 1) % kDoneRing;
        H(hipEventRecord(ev, stream));
        for (TrialPlan *p : batch) p->done = ev;
        rounds += 1.0;
        fit_rounds += (double)batch.size();
        return e;
    }

};

cr_batcher *cr_batcher_create(int device) {
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    cr_batcher *b = new cr_batcher();
    b->device = device;
    bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    for (int q = 0; ok && q < kDoneRing; ++q)
        ok = hipEventCreateWithFlags(&b->done[q], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        cr_batcher_destroy(b);
        return nullptr;
    }
    return b;
}

void cr_batcher_destroy(cr_batcher *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto &ev : b->done)
        if (ev) (void)hipEventDestroy(ev);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// The first fit thread to hand over a round becomes the leader: it waits (spinning, at most
// kGatherUs) until every active fit has handed over its round, launches them all, and marks each
// plan launched.  The other fit threads spin on their own plan's flag (thread hand-offs through
// condition variables cost tens of microseconds, as much as a small fit's whole iteration).
int cr_batcher_run(cr_batcher *b, TrialPlan *plan) {
    std::atomic<int> *flag = reinterpret_cast<std::atomic<int> *>(&plan->launched_flag);
    flag->store(0, std::memory_order_relaxed);
    bool lead = false;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->pending.push_back(plan);
        if (!b->leader) { b->leader = true; lead = true; }
    }
    if (lead) {
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(kGatherUs);
        std::vector<TrialPlan *> batch;
        for (;;) {
            {
                std::lock_guard<std::mutex> lk(b->mu);
                if ((int)b->pending.size() >= b->active || std::chrono::steady_clock::now() >= deadline) {
                    batch.swap(b->pending);
                    break;
                }
            }
            std::this_thread::yield();
        }
        const hipError_t e = b->launch(batch);
        {
            std::lock_guard<std::mutex> lk(b->mu);
            b->leader = false;
        }
        for (TrialPlan *p : batch) {
            p->status = e == hipSuccess ? CR_OK : CR_EDEVICE;
            reinterpret_cast<std::atomic<int> *>(&p->launched_flag)->store(1, std::memory_order_release);
        }
    } else {
        for (unsigned spins = 0; flag->load(std::memory_order_acquire) == 0; ++spins)
            if ((spins & 63) == 63) std::this_thread::yield();
    }
    return plan->status;
}

void cr_batcher_active(cr_batcher *b, int delta) {
    std::lock_guard<std::mutex> lk(b->mu);
    b->active += delta;
}

void cr_batcher_stats(cr_batcher *b, double *rounds, double *pass_launches, double *fit_rounds) {
    std::lock_guard<std::mutex> lk(b->mu);
    if (rounds) *rounds = b->rounds;
    if (pass_launches) *pass_launches = b->pass_launches;
    if (fit_rounds) *fit_rounds = b->fit_rounds;
}
