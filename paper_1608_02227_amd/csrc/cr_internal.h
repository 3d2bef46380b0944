// Internal state of one fit (shared by the C API and the serving loop).
#pragma once

#include "../../include/cr.h"
#include "cr_kernels.h"

#include <vector>

// Caller-provided device memory for one solver: every device buffer of the fit is carved from
// [base, base + size) in 256-byte aligned pieces instead of being allocated.  With `counting` set
// nothing is carved; `off` only adds up what the fit would take.
struct cr_workspace {
    char *base = nullptr;
    size_t size = 0;
    size_t off = 0;
    bool counting = false;
    // the most recent piece carved and the offset before it: releasing that piece (a temporary
    // staging buffer) gives its bytes back
    char *last = nullptr;
    size_t last_off = 0;
};

struct cr_batcher;

// One fit's trial round (pass, finalize, reduction with the step decision, queued update) handed
// to a cr_batcher, which launches the rounds of all fits waiting at that moment grouped.
struct TrialPlan {
    cr::Geometry g{};
    cr::PassMode mode = cr::PASS_TRIAL;
    bool fp32 = false;
    cr::LamRep rep = cr::REP_F64;
    cr::PassArgs pass{};
    cr::TrialFinalizeArgs fin{};
    cr::TrialReduceArgs red{};
    cr::AcceptArgs acc{};
    hipEvent_t ready = nullptr;   // recorded on the fit's stream behind the work the round reads
    hipEvent_t done = nullptr;    // set by the batcher: recorded behind the round's launches
    alignas(4) int launched_flag = 0;   // set (atomically) once the round is launched
    int status = CR_OK;
};

// Groups the adaptive step's trial rounds of several fits (serving): the rounds of the fits
// currently iterating are gathered and launched as grouped kernels on the batcher's stream.
cr_batcher *cr_batcher_create(int device);
void cr_batcher_destroy(cr_batcher *b);
// Blocks until the plan's round has been launched; then plan->done orders the fit's next work.
int cr_batcher_run(cr_batcher *b, TrialPlan *plan);
// A fit enters (+1) or leaves (-1) its iterations: a round waits (briefly) for every active fit.
void cr_batcher_active(cr_batcher *b, int delta);
// Rounds, grouped pass launches and fit rounds launched so far.
void cr_batcher_stats(cr_batcher *b, double *rounds, double *pass_launches, double *fit_rounds);

struct cr_solver {
    cr::Geometry g{};
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    cr_options opt{};
    double delta = 1.0;
    double scale = 1.0;          // S_y = max(1, max ybar - min ybar)
    int precision = CR_FP64;     // requested mode
    cr::LamRep rep = cr::REP_F64;  // current multiplier representation
    bool fp32pass = false;       // current pass arithmetic is FP32

    // device buffers (padded as described by Geometry)
    // Multiplier buffers (FP64 matrix, or FP32 low part against lam_hi).  Roles: lam[cur] = lam^k,
    // lam[prv] = lam^{k-1}; the FP64 storing trial pass writes its two candidates to lam[fa],
    // lam[fb] (the re-forming forms store none).
    void *lam[4] = {nullptr, nullptr, nullptr, nullptr};
    int prv = 1, fa = 2, fb = 3;
    void *lam_hi = nullptr;              // split: shared high part
    double *ubase = nullptr, *wbase = nullptr;   // split: FP64 C^T H
    double *xhat64 = nullptr, *ybar64 = nullptr;
    double *y64 = nullptr, *xi64 = nullptr, *dmy64 = nullptr;      // eta^{k+1} for the next step
    float *xhat32 = nullptr, *y32 = nullptr, *xi32 = nullptr, *dmy32 = nullptr;
    // Re-forming forms of the adaptive step (split modes; FP64 with reform_fp64): the accepted
    // candidate is not stored by its trial pass; the next pass re-forms it from the two stored
    // iterates, the accepted step and the pass arrays of that trial, kept here (swapped with the
    // current ones at each acceptance; the FP32 copies in mixed modes).
    double *yo64 = nullptr, *xio64 = nullptr, *dmyo64 = nullptr;
    float *yo32 = nullptr, *xio32 = nullptr, *dmyo32 = nullptr;
    bool pend = false;          // an accepted iterate lam^k is not yet stored
    double pend_beta = 0.0;     // its lam~ = lam[cur] + pend_beta (lam[cur] - lam[prv])
    double pend_invs = 0.0;     // and its step 1 / s_k
    double adv_passes = 0.0;    // re-forming trial passes launched
    bool deferred() const { return adaptive && (rep != cr::REP_F64 || opt.reform_fp64 != 0); }
    // FP64 buffers the adaptive step's storing trial pass needs (two iterates + two candidates)
    int fp64_buffers() const { return adaptive && opt.reform_fp64 == 0 ? 4 : 2; }
    double *yc = nullptr, *xic = nullptr, *dmyc = nullptr;         // eta(lam^k) for tests/output
    double *yr = nullptr, *xir = nullptr, *dmyr = nullptr;         // scratch primal (repair, prime)
    double *rowred = nullptr;
    void *part_acc = nullptr, *part_col = nullptr;
    // adaptive step: second set of partials, adjoints of the two candidate differences, and the
    // FP64 primal points eta(lam^k) (index ecur) and eta(lam^{k-1}) (index 1 - ecur)
    void *part_acc2 = nullptr, *part_col2 = nullptr;
    double *block_part = nullptr;   // per-block sums of the trial finalize
    double *decision = nullptr;     // the trial reduction's step decision (device, 4 values)
    // K-block partial dualization (options.block_size > 1): block size, the block IPM's workspace
    // and its iteration counts per block
    int blk = 0;
    double *blk_ws = nullptr;
    int *blk_iters = nullptr;
    bool blk_warm = false;          // a Step 1 has run: its slacks and multipliers start the next
    unsigned timing_tick = 0;       // samples one in four trial launches for the pass timing
    double *uD[2] = {nullptr, nullptr}, *wD[2] = {nullptr, nullptr};
    double *ye[2] = {nullptr, nullptr}, *xie[2] = {nullptr, nullptr}, *dmye[2] = {nullptr, nullptr};
    int ecur = 0;
    bool adaptive = false;
    double upsilon = 2.0;
    double s_step = 0.0;         // s_k of the adaptive rule (starts at L)
    double trials = 0.0;
    double restarts = 0.0;
    double xspan = 0.0;          // max |x - mean(x)| (certificate tie test)
    double xi_sq = 0.0;          // ||xi(lam^k)||^2 at the last stopping test
    // own-slope repair of the certificate: height potentials (ping-pong), per-block change counts
    static constexpr int kOwnRounds = 16;
    double *cpot[2] = {nullptr, nullptr};
    double *changed = nullptr;
    bool own_converged = false;
    int own_rounds = 0;
    double *part_red = nullptr, *part_min = nullptr;
    int *part_arg = nullptr;
    double *scal = nullptr;
    double *h_scal = nullptr;    // pinned; h_scal[24] holds the trial sequence word
    unsigned long long trial_seq = 0;
    unsigned long long *h_seq() const { return reinterpret_cast<unsigned long long *>(h_scal + 24); }
    int wait_trial(unsigned long long seq);
    std::vector<void *> owned;
    // Workspace mode (set before the state is allocated): buffers come from `ws`, release() does
    // nothing, no events are created (no pass timing), and the FP64 promotion takes place only if
    // the rest of the workspace holds the FP64 copy of the multipliers.  Without pinned host memory (`h_pinned` false)
    // the trial scalars are read back by a copy and a stream synchronization instead of polling.
    cr_workspace *ws = nullptr;
    bool h_pinned = true;
    bool h_owned = false;           // h_scal was allocated by the solver (hipHostMalloc)
    double *in_x = nullptr, *in_y = nullptr, *in_mu = nullptr;   // input staging (set-up only)
    double h_local[32] = {};
    double *trial_out = nullptr;    // device copy of the trial scalars when h_scal is not pinned
    // grouped trial rounds (serving): the adaptive step hands its rounds to `batch` (needs pinned
    // h_scal); ev_ready orders them behind this fit's stream
    cr_batcher *batch = nullptr;
    hipEvent_t ev_ready = nullptr;

    // iteration state
    double L = 0.0, sigma2 = 0.0, preprocess_s = 0.0;
    int power_iters = 0;
    int64_t k = 0, k_low = 0, checked_k = -1;
    // column walking direction of the next multiplier sweep (alternates, see PassArgs::rev)
    int sweep_rev = 0;
    int next_sweep() { const int r = sweep_rev; sweep_rev ^= 1; return r; }
    // the last stopping test's device results (eta(lam^k) in yc / xic / dmyc, the KKT reductions in
    // scal[0..5]) still describe the current iterate; cleared by anything that moves it
    bool test_fresh = false;
    // lam is still the zero start: its stopping report is known in closed form (below)
    bool lam_zero = true;
    double yrange = 0.0;         // max ybar - min ybar
    float xscale = 1.f;          // 2^-e with max |Xhat| (ones column included) in [2^(e-1), 2^e)
    int cur = 0;                 // buffer holding lam^k
    double t = 1.0;              // t_{k+1}
    double beta_last = 0.0;      // beta_k (0 before the first iteration)
    bool primed = false;
    cr_report last_report{};

    // sampled device time of the fused pass (events on `stream`)
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    bool ev_pending = false, ev_pending_low = false;
    double step_ms_sum[2] = {0.0, 0.0};   // [0] low precision, [1] FP64
    double step_n[2] = {0.0, 0.0};
    void collect_timing();

    ~cr_solver();
    int alloc(void **p, size_t bytes);
    int allocate_state(int64_t N, int64_t n);   // every device buffer of the fit
    void release(void *p);
    int adjoint_to(int idx, double *y, double *xi, double *dmy, bool with_rowred, float *y32_, float *xi32_,
                   float *dmy32_);
    int rebase(bool *eta_in_yc = nullptr);
    int prime();
    int step_once();
    int step_adaptive();
    int refresh_eta(bool have_cur_in_yc);
    int materialize();
    int lambda_rows_via_scratch(double *lambda);
    int project_blocks(double *y, double *xi, double *dmy, bool with_rowred, double *lam_out);
    int lipschitz(double *L, double *s2, int32_t *it);
    int check(cr_report *rep, bool certificate);
    int promote();
    int solve(double tol, cr_report *rep);
};

// ws: optional workspace (see cr_workspace); pinned_scal: optional host array of 32 doubles in
// pinned memory for the scalar read-backs (null: the solver allocates its own, or, in workspace
// mode, uses an unpinned array of its own).
int cr_solver_create_impl(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                          const cr_options *opt, const double *lambda0, bool on_device, cr_solver **out,
                          cr_workspace *ws = nullptr, double *pinned_scal = nullptr);
// Device bytes a fit of this shape and these options takes from a workspace (exact, including the
// 256-byte alignment of every piece), with `promotion` also the FP64 copy a mixed-precision fit
// takes if it promotes; 0 if the arguments are invalid.
size_t cr_workspace_bytes(int64_t N, int64_t n, const cr_options *opt, int device, bool promotion = false);
// One complete fit (the body of cr_fit / cr_fit_device), optionally inside a workspace.
// batch/ev_ready (optional): group the adaptive step's trial rounds through `batch`, ordering
// them behind the fit's stream with the caller's event ev_ready.
int cr_fit_impl(int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
                const cr_options *opt, double *y, double *xi, double *lambda, cr_report *rep, bool dev,
                cr_workspace *ws = nullptr, double *pinned_scal = nullptr, cr_batcher *batch = nullptr,
                hipEvent_t ev_ready = nullptr);
size_t cr_state_bytes(int64_t N, int64_t n, int precision, bool adaptive);

namespace cr {
// y = cya ya + cyb yb, xi = cxa xia + cxb xib, dmy = xi^T x - y (FP64); float copies when given.
hipError_t launch_lincomb(const Geometry &g, const double *ya, const double *xia, const double *yb,
                          const double *xib, double cya, double cyb, double cxa, double cxb, const double *xhat64,
                          double *y, double *xi, double *dmy, float *y32, float *xi32, float *dmy32, hipStream_t st);
}  // namespace cr
