/*
 * cr.h - C ABI of libcr: dual-smoothing (P-APG) least-squares convex regression on one
 * MI355X (gfx950) GPU.
 *
 * Problem (Aybat & Wang, arXiv:1608.02227, Section 2.1, eq. "regularize"): given locations
 * x_1..x_N in R^n and observations ybar_1..ybar_N, find fitted values y in R^N and
 * subgradients xi_1..xi_N in R^n minimizing
 *     1/2 sum_l (y_l - ybar_l)^2 + delta/2 sum_l ||xi_l||^2
 * subject to the N(N-1) pair constraints  y_j - y_i + xi_i^T (x_i - x_j) >= 0,  i != j
 * (eq. "original"; Definition "def:A1A2" orders the pairs lexicographically).  delta is the
 * Tikhonov weight the paper calls gamma.
 *
 * Method: P-APG (Fig. "fig:papg") with every pair constraint dualized (each point its own
 * block).  Step 1 is then closed-form: y = ybar + A1^T lam~, xi = A2^T lam~ / delta; Step 2 is
 * the projected dual step lam = (lam~ - C eta / L)_+; Steps 3-4 are the FISTA momentum.  The
 * Lipschitz constant is L = sigma_max(C)^2 / delta (eq. "eq:lischitz"), estimated by power
 * iteration unless the caller supplies it.  The multipliers lam are an N x N matrix whose
 * entry (i, j) belongs to the constraint of pair (i, j); the diagonal is always 0.
 *
 * Conventions for every entry point:
 *   - Arrays are row-major and dense: x is N x n, xi is N x n, lam is N x N.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory on the
 *     options' device.  The library copies what it needs; it keeps no caller pointer after a
 *     call returns (serving entry points copy inputs at submission).
 *   - Return value: CR_OK (0) or a negative CR_E* code; cr_strerror() names it.  Outputs are
 *     left untouched on CR_EINVAL / CR_ENOMEM / CR_EDEVICE.  On CR_ENOCONV and CR_ENUMERIC the
 *     outputs and the report describe the last iterate.
 *   - Thread safety: separate solvers and contexts may be used from separate threads; one
 *     solver or context must not be used by two threads at once.
 */
#ifndef CR_H
#define CR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CR_OK 0
#define CR_EINVAL (-1)   /* bad argument: N < 1, n < 1, delta <= 0, tol <= 0, non-finite data */
#define CR_ENOMEM (-2)   /* device memory (or a context's byte budget) cannot hold the state */
#define CR_ENOCONV (-3)  /* iteration or time budget exhausted before the tolerance */
#define CR_ENUMERIC (-4) /* NaN or Inf met in the iterates */
#define CR_EDEVICE (-5)  /* a HIP call failed, or no gfx950 device */
#define CR_EAGAIN (-6)   /* serving: the request has not finished yet */
#define CR_ENOTFOUND (-7)/* serving: unknown request id */
#define CR_ECANCELED (-8)/* serving: the context was destroyed before the request ran */

/* Arithmetic of the multiplier state and of the pair pass. */
typedef enum {
    CR_FP64 = 0,        /* lam stored in FP64, FP64 pair pass (FP64 MFMA contractions)          */
    CR_MIXED_FP32 = 1,  /* lam = H + l: shared FP32 high part, FP32 low part per iterate; FP32    */
                        /* MFMA pair pass; FP64 stopping test, adjoint of H and re-basing at each  */
                        /* test; FP64 refinement (promotion) only if progress stalls               */
    CR_MIXED_BF16 = 2   /* as CR_MIXED_FP32 with the shared high part H stored in BF16           */
} cr_precision;

typedef struct {
    int32_t precision;       /* cr_precision; default CR_FP64 */
    int32_t check_every;     /* stopping test every m iterations; default 50 */
    int64_t max_iters;       /* iteration budget; default 2,000,000 */
    double time_budget_s;    /* wall-clock budget of the iteration loop; 0 = none */
    double L;                /* > 0: use this Lipschitz constant; 0: power iteration (default) */
    int32_t power_max_iters; /* power-iteration cap; default 300 */
    double power_rtol;       /* power-iteration relative stopping change; 0 (default): 1e-8 with the
                                constant step, 1e-2 with the adaptive step (which only starts from
                                s_0 = L and checks every step) */
    int32_t momentum;        /* 1: P-APG (default); 0: plain projected dual gradient ascent */
    int32_t certificate;     /* 1: compute the feasible repair and certified gap (default 1) */
    int32_t device;          /* HIP device ordinal; default 0 */
    void *stream;            /* hipStream_t to run on; NULL: the library's own stream */
    int32_t stall_checks;    /* mixed modes: switch to FP64 after this many consecutive stopping
                                tests without a new lowest KKT residual; default 100 */
    int32_t step_rule;       /* 1 (default): adaptive step of the paper's eq. "eq:adaptive-check"
                                (PAPG_A) with s_0 = L and s_k = s_{k-1} upsilon^(l_k - 1);
                                0: constant step 1/L (PAPG_C) */
    double upsilon;          /* adaptive step factor (> 1); default 2 */
    int32_t restart;         /* adaptive step only. 1: reset the momentum (t := 1) after an iteration
                                whose accepted step opposes its own movement,
                                <lam^{k+1} - lam~^{k+1}, lam^{k+1} - lam^k> < 0 (gradient restart
                                of O'Donoghue and Candes); 0: the paper's schedule unchanged.
                                Default 1 */
    int32_t stop_rule;       /* 0 (default): stop when report.kkt <= tol; 1: stop when the certified
                                gap report.cert_gap <= tol, i.e. the multipliers are tol-optimal for
                                the dual (the inner test of the continuation, Section 2.4.1) */
    int32_t check_rule;      /* 1 (default): after a test that improved on the previous one, the next
                                comes where a geometric decay through the two would reach tol, but
                                no sooner than check_every / 5 (at least 1) and no later than
                                check_every iterations; 0: a test every check_every iterations */
    int32_t reform_fp64;     /* FP64 mode with the adaptive step.  0 (default): the trial pass stores
                                both candidates (reads 2, writes 2 FP64 iterates: 32 B per pair;
                                three FP64 contractions); 1: the next trial pass re-forms the
                                accepted candidate instead (24 B per pair, a fourth FP64
                                contraction).  The FP64 matrix cores bound that pass, so the
                                default is the faster one (measured at N = 8000, n = 40: 0.49 ms
                                against 0.52 ms).  The split modes always re-form. */
    int32_t center;          /* mixed modes: 1 (default) works in the frame x - mean(x) (every pair
                                constraint and the adjoint depend only on differences x_i - x_j, so
                                y, xi and lam are the same, and the FP32 residual loses less to
                                cancellation); 0 keeps the caller's coordinates.  FP64 mode always
                                keeps them. */
    int32_t keep_lambda;     /* serving (cr_submit): 1 keeps the request's final multipliers (N x N
                                FP64, host) until they are collected through the lambda argument of
                                cr_wait / cr_poll; 0 (default) drops them.  Ignored elsewhere. */
    int32_t block_size;      /* 0 (default): every pair constraint dualized (each point its own
                                block).  p in [2, 100]: K-block partial dualization (Section 2.1):
                                contiguous blocks of p points (the last may be shorter; at least two
                                blocks), only the pairs between blocks dualized, and Step 1 solving
                                each block's QP (eq. "eq:step1-problem") by a primal-dual interior-
                                point method on the device (each Step 1 after a solver's first starts
                                from the slacks and multipliers the previous one ended on, lifted
                                into the interior).  Needs CR_FP64 and the constant step
                                (step_rule 0).  The returned multipliers are then theta (between
                                blocks) plus the blocks' own multipliers (inside the blocks); a warm
                                start's entries inside the blocks are ignored. */
    int32_t reserved2;
    const double *lambda0;   /* optional N x N warm start lam^0 (its diagonal is ignored; entries
                                must be finite and >= 0, else CR_EINVAL), in the memory of the call's
                                other inputs: host for cr_fit / cr_fit_continuation / cr_submit (which
                                copies it), device for cr_fit_device / cr_fit_device_noalloc.  NULL
                                (default): lam^0 = 0 (Theorem "bound").  cr_solver_create's own
                                lambda0 argument, when given, takes precedence. */
} cr_options;

typedef struct {
    int32_t status;          /* CR_OK, CR_ENOCONV or CR_ENUMERIC */
    int32_t precision;       /* precision mode used */
    int64_t iters;           /* P-APG iterations taken */
    int64_t iters_low;       /* of which in the low-precision phase (mixed modes) */
    double seconds;          /* wall time of the whole fit, preprocessing included */
    double preprocess_seconds; /* wall time of the Lipschitz estimate */
    double L;                /* Lipschitz constant used */
    double sigma2;           /* sigma_max(C)^2 estimate (0 when L was given) */
    int32_t power_iters;     /* power iterations taken */
    int32_t checks;          /* stopping tests evaluated */
    /* Stopping quantities at the returned multipliers, all divided by
       S_y = max(1, max ybar - min ybar):
         kkt = max(max_ij |min(lam_ij, s_ij)|, stat_y, stat_xi) with s = C eta(lam). */
    double kkt;
    double nat_res_max;      /* max_ij |min(lam_ij, s_ij)| / S_y                           */
    double stat_y;           /* ||y - ybar - A1^T lam||_inf / S_y of the returned y            */
    double stat_xi;          /* ||delta xi - A2^T lam||_inf / (delta S_y) of the returned xi   */
    double max_viol;         /* max_ij (-s_ij)_+ / S_y                                       */
    double infeas_rms;       /* ||(C eta)_-||_2 / sqrt(N^2 - N)      (paper, Section 4.1)     */
    double dual_gap_paper;   /* |lam^T C eta| / (N^2 - N)            (paper, Section 4.1)     */
    double comp_sum;         /* sum_ij lam_ij s_ij                                           */
    double primal_obj;       /* r_delta(eta(lam))                                            */
    double dual_obj;         /* g_delta(lam) = primal_obj - comp_sum                          */
    double scale;            /* S_y */
    /* Certificate (options.certificate): the max-affine repair of eta(lam) is feasible, so
       cert_gap = r_delta(repair) - g_delta(lam) >= p* - g_delta(lam) >= 0 and, by the paper's
       Theorem "thm:rate", ||y(lam) - y*||_2 <= y_err_bound = sqrt(2 cert_gap). */
    double cert_primal;
    double cert_gap;
    double y_err_bound;
    /* Device time of the dominant fused pair pass, from HIP events recorded on the solver's
       stream: the constant step's pass, the FP64 adaptive step's trial pass, or the split forms'
       re-forming trial pass.  Average ms per launch and number of sampled launches, for the
       low-precision and the FP64 phase. */
    double step_ms_low;
    double step_ms_fp64;
    double step_samples_low;
    double step_samples_fp64;
    /* Adaptive step: the last accepted s_k (L for the constant step) and the number of Step-2
       candidates evaluated (two per fused trial pass). */
    double step_final;
    double trials;
    double restarts;         /* momentum restarts taken (options.restart) */
    double adv_passes;       /* split forms, adaptive step: trial passes that also re-formed and
                                stored the previous accepted iterate (the rest only read) */
} cr_report;

/* Fills *opt with the defaults listed above. */
void cr_default_options(cr_options *opt);

/* Name of a CR_* code (static string). */
const char *cr_strerror(int code);

/* Library version and device check: returns CR_OK when a gfx950 device `device` is usable. */
int cr_device_check(int device);

/*
 * cr_fit - one complete fit, host memory in and out.
 *   x      host, N x n, locations (read)
 *   ybar   host, N, observations (read)
 *   delta  Tikhonov weight (> 0)
 *   tol    stopping tolerance on report.kkt (> 0)
 *   opt    options or NULL for defaults
 *   y      host, N, fitted values of eta(lam) in FP64 (written)
 *   xi     host, N x n, subgradients of eta(lam) in FP64 (written)
 *   lambda host, N x N, final multipliers in FP64, or NULL (written)
 *   rep    report or NULL (written)
 * Runs: preprocess (Lipschitz constant), P-APG iterations with a stopping test every
 * opt->check_every iterations, FP64 recovery of (y, xi) from the final multipliers, and the
 * optional certificate.  N = 1 returns y = ybar, xi = 0 without touching the GPU.
 */
int cr_fit(int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
           const cr_options *opt, double *y, double *xi, double *lambda, cr_report *rep);

/* cr_fit_device - as cr_fit, but x, ybar, y, xi and lambda are device pointers on opt->device,
 * and all work runs on opt->stream (or the library's stream).  Returns after the result is
 * written. */
int cr_fit_device(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                  double tol, const cr_options *opt, double *y, double *xi, double *lambda,
                  cr_report *rep);

/*
 * cr_fit_device_noalloc - cr_fit_device without any allocation, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs and results as cr_fit_device (the same kernels in the same order, so
 * the results are bitwise equal), with these differences:
 *   - every device buffer of the fit is carved from a library-owned scratch array of
 *     cr_noalloc_scratch_bytes() bytes (128 MiB) that each device the library runs on holds until
 *     the process ends; a fit needing more (cr_noalloc_required_bytes) returns CR_ENOMEM before
 *     any device work.  The limit is N of about 2,600 in the mixed modes and about 1,700 in FP64
 *     with the adaptive step (n = 40).
 *   - no device or pinned host memory is allocated and no stream or event is created: all device
 *     work runs on opt->stream (NULL: the null stream); the pass-time fields of the report are 0.
 *   - the mixed modes promote to FP64 (the stalled-fit safety net) only if the rest of the scratch
 *     holds the FP64 copy of the multipliers (N up to about 1,500 at n = 40); otherwise they keep
 *     the split form.
 *   - the scratch keeps the previous call's contents; each call clears what it uses before use.
 *     Calls from several host threads on one device are serialized by the library (they would
 *     otherwise race on the shared array); other devices and other processes have their own copy.
 */
int cr_fit_device_noalloc(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                          double tol, const cr_options *opt, double *y, double *xi, double *lambda,
                          cr_report *rep);
/* Size of the scratch array of cr_fit_device_noalloc, and the bytes of it one fit needs
 * (0 for N = 1 or invalid arguments). */
size_t cr_noalloc_scratch_bytes(void);
size_t cr_noalloc_required_bytes(int64_t N, int64_t n, const cr_options *opt);

/*
 * Continuation to the unregularized least-squares estimator (Section 2.4.1).
 *   eps_t = eps0 / beta^t (beta > 1), outer iteration t = 1..T uses the Tikhonov weight
 *   gamma_t = kappa_gamma eps_t and computes a delta_t-optimal dual solution, delta_t =
 *   kappa_delta eps_t (certified gap <= delta_t), by P-APG started from the previous one
 *   (theta^(0) = 0).  L_gamma = sigma_max(C)^2 / gamma_t reuses one power iteration.  By the
 *   section's bound ||y^(t) - y*|| <= ||xi*|| sqrt(gamma_t) + sqrt(2 delta_t), y* the estimator
 *   of eq. "original" (xi* its least-norm subgradients).
 */
typedef struct {
    double eps0;             /* > 0 */
    double beta;             /* > 1 */
    double kappa_gamma;      /* > 0 */
    double kappa_delta;      /* > 0 */
    int32_t T;               /* outer iterations, >= 1 */
    int32_t reserved;
} cr_cont_params;

typedef struct {
    double gamma;            /* Tikhonov weight of this outer iteration */
    double delta;            /* its dual tolerance (certified-gap target) */
    int64_t iters;           /* inner P-APG iterations */
    int32_t status;          /* CR_OK (certified gap <= delta), CR_ENOCONV or CR_ENUMERIC */
    int32_t reserved;
    double cert_gap;         /* certified gap at the end of the inner iterations */
    double kkt;              /* KKT residual there (report.kkt) */
    double xi_norm;          /* ||xi^(t)||_2 of the returned subgradients */
    double seconds;          /* wall time of this outer iteration */
} cr_cont_step;

/*
 * cr_fit_continuation - host arrays as in cr_fit.  opt->max_iters and opt->time_budget_s apply to
 * each inner solve; opt->stop_rule is ignored (the certified gap is the inner test).  y, xi
 * (required) receive (y^(T), xi^(T)); lambda (optional, N x N) theta^(T); steps (optional, T
 * entries) one record per outer iteration; rep the report of the last inner solve with
 * iters = the total over all outer iterations.  Returns CR_OK when every inner solve reached its
 * tolerance, else the first failing inner status (the iterations go on with the next gamma_t
 * after CR_ENOCONV).
 */
int cr_fit_continuation(int64_t N, int64_t n, const double *x, const double *ybar, const cr_cont_params *cp,
                        const cr_options *opt, double *y, double *xi, double *lambda, cr_cont_step *steps,
                        cr_report *rep);

/* ---- Step-level entry points: a solver whose state stays on the device. ----------------- */
typedef struct cr_solver cr_solver;

/* Creates the device state for one fit (copies x and ybar, host pointers).  lambda0 is an
 * optional N x N host warm start (its diagonal is ignored), else lam^0 = 0 (Theorem "bound").
 * Device memory: two N^2 multiplier buffers of the precision's width plus O(N n). */
int cr_solver_create(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                     const cr_options *opt, const double *lambda0, cr_solver **out);
int cr_solver_destroy(cr_solver *s);

/* Preprocess: power iteration for sigma_max(C)^2; sets L = sigma2 / delta (eq. "eq:lischitz").
 * L, sigma2 and iters may be NULL. */
int cr_solver_lipschitz(cr_solver *s, double *L, double *sigma2, int32_t *iters);
/* Uses the given L (> 0) instead. */
int cr_solver_set_L(cr_solver *s, double L);

/* cr_solver_set_delta - change the Tikhonov weight of an existing solver (the continuation's
 * gamma_t): the multipliers are kept as the warm start, L becomes sigma_max(C)^2 / delta when the
 * power iteration has run (else it runs at the next solve), the FISTA sequence restarts (t = 1)
 * and the adaptive step restarts from s = L.  delta > 0 and finite, else CR_EINVAL. */
int cr_solver_set_delta(cr_solver *s, double delta);

/* Advances the P-APG iteration `iters` times (accepted iterations under the adaptive rule) in the
 * solver's current precision. */
int cr_solver_iterate(cr_solver *s, int64_t iters);

/* Runs iterations with stopping tests until report.kkt <= tol or a budget ends (cr_fit's loop).
 * Returns CR_OK, CR_ENOCONV or CR_ENUMERIC. */
int cr_solver_solve(cr_solver *s, double tol, cr_report *rep);

/* Switches the multiplier state to FP64 (a no-op in CR_FP64 mode). */
int cr_solver_promote(cr_solver *s);

/* Iteration counter k (number of completed iterations). */
int64_t cr_solver_iterations(const cr_solver *s);

/* Copies lam^k (N x N, FP64, host) out. */
int cr_solver_get_lambda(cr_solver *s, double *lambda);
/* Copies rows [row0, row0 + nrows) of lam^k (nrows x N, FP64, host) out; rows must lie in [0, N). */
int cr_solver_get_lambda_rows(cr_solver *s, int64_t row0, int64_t nrows, double *rows);
/* FP64 closed-form eta(lam^k) = (ybar + A1^T lam^k, A2^T lam^k / delta) to host. */
int cr_solver_get_primal(cr_solver *s, double *y, double *xi);
/* FP64 stopping report of lam^k (and the certificate if opt.certificate). */
int cr_solver_report(cr_solver *s, cr_report *rep);
/* K-block partial dualization (options.block_size = p > 1; Section 2.1, Step 1 split into the
 * blocks' QPs of eq. "subgradient_split"): *nblocks = ceil(N / p) (0 with every pair dualized), and,
 * when iters is not NULL, the interior-point iterations each block's QP took in the most recent
 * Step 1 (0 before the first), copied to the host array iters[0 .. *nblocks) after the solver's
 * stream has drained.  cap < *nblocks with iters given: CR_EINVAL. */
int cr_solver_block_iters(cr_solver *s, int32_t *iters, int64_t cap, int64_t *nblocks);

/* Tiling of the pair sweep for an N-point, n-feature fit on `device` (diagnostics and memory
 * probes): padded rows (= the multiplier arrays' leading dimension), column chunks per 128-row
 * strip, columns per chunk, and workgroups per pass. */
int cr_pass_geometry(int64_t N, int64_t n, int device, int32_t *rows, int32_t *chunks,
                     int32_t *chunk_cols, int32_t *workgroups);

/* ---- Operators on device data (one call each; device pointers, synchronous). ------------ */
/* s = C eta: s_ij = y_j - y_i + xi_i^T (x_i - x_j), zero diagonal; s is N x N (Def. "def:A1A2"). */
int cr_op_residual(int64_t N, int64_t n, const double *x, const double *y, const double *xi,
                   double *s, int device);
/* (u, w) = C^T lam: u = colsum - rowsum, w_m = rowsum_m x_m - (Lam X)_m (Section 2.5). */
int cr_op_adjoint(int64_t N, int64_t n, const double *x, const double *lam, double *u, double *w,
                  int device);

/* ---- Serving: continuous batching of fits on one device. --------------------------------- */
typedef struct cr_ctx cr_ctx;

/* byte_budget: device bytes the resident state of all admitted fits may use (0 = 80% of free
 * device memory); max_slots: fits resident at once.  Each slot owns a stream, a small pinned
 * host buffer and a device arena that grows to the largest fit the slot has run and is then
 * reused (fits allocate nothing while the arena is large enough); the arenas are freed by
 * cr_ctx_destroy.  The context takes no caller stream: its fits overlap on the device because
 * each slot runs on a stream of its own, and one shared stream would serialize them (a single
 * fit on a caller's stream is cr_fit_device with opt->stream). */
int cr_ctx_create(int device, size_t byte_budget, int32_t max_slots, cr_ctx **out);
/* Running fits finish; queued ones are dropped and their waiters (cr_wait) return CR_ECANCELED.
 * Returns once no thread is inside a call on ctx any more; ctx is then invalid. */
int cr_ctx_destroy(cr_ctx *ctx);
/* Queues a fit (copies x, ybar and a warm start opt->lambda0); non-blocking.  Returns its id in
 * *req_id. */
int cr_submit(cr_ctx *ctx, int64_t N, int64_t n, const double *x, const double *ybar,
              double delta, double tol, const cr_options *opt, int64_t *req_id);
/* Non-blocking: CR_EAGAIN while running, else the fit's status; results copied out once, after
 * which the id is unknown.  y (N), xi (N x n), rep, latency_s (submission to completion) may each
 * be NULL.  lambda (N x N, host) receives the final multipliers and needs the request to have been
 * submitted with opt->keep_lambda = 1; otherwise a non-NULL lambda returns CR_EINVAL and leaves the
 * result in place. */
int cr_poll(cr_ctx *ctx, int64_t req_id, double *y, double *xi, double *lambda, cr_report *rep,
            double *latency_s);
/* Blocking version of cr_poll. */
int cr_wait(cr_ctx *ctx, int64_t req_id, double *y, double *xi, double *lambda, cr_report *rep,
            double *latency_s);
/* Device bytes the serving context reserves for one fit of this shape and precision with the
 * default step rule (its whole device state: the multiplier iterates, the partial sums and the
 * O(N n) vectors; mixed modes include the FP64 copy a promotion would take).  Admission requires
 * the sum over running fits to fit the budget. */
size_t cr_fit_state_bytes(int64_t N, int64_t n, int32_t precision);

/* Counters: fits queued, running, finished; bytes of multiplier state resident. */
int cr_ctx_stats(cr_ctx *ctx, int64_t *queued, int64_t *running, int64_t *finished,
                 size_t *resident_bytes);
/* Grouped iterations (off by default): fits admitted from now on with N <= max_n (0 = off) using
 * the adaptive step hand each iteration's trial round (the pair sweep, its finalize, the step
 * decision and the update) to the context's batcher, which launches the rounds of all such fits
 * iterating at that moment as grouped kernels on one stream (one launch per kernel variant instead
 * of one per fit).  Results are bitwise those of the fit run alone.  On one MI355X per-slot
 * streams retire more fit iterations per second (the rounds of different fits overlap on the
 * device; grouped rounds run in lockstep), hence the default. */
int cr_ctx_set_grouping(cr_ctx *ctx, int64_t max_n);
/* Counters of the grouped iterations: rounds launched, grouped pass launches, and the fit rounds
 * they carried. */
int cr_ctx_group_stats(cr_ctx *ctx, double *rounds, double *pass_launches, double *fit_rounds);

#ifdef __cplusplus
}
#endif
#endif /* CR_H */
