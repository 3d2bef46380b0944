// Internal launch interface of the gfx950 kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cr {

// Representation of the N x N multiplier state.
//   REP_F64        : one FP64 matrix per iterate.
//   REP_SPLIT_F32  : lam = H + l with a high part H (FP32) shared by the two stored iterates and
//                    one FP32 low part per iterate (16 bytes per pair per iteration instead of 24).
//   REP_SPLIT_BF16 : the same with H in BF16 (14 bytes per pair per iteration).
// The split forms keep FP64-level resolution of the small per-iteration updates (steps of
// s/L can be 1e-11 against multipliers of 1e-2), which a plain FP32 matrix rounds away.
enum LamRep : int { REP_F64 = 0, REP_SPLIT_F32 = 1, REP_SPLIT_BF16 = 2 };

// What one sweep over the pairs computes (all modes form the residual tile s = C eta except
// ADJ and REBASE).
enum PassMode : int {
    PASS_STEP = 0,   // Steps 2-4 fused with the adjoint of the next extrapolated point
    PASS_ADJ = 1,    // adjoint C^T lam of a stored multiplier matrix
    PASS_KKT = 2,    // stopping-test reductions at a stored multiplier matrix
    PASS_POWER = 3,  // z = C v and C^T z (power iteration), plus ||z||^2
    PASS_REPAIR = 4, // column minima of s and their arg-min rows (max-affine repair)
    PASS_RESID = 5,  // writes s = C eta (FP64, zero diagonal and padding) into lam_b
    PASS_REBASE = 6, // split forms: H <- round(H + l_k), both low parts re-expressed against the
                     // new H, and the FP64 adjoint of the new H (cached for the constant step) or,
                     // with rebase_lam, of lam^k
    PASS_TRIAL = 7,  // adaptive step: two Step-2 candidates lam~ - s / s_a and lam~ - s / s_b from
                     // one read of the iterates, written to lam_c / lam_d, with the adjoints of
                     // D = candidate - lam~ (part_acc / part_acc2), ||D||^2 (part_red slots 0, 1)
                     // and <D, candidate - lam^k> (slots 2, 3)
    PASS_TRIAL_NS = 8, // PASS_TRIAL without storing the candidates (split forms; the accepted one
                       // is re-formed by the next PASS_ADV)
    PASS_ADV = 9     // split forms: first re-form the accepted candidate of the previous trial,
                     // lam^k = (lam~^k - s(eta~^k) / s_k)_+ from lam_a = lam^{k-1}, lam_b = lam^{k-2},
                     // beta_prev, inv_Lo and the previous pass arrays (xi_o, yv_o, dmy_o), store it
                     // over lam_b, then run PASS_TRIAL_NS from (lam^k, lam^{k-1}) with beta_next
};

// Tiling shared by host and device code.
#ifndef CR_WAVES
#define CR_WAVES 8
#endif
constexpr int kWaves = CR_WAVES;         // waves per workgroup
constexpr int kRows = 16 * kWaves;       // rows i per workgroup (one 16-row MFMA block per wave)
constexpr int kSuper = 64;               // columns j staged in LDS per step
constexpr int kMaxMB = 4;                // feature blocks of 16: n + 1 <= 64
constexpr int kRed = 4;                  // reduction slots per workgroup

struct Geometry {
    int N;          // points
    int n;          // features
    int NP;         // padded feature stride: 16 * MB >= n + 1 (column n of xhat holds 1)
    int MB;         // NP / 16
    int ks1;        // ceil(n / 4): K-steps of the residual contraction
    int Nr;         // padded rows (multiple of kRows); also the padded column count ld
    int ld;         // leading dimension of the multiplier buffers (== Nr)
    int strips;     // Nr / kRows
    int chunks;     // column chunks per strip (workgroups per strip)
    int chunk_cols; // columns per chunk (multiple of kSuper)
    int grid() const { return strips * chunks; }
};

// Tiling of an N-point fit.  `slots` is the number of workgroups the device runs at once (compute
// units x resident workgroups per unit); the column chunk count is chosen so that the workgroup
// count fills whole rounds of `slots` as evenly as possible, preferring fewer chunks (less
// partial-sum traffic).  slots <= 0 uses 256.
Geometry make_geometry(int N, int n, int slots = 0);

// One sweep over all pairs.  T is the arithmetic type of the contraction and epilogue; the
// multipliers use representation `rep`.  Pointer roles (all device, padded as in Geometry):
//   lam_h   : split forms: the shared high part H (FP32 or BF16), Nr x ld
//   lam_a   : REP_F64: lam^{k-1} (STEP) or the multipliers to read (ADJ, KKT);
//             split: the FP32 low part of lam^{k-1} (STEP), of lam (ADJ, KKT), of lam^k (REBASE)
//   lam_b   : REP_F64: lam^{k-2} in, lam^k out (STEP); s out (RESID);
//             split: low part of lam^{k-2} in, of lam^k out (STEP); of lam^{k-1} (REBASE)
//   xhat    : Nr x NP locations of type T; column n is 1 for real rows, padding is 0
//   xi      : Nr x NP subgradients (or the power vector's xi part), type T, zero padded
//   yv      : Nr fitted values (or the power vector's y part), type T
//   dmy     : Nr values d_i - y_i with d_i = xi_i^T x_i, type T
//   part_acc: chunks x Nr x NP partial (Lam X) rows of type T; column n holds row sums
//   part_col: strips x ld partial column sums of type T
//   part_red: grid x kRed double reductions (KKT: max nat, max viol, sum neg^2, sum lam s;
//             POWER: sum z^2)
//   part_min / part_arg: strips x ld column minima and arg-min rows (REPAIR)
struct PassArgs {
    void *lam_h;
    const void *lam_a;
    void *lam_b;
    const void *xhat;
    const void *xi;
    const void *yv;
    const void *dmy;
    void *part_acc;
    void *part_col;
    double *part_red;
    double *part_min;
    int *part_arg;
    double beta_prev;   // beta_{k-1}: lam~^k = lam^{k-1} + beta_{k-1} (lam^{k-1} - lam^{k-2})
    double beta_next;   // beta_k:     lam~^{k+1} = lam^k + beta_k (lam^k - lam^{k-1})
    double inv_L;       // 1 / L (TRIAL: 1 / s_a)
    // PASS_TRIAL only
    void *lam_c;        // candidate a (REP_F64: matrix; split: low part against lam_h)
    void *lam_d;        // candidate b
    double inv_L2;      // 1 / s_b
    void *part_acc2;    // adjoint partials of candidate b's difference
    void *part_col2;
    // PASS_ADV only: pass arrays of the previous trial and its accepted step
    const void *xi_o;
    const void *yv_o;
    const void *dmy_o;
    double inv_Lo;      // 1 / s_k of the accepted candidate being re-formed
    // PASS_REPAIR only (optional): per-row offsets c_i; the pass then takes column minima of
    // s_ij - c_i (the relaxation rounds of the own-slope repair)
    const double *row_off;
    // PASS_REBASE only: 0 accumulates the adjoint of the new high part H', 1 that of lam^k as
    // stored after the re-basing (H' + l_k')
    int rebase_lam;
    // 1: every workgroup walks its column chunk from the end back to the start (the fit alternates
    // the direction from one multiplier sweep to the next, so that a sweep starts on the lines the
    // previous one touched last, which the last-level cache still holds)
    int rev;
    // split trial passes: the power of two that scales the fit's locations (Xhat, ones column
    // included) into [0.5, 1) for the FP16 residual
    float x_scale;
    // > 1: K-block partial dualization with blocks of `blk` consecutive points; the pass treats the
    // pairs inside a block like the diagonal (no multiplier, no contribution)
    int blk;
};

hipError_t launch_pass(const Geometry &g, PassMode mode, bool fp32, LamRep rep,
                       const PassArgs &a, hipStream_t st);

// Finalize: turn the partial sums of one sweep into the primal point.
//   PRIMAL: y = ybar + (c - r), xi_m = (r x_m - (Lam X)_m) / delta, dmy = xi^T x - y
//   POWER : y = (c - r), xi_m = r x_m - (Lam X)_m (C^T z), dmy likewise
// Inputs: the partials of type T (fp32 flag), xf (Nr x NP, FP64 locations matching the pass),
// ybar (Nr).  Outputs: FP64 y, xi, dmy (Nr, Nr x NP, Nr); optional float copies y32/xi32/dmy32
// (may be null); rowred (Nr x 2: (y - ybar)^2 or y^2, and ||xi||^2), may be null.
//   ubase/wbase (optional, FP64 Nr / Nr x NP): adjoint of a cached high part, added to the
//   partial sums before the primal formula (split representations).
struct FinalizeArgs {
    const void *part_acc;
    const void *part_col;
    const double *xf;
    const double *ybar;
    const double *ubase;
    const double *wbase;
    double *y, *xi, *dmy;
    float *y32, *xi32, *dmy32;
    double *rowred;
    double inv_delta;
    int power;               // 1: POWER variant
};
hipError_t launch_finalize(const Geometry &g, bool fp32, const FinalizeArgs &a, hipStream_t st);

// Adjoints of both candidate differences of a trial pass (power-mode finalize, no ybar) and
// per-block partial sums (||A1^T D_0||^2, ||A2^T D_0||^2, ||A1^T D_1||^2, ||A2^T D_1||^2).
struct TrialFinalizeArgs {
    const void *part_acc[2];
    const void *part_col[2];
    const double *xf;       // Xhat, FP64, Nr x NP
    double *uD[2];          // Nr
    double *wD[2];          // Nr x NP
    double *block_part;     // (Nr / 16) x 4
};
hipError_t launch_trial_finalize(const Geometry &g, bool fp32, const TrialFinalizeArgs &a, hipStream_t st);

// What the trial reduction needs to take the step test's decision itself: the two candidates'
// s values, delta, the current t_k, and the restart and momentum options.
struct TrialRule {
    double s_a, s_b, delta, t;
    int restart, momentum;
};

// The eight trial scalars: out[0..3] = column sums of block_part ((Nr / 16) x 4), out[4..7] = sums
// of part_red slots 0..3 over the pass's workgroups; then the step test's decision in out[8..11]
// and, if `decision` is set, in device memory there too (candidate 0 / 1, -1 for neither, -2 for
// a non-finite scalar; beta_k; t_{k+1}; restart flag).  Single workgroup, fixed order; `out` may be
// pinned host memory.  If seq_out is set, `seq` is written there after the values are visible at
// system scope (a host polling pinned memory may then read them).
hipError_t launch_trial_reduce(const Geometry &g, const double *block_part, const double *part_red, double *out,
                               unsigned long long *seq_out, unsigned long long seq, const TrialRule &rule,
                               double *decision, hipStream_t st);


// Accepted adaptive step: eta(lam^{k+1}) from eta(lam~^{k+1}) (yt, xit) and the adjoint of D,
// then the next pass arrays (1 + beta) eta(lam^{k+1}) - beta eta(lam^k) into (y, xi, dmy).  With
// `decision` (the trial reduction's device output) the candidate and beta are taken from there and
// the launch does nothing when no candidate was accepted, so it can be queued before the host has
// seen the test; without it candidate 0 and `beta` are used.
hipError_t launch_accept(const Geometry &g, const double *yt, const double *xit, double *y, double *xi, double *dmy,
                         const double *const uD[2], const double *const wD[2], const double *yk, const double *xik,
                         double *ye, double *xie, double *dmye, float *y32, float *xi32, float *dmy32,
                         const double *xhat64, double inv_delta, double beta, const double *decision, hipStream_t st);

// ---- K-block partial dualization: Step 1's block QPs (cr_blocks.hip) -----------------------
// Points per block at most (the IPM keeps a block's Schur complement and locations in LDS).
constexpr int kMaxBlock = 100;
// One launch projects the closed-form point of every block of p consecutive points (the last block
// may be shorter) onto the block's pair constraints in the norm of diag(I, delta I), by a
// primal-dual interior-point method per block (one workgroup each).  y, xi (padded rows, stride NP)
// hold the closed-form point in and the projection out; dmy receives xi^T x - y; rowred (optional)
// the rows' (y - ybar)^2 and ||xi||^2; lam (optional, leading dimension ld) the blocks' multipliers in
// the intra-block entries; iters (optional, one int per block) the IPM iterations taken.
struct BlockProjArgs {
    const double *xhat;
    double *y, *xi, *dmy;
    const double *ybar;
    double *rowred;
    double *lam;
    int ld;
    double *ws;               // workspace: blocks x ws_doubles
    size_t ws_doubles;        // block_ws_doubles(p, n)
    int *iters;
    double delta, tol;
    int N, n, NP, p, max_iter;
    int warm;                 // the workspace holds the previous Step 1's slacks and multipliers
};
size_t block_ws_doubles(int p, int n);
hipError_t launch_block_project(const Geometry &g, const BlockProjArgs &a, hipStream_t st);

// ---- grouped launches (serving: the same step of several small fits in one launch) ----------
// Fit f of a group owns the launch's workgroups [off[f], off[f + 1]); its tiles, reductions and
// outputs are exactly those of its own launch, so results are bitwise the same grouped or alone.
// The descriptors travel as kernel arguments (no device memory), kGroupMax fits per launch.
constexpr int kGroupMax = 8;

struct PassGroup {
    int nfit;
    int off[kGroupMax + 1];
    Geometry g[kGroupMax];
    PassArgs a[kGroupMax];
};
// Fits can share a grouped pass when these agree: mode, arithmetic, representation, feature
// blocks and the residual K-step trim (the kernel's template parameters).
int pass_group_key(const Geometry &g, PassMode mode, bool fp32, LamRep rep);
hipError_t launch_pass_group(PassMode mode, bool fp32, LamRep rep, const PassGroup &G, hipStream_t st);

struct TrialFinalizeGroup {
    int nfit;
    int off[kGroupMax + 1];
    Geometry g[kGroupMax];
    TrialFinalizeArgs a[kGroupMax];
};
// All fits of the group share fp32 and MB.
hipError_t launch_trial_finalize_group(bool fp32, int MB, const TrialFinalizeGroup &G, hipStream_t st);

struct TrialReduceArgs {
    const double *block_part;
    int nblk;                 // Nr / 16
    const double *part_red;
    int nred;                 // the pass's workgroup count
    double *out;
    unsigned long long *seq_out;
    unsigned long long seq;
    TrialRule rule;
    double *decision;
};
struct TrialReduceGroup {
    int nfit;
    TrialReduceArgs a[kGroupMax];
};
hipError_t launch_trial_reduce_group(const TrialReduceGroup &G, hipStream_t st);

// The arguments of launch_accept (see there).
struct AcceptArgs {
    const double *yt, *xit;
    double *y, *xi, *dmy;
    const double *uD0, *uD1, *wD0, *wD1;
    const double *yk, *xik;
    double *ye, *xie, *dmye;
    float *y32, *xi32, *dmy32;
    const double *xhat64;
    double inv_delta, beta;
    const double *decision;
    int N, n, NP;
};
struct AcceptGroup {
    int nfit;
    int off[kGroupMax + 1];
    AcceptArgs a[kGroupMax];
};
hipError_t launch_accept_group(const AcceptGroup &G, hipStream_t st);
hipError_t launch_accept_args(const Geometry &g, const AcceptArgs &a, hipStream_t st);
AcceptArgs make_accept_args(const Geometry &g, const double *yt, const double *xit, double *y, double *xi,
                            double *dmy, const double *const uD[2], const double *const wD[2], const double *yk,
                            const double *xik, double *ye, double *xie, double *dmye, float *y32, float *xi32,
                            float *dmy32, const double *xhat64, double inv_delta, double beta,
                            const double *decision);

// Sums / maxima of per-block partials: out[q] = op_q over blocks of part[b * stride + q],
// with op = max for q < nmax and sum otherwise.  Single workgroup, deterministic order.
hipError_t launch_reduce(const double *part, int blocks, int stride, int nmax, int nout,
                         double *out, hipStream_t st);

// Multiplies y, xi, dmy (FP64, Nr / Nr x NP / Nr) by 1/sqrt(sq[0] + sq[1]); optional FP32 copies
// of the result (all three null or all three set).
hipError_t launch_normalize(const Geometry &g, double *y, double *xi, double *dmy, float *y32, float *xi32,
                            float *dmy32, const double *sq, hipStream_t st);

// FP64 multipliers (Nr x ld) from a split representation: dst = H + lo.
hipError_t launch_merge(const Geometry &g, LamRep rep, const void *hi, const float *lo, double *dst,
                        hipStream_t st);

// Dense N x N FP64 (row stride N) into / out of the padded representation (diagonal and padding
// zeroed on the way in).  REP_F64: `main` is the FP64 matrix and `lo` is unused; split forms:
// `main` is H and `lo` the low part of the iterate (split as H = round(lam), lo = lam - H).
hipError_t launch_pack_lambda(const Geometry &g, const double *dense, LamRep rep, void *main, float *lo,
                              hipStream_t st);
hipError_t launch_unpack_lambda(const Geometry &g, LamRep rep, const void *main, const float *lo,
                                double *dense, hipStream_t st);
// Rows [row0, row0 + nrows) only, into a dense nrows x N FP64 array.
hipError_t launch_unpack_rows(const Geometry &g, LamRep rep, const void *main, const float *lo, int row0,
                              int nrows, double *dense, hipStream_t st);

// Builds xhat (FP64 x - mu, ones in column n, zero padding) and optionally its float copy
// from dense N x n locations, and pads ybar (may be null).  mu may be null (no shift).
hipError_t launch_prepare(const Geometry &g, const double *x, const double *ybar,
                          const double *mu, double *xhat64, float *xhat32, double *ybar_pad,
                          hipStream_t st);

// Power-iteration start: v_y,l = -1 + 2 l / (N - 1), v_xi = 1, scaled by 1/||v||; writes
// y, xi and dmy = xi^T x - y (FP64, padded) from xhat64, plus optional FP32 copies (all three
// null or all three set).
hipError_t launch_power_init(const Geometry &g, const double *xhat64, double *y, double *xi,
                             double *dmy, float *y32, float *xi32, float *dmy32, hipStream_t st);

// Pads dense FP64 y (N) and xi (N x n) into Nr / Nr x NP arrays and sets dmy = xi^T x - y.
hipError_t launch_pad_primal(const Geometry &g, const double *y_in, const double *xi_in,
                             const double *xhat64, double *y, double *xi, double *dmy,
                             hipStream_t st);

// Repair: for column j, colmin over strips -> y'_j = y_j - min(0, colmin); xi'_j is the slope of
// the arg-min piece if colmin < -tau_j, else xi_j, with tau_j = 1e-10 (1 + |y_j| + ||xi_j||_1 xspan)
// (xspan = max |x - mean(x)|); writes y'(Nr), xi'(Nr x NP) and rowred' (Nr x 2) for the objective.
hipError_t launch_repair_finish(const Geometry &g, const double *part_min, const int *part_arg,
                                const double *y, const double *xi, const double *ybar,
                                double *y_rep, double *xi_rep, double *rowred, double xspan, hipStream_t st);

// One relaxation round of the own-slope repair from the column minima m_j = min_i (s_ij - c_i) of a
// PASS_REPAIR with offsets c_in: c_out_j = max(c_in_j, -m_j) (padding 0); rowred_j =
// (y_j + c_out_j - ybar_j)^2; changed[b] = number of columns of block b (256 columns) whose c grew
// by more than tau_j (as in launch_repair_finish).  Grid: ceil(Nr / 256) blocks.
hipError_t launch_relax_finish(const Geometry &g, const double *part_min, const double *c_in, double *c_out,
                               const double *y, const double *xi, const double *ybar, double xspan,
                               double *rowred, double *changed, hipStream_t st);

// Sets `bytes` bytes at p (256-byte aligned) to zero with a plain fill kernel (no memset node, so
// the clear also replays correctly where a caller captures the stream into a graph).
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);

// Copies the FP64 y (Nr) and xi (Nr x NP) to dense N and N x n arrays.
hipError_t launch_unpad_primal(const Geometry &g, const double *y, const double *xi,
                               double *y_out, double *xi_out, hipStream_t st);

}  // namespace cr
