// Step 1 of P-APG under a K-block partition (Section 2.1, eq. "subgradient_split"): every block's
// QP solved by a primal-dual path-following interior-point method (Section 2.5), all blocks at once,
// one workgroup per block.
//
// With the pairs between blocks dualized, block b's Step-1 problem is the G-norm projection of the
// closed-form point eta0 = (ybar + A1^T theta, A2^T theta / delta) onto the block's own pair
// constraints (eq. "eq:step1-problem" with c = -G eta0, G = diag(I, delta I)):
//     min 1/2 ||y - y0||^2 + delta/2 ||xi - xi0||^2   s.t.  s_ac = y_c - y_a + xi_a^T (x_a - x_c) >= 0
// over the block's points a != c.  The IPM keeps slacks s > 0 and multipliers theta > 0 of the
// perturbed KKT system (eq. "eq:KKT-perturbed") and takes Mehrotra predictor-corrector Newton
// steps; each step solves the normal equations (eq. "eq:normal-equation") whose matrix
// M = G + A^T diag(theta / s) A is block arrowhead (eq. "eq:arrowhead", components as in
// eq. "eq:M-components"): a p x p block M00 for y, one n x n block M_aa per point for xi_a, and the
// p x n couplings M0a.  The solve eliminates the xi blocks first (Theorem
// "lem:cholesky-block-arrowhead"): z_a = M_aa^-1 b_a, then the y system with the Schur complement
// S = M00 - sum_a M0a M_aa^-1 M0a^T, then xi_a = M_aa^-1 (b_a - M0a^T dy).  (The theorem's closed
// form writes M00^-1 where this elimination needs S; S is what makes it exact.)
//
// Work split (512 threads, 8 waves, one block of q <= 100 points per workgroup):
//  * pair passes run one row a per wave at a time, lanes over the partners c; sums over c of an
//    n-vector (the xi parts of r_d, A^T w and M0a^T dy) split the lanes into 64 / n groups of n;
//    the M_aa sums take 4 rows per wave (d transposed in LDS) so that each x_c x_c^T entry serves four;
//  * the residuals r_p, r_d and the slack steps keep the difference form x_a - x_c; the Newton
//    matrix blocks M_aa use the expanded form sum_c d_ac x_c x_c^T - D_a x_a x_a^T + x_a g_a^T +
//    g_a x_a^T on locations centred on the block's mean (they only shape the direction);
//  * each M_aa is factored, and every single-vector triangular solve with it run, by one thread with
//    the vector in registers (n <= NB, a compile-time bound): the points' dependent chains run side
//    by side; V_a's q columns take one wave per point, one lane per column, with the factor in the
//    wave's LDS buffer when it fits (n <= 27);
//  * S = M00 - V^T V (V = stacked F_a^-1 M0a^T, q n x q) runs as a register-tiled product (4 x 4
//    tiles of the lower triangle, the q n rows split in three), V staged through LDS;
//  * S is factored as L D L^T in LDS with one barrier per column; the two triangular solves with it
//    run in one wave without barriers, the vector held two entries per lane.
// Every loop has a trip count uniform over the workgroup and every barrier is reached by all threads.

#include "cr_kernels.h"

#include <hip/hip_runtime.h>

namespace cr {
namespace {

constexpr int kBT = 512;                  // threads per workgroup
constexpr int kWaves = kBT / 64;          // 8
constexpr int kWB = 384;                  // per-wave LDS buffer: two q-rows (128 each) + two 64-vectors
constexpr int kKS = 3;                    // row groups of a stage of the Schur-complement product
// rows of V per LDS stage of that product: 48 while the block's LDS leaves room (n <= 32), else 24
constexpr int stage_rows(int NB) { return NB <= 32 ? 48 : 24; }
// shared scratch (row buffers / column partials / V stage)
constexpr int scratch_doubles(int NB) {
    return stage_rows(NB) * kMaxBlock > kWaves * kWB ? stage_rows(NB) * kMaxBlock : kWaves * kWB;
}
constexpr int kLE = (kMaxBlock * (kMaxBlock + 1) / 2 + kBT - 1) / kBT;   // lower-triangle entries per thread
static_assert(2 * kWaves * kMaxBlock <= kWaves * kWB, "scratch too small");
static_assert(kMaxBlock <= 128, "two partner slots per lane");

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Orders one wave's LDS accesses (the lanes run in lockstep; this keeps the compiler from moving
// loads or stores across the point where other lanes' values are consumed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ double read_lane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Workgroup reductions (all threads call; `sh` holds one double per wave).
__device__ __forceinline__ double wg_sum(double v, double *sh) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < kWaves; ++i) r += sh[i];
    return r;
}
__device__ __forceinline__ double wg_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kWaves; ++i) r = fmax(r, sh[i]);
    return r;
}
__device__ __forceinline__ double wg_min(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kWaves; ++i) r = fmin(r, sh[i]);
    return r;
}

// Per-block arrays in the global workspace (q points, n features; P2 = q^2 pair slots, the
// diagonal slots unused).
struct BlockWs {
    double *sl, *th, *dd, *rp, *dsa, *dta, *dsv;   // P2 each: slack, multiplier, theta/s, r_p, affine
                                                   // steps (slack, multiplier), the step's slack change
    double *V;      // q n x q: V[(a n + m) q + c] = (F_a^-1 M0a^T)[m][c]
    double *F;      // q x n x n: Cholesky factor of M_aa (lower, row-major; diagonal as computed)
    double *y, *y0, *ry;                             // q each
    double *xi, *xi0, *rxi, *gv, *bxi, *dxi, *zz, *fd;   // q n each (fd: 1 / diagonal of F_a)
    double *ksl, *kth, *ky, *kxi;                    // the best point met so far (s, theta, y, xi)
};

__device__ __forceinline__ BlockWs carve(double *W, int q, int n) {
    const size_t P2 = (size_t)q * q, qn = (size_t)q * n;
    BlockWs w;
    w.sl = W; w.th = w.sl + P2; w.dd = w.th + P2; w.rp = w.dd + P2; w.dsa = w.rp + P2; w.dta = w.dsa + P2;
    w.dsv = w.dta + P2;
    w.V = w.dsv + P2;
    w.F = w.V + qn * q;
    w.y = w.F + qn * n; w.y0 = w.y + q; w.ry = w.y0 + q;
    w.xi = w.ry + q; w.xi0 = w.xi + qn; w.rxi = w.xi0 + qn; w.gv = w.rxi + qn; w.bxi = w.gv + qn;
    w.dxi = w.bxi + qn; w.zz = w.dxi + qn; w.fd = w.zz + qn;
    w.ksl = w.fd + qn; w.kth = w.ksl + P2; w.ky = w.kth + P2; w.kxi = w.ky + q;
    return w;
}

// Packed lower-triangle index and its inverse (row of entry e).
__device__ __forceinline__ int tix(int i, int j) { return i * (i + 1) / 2 + j; }
__device__ __forceinline__ int tri_row(int e) {
    int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    while (i * (i + 1) / 2 > e) --i;
    return i;
}

// z <- F^-T F^-1 z for one point's factor (n <= NB; entries of z beyond n are zero).
template <int NB>
__device__ __forceinline__ void factor_solve(const double *F, const double *fd, int n, double (&z)[NB]) {
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        if (m < n) {
            double r = z[m];
#pragma unroll
            for (int j = 0; j < m; ++j) r -= F[m * n + j] * z[j];
            z[m] = r * fd[m];
        }
    }
#pragma unroll
    for (int m = NB - 1; m >= 0; --m) {
        if (m < n) {
            double r = z[m];
#pragma unroll
            for (int j = m + 1; j < NB; ++j)
                if (j < n) r -= F[j * n + m] * z[j];
            z[m] = r * fd[m];
        }
    }
}

}  // namespace

size_t block_ws_doubles(int p, int n) {
    const size_t P2 = (size_t)p * p, qn = (size_t)p * n;
    return 9 * P2 + qn * p + qn * n + 4 * (size_t)p + 9 * qn + 64;
}

namespace {

template <int NB>
__global__ __launch_bounds__(kBT) void block_ipm_kernel(BlockProjArgs A) {
    constexpr int XS = NB + 1;                                    // odd row stride of the locations
    constexpr int kKC = stage_rows(NB), kScr = scratch_doubles(NB);
    constexpr int kPre = (kKC * kMaxBlock + kBT - 1) / kBT;
    static_assert(kKC % kKS == 0, "stage rows split into kKS groups");
    __shared__ double sS[kMaxBlock * (kMaxBlock + 1)];           // d_ac, then M00, S and its L D L^T
    __shared__ double sX[kMaxBlock * XS];                        // locations, centred on the block mean
    __shared__ __align__(16) double sW[kScr];                    // row buffers / partials / V stage
    __shared__ double sRt[kMaxBlock], sRd[kMaxBlock];            // row sums of theta and d
    __shared__ double sFl[kMaxBlock], sDi[kMaxBlock];            // diagonal of M00; 1 / pivots of S
    __shared__ double sBy[kMaxBlock], sDy[kMaxBlock];            // y part of the right-hand side; dy
    __shared__ double sh[kWaves];
    const int b = blockIdx.x, t = threadIdx.x, wid = t >> 6, ln = t & 63;
    const int i0 = b * A.p;
    const int q = min(A.p, A.N - i0);
    const int n = A.n, NP = A.NP;
    const double delta = A.delta;
    if (q <= 0) return;                       // uniform over the workgroup
    const int ld = q | 1;                     // odd row stride of S
    BlockWs w = carve(A.ws + (size_t)b * A.ws_doubles, q, n);
    double *rb1 = sW + wid * kWB, *rb2 = rb1 + 128, *rbn = rb2 + 128, *rbp = rbn + 64;
    // lanes (gq, gm) for sums over c of an n-vector: group gq takes c = gq, gq + G, ...
    const int G = 64 / n, gq = ln / n, gm = ln - gq * n;
    const int tri = n * (n + 1) / 2;
    // a point's packed factor fits a wave's buffer (n <= 27): V reads it from LDS
    const bool fl = tri <= kWB;
    double *wF = rb1;

    // eta0 in; the locations centred on the block's mean (differences x_a - x_c are unchanged)
    for (int m = t; m < n; m += kBT) {
        double s = 0.0;
        for (int a = 0; a < q; ++a) s += A.xhat[(size_t)(i0 + a) * NP + m];
        sW[m] = s / q;
    }
    for (int e = t; e < q; e += kBT) { w.y0[e] = A.y[i0 + e]; w.y[e] = w.y0[e]; }
    __syncthreads();
    for (int e = t; e < q * n; e += kBT) {
        const int a = e / n, m = e - a * n;
        w.xi0[e] = A.xi[(size_t)(i0 + a) * NP + m];
        w.xi[e] = w.xi0[e];
        sX[a * XS + m] = A.xhat[(size_t)(i0 + a) * NP + m] - sW[m];
    }
    __syncthreads();

    // s_ac of the current eta (difference form), the row's xi_a staged in rbn
    auto lin = [&](int a, int c, double ya) -> double {
        double v = w.y[c] - ya;
#pragma unroll 4
        for (int m = 0; m < n; ++m) v += rbn[m] * (sX[a * XS + m] - sX[c * XS + m]);
        return v;
    };
    // out1 = sum_c r1[c] (x_a - x_c), out2 likewise with r2, on lanes m < n (r1, r2: LDS rows of the
    // wave, zero at c = a); rbn and rbp are overwritten
    auto rowvec = [&](int a, const double *r1, const double *r2, double &o1, double &o2) {
        double s1 = 0.0, s2 = 0.0;
        if (gq < G) {
            const double xm = sX[a * XS + gm];
#pragma unroll 4
            for (int c = gq; c < q; c += G) {
                const double u = xm - sX[c * XS + gm];
                s1 += r1[c] * u;
                if (r2) s2 += r2[c] * u;
            }
        }
        wave_sync();
        if (gq < G) { rbp[ln] = s1; rbn[ln] = s2; }
        wave_sync();
        o1 = 0.0; o2 = 0.0;
        if (ln < n)
            for (int g = 0; g < G; ++g) { o1 += rbp[g * n + ln]; o2 += rbn[g * n + ln]; }
        wave_sync();
    };
    // column sums of per-lane partials (slots c = ln, ln + 64) over the waves: returns on threads
    // c < q through `use(c, sum)`
    auto colsum = [&](double p0, double p1, auto &&use) {
        __syncthreads();
        if (ln < q) sW[wid * kMaxBlock + ln] = p0;
        if (ln + 64 < q) sW[wid * kMaxBlock + ln + 64] = p1;
        __syncthreads();
        for (int c = t; c < q; c += kBT) {
            double s = 0.0;
            for (int i = 0; i < kWaves; ++i) s += sW[i * kMaxBlock + c];
            use(c, s);
        }
        __syncthreads();
    };

    // starting point: eta = eta0 and, cold, s = max(A eta0, 1), theta = 1; warm (A.warm: the
    // workspace holds the slacks and multipliers the previous Step 1 ended on, for a nearby
    // projection), both lifted to at least 1e-4 of the block's scale
    double ysc = 0.0;
    for (int e = t; e < q; e += kBT) ysc = fmax(ysc, fabs(w.y0[e]));
    for (int a = wid; a < q; a += kWaves) {
        if (ln < n) rbn[ln] = w.xi[a * n + ln];
        wave_sync();
        const double ya = w.y[a];
        for (int s = 0; s < 2; ++s) {
            const int c = ln + 64 * s;
            if (c >= q) continue;
            const size_t e = (size_t)a * q + c;
            if (c == a) { w.sl[e] = 1.0; w.th[e] = 0.0; continue; }
            const double v = lin(a, c, ya);
            ysc = fmax(ysc, fabs(v));
            if (!A.warm) {
                w.sl[e] = fmax(v, 1.0);
                w.th[e] = 1.0;
            }
        }
        wave_sync();
    }
    const double scale = 1.0 + wg_max(ysc, sh);
    if (A.warm) {
        const double lift = 1e-4 * scale;
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c < q; c += 64) {
                if (c == a) continue;
                const size_t e = (size_t)a * q + c;
                w.sl[e] = fmax(w.sl[e], lift);
                w.th[e] = fmax(w.th[e], lift);
            }
        __syncthreads();
    }
    const double tol = A.tol * scale;
    // complementarity target: a weakly active constraint (zero slack and zero multiplier at the
    // solution) keeps both near sqrt(mu), and the projection's error follows them; mu is driven
    // seven orders below tol in units of the block's scale squared.  Near that target the normal
    // equations span many orders and the dual residual may stall above tol while mu keeps falling:
    // the iteration keeps the best point met (merit phi = max(r_p / tol, r_d / tol, mu / tol_mu)),
    // stops once mu has passed the target by four more orders, and returns the best point.
    const double tol_mu = 1e-7 * A.tol * scale * scale;
    double phi_best = INFINITY;
    const double mpairs = (double)q * (double)(q - 1);

    int it = 0;
    for (; it < A.max_iter && q > 1; ++it) {
        // --- residuals: r_p = A eta - s, d = theta / s, mu; r_d = G eta + c - A^T theta; g_a
        double rpmax = 0.0, gap = 0.0, rdmax = 0.0;
        double cth0 = 0.0, cth1 = 0.0, cdd0 = 0.0, cdd1 = 0.0;
        for (int a = wid; a < q; a += kWaves) {
            if (ln < n) rbn[ln] = w.xi[a * n + ln];
            wave_sync();
            const double ya = w.y[a];
            double rth = 0.0, rdd = 0.0;
            for (int s = 0; s < 2; ++s) {
                const int c = ln + 64 * s;
                double thv = 0.0, dv = 0.0;
                if (c < q && c != a) {
                    const size_t e = (size_t)a * q + c;
                    const double slv = w.sl[e];
                    thv = w.th[e];
                    const double r = lin(a, c, ya) - slv;
                    w.rp[e] = r;
                    rpmax = fmax(rpmax, fabs(r));
                    gap += slv * thv;
                    dv = thv / slv;
                    w.dd[e] = dv;
                }
                if (c < q) { rb1[c] = thv; rb2[c] = dv; sS[c * ld + a] = dv; }   // d transposed in LDS
                if (s == 0) { cth0 += thv; cdd0 += dv; } else { cth1 += thv; cdd1 += dv; }
                rth += thv;
                rdd += dv;
            }
            rth = wave_sum(rth);
            rdd = wave_sum(rdd);
            wave_sync();
            double s1, s2;
            rowvec(a, rb1, rb2, s1, s2);      // sum_c theta_ac (x_a - x_c), g_a = sum_c d_ac (x_a - x_c)
            if (ln < n) {
                const int e = a * n + ln;
                const double r = delta * (w.xi[e] - w.xi0[e]) - s1;
                w.rxi[e] = r;
                rdmax = fmax(rdmax, fabs(r));
                w.gv[e] = s2;
            }
            if (ln == 0) { sRt[a] = rth; sRd[a] = rdd; }
            wave_sync();
        }
        colsum(cth0, cth1, [&](int c, double ct) {
            // y part of r_d: (y - y0) - (column sum - row sum) of theta
            const double r = (w.y[c] - w.y0[c]) - (ct - sRt[c]);
            w.ry[c] = r;
            rdmax = fmax(rdmax, fabs(r));
        });
        colsum(cdd0, cdd1, [&](int c, double cd) { sFl[c] = 1.0 + sRd[c] + cd; });   // diagonal of M00
        rpmax = wg_max(rpmax, sh);
        const double mu = wg_sum(gap, sh) / mpairs;
        rdmax = wg_max(rdmax, sh);
        // uniform: the reductions broadcast
        const double phi = fmax(fmax(rpmax, rdmax) / tol, mu / tol_mu);
        if (phi < phi_best) {
            phi_best = phi;
            for (int a = wid; a < q; a += kWaves)
                for (int c = ln; c < q; c += 64) {
                    const size_t e = (size_t)a * q + c;
                    w.ksl[e] = w.sl[e];
                    w.kth[e] = w.th[e];
                }
            for (int e = t; e < q; e += kBT) w.ky[e] = w.y[e];
            for (int e = t; e < q * n; e += kBT) w.kxi[e] = w.xi[e];
        }
        if (phi <= 1.0 || mu < 1e-4 * tol_mu) break;

        // --- M_aa = delta I + sum_c d_ac x_c x_c^T - D_a x_a x_a^T + x_a g_a^T + g_a x_a^T (the expanded
        // form of sum_c d_ac (x_a - x_c)(x_a - x_c)^T): a wave takes 4 rows and 64 entries (m1 >= m2),
        // so that one product x_c[m1] x_c[m2] serves four rows; d is read transposed from LDS
        {
            const int nrg = (q + 3) >> 2, nch = (tri + 63) >> 6;
            for (int task = wid; task < nrg * nch; task += kWaves) {
                const int rg = task / nch, ch = task - rg * nch;
                const int e = ch * 64 + ln;
                const int m1 = e < tri ? tri_row(e) : 0, m2 = e < tri ? e - tix(m1, 0) : 0;
                int ar[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) ar[r] = min(4 * rg + r, q - 1);
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                for (int c = 0; c < q; ++c) {
                    const double z = sX[c * XS + m1] * sX[c * XS + m2];
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] += sS[c * ld + ar[r]] * z;
                }
                if (e < tri) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int a = 4 * rg + r;
                        if (a >= q) break;
                        const double xa1 = sX[a * XS + m1], xa2 = sX[a * XS + m2];
                        double v = acc[r] - sRd[a] * xa1 * xa2 + xa1 * w.gv[a * n + m2] + w.gv[a * n + m1] * xa2;
                        if (m1 == m2) v += delta;
                        w.F[(size_t)a * n * n + m1 * n + m2] = v;
                    }
                }
            }
        }
        __syncthreads();

        // --- factor each M_aa (one thread per point, the current row in registers, earlier rows from
        // the workspace), then V_a[:, c] = F_a^-1 (M0a^T)[:, c] (d_ac (x_a - x_c) for c != a, -g_a for
        // c = a): one wave per point, one lane per column with the column in registers, the factor
        // read from the wave's LDS buffer when it fits there (n <= 27), else from the workspace
        for (int a = t; a < q; a += kBT) {
            double *F = w.F + (size_t)a * n * n;
            double *fd = w.fd + (size_t)a * n;
            for (int i = 0; i < n; ++i) {
                double r[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) r[j] = (j < i) ? F[i * n + j] : 0.0;
                const double a_ii = F[i * n + i];
                double dg = a_ii;
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    if (j < i) {
                        double s = r[j];
#pragma unroll
                        for (int k = 0; k < j; ++k) s -= r[k] * F[j * n + k];
                        s *= fd[j];
                        r[j] = s;
                        dg -= s * s;
                    }
                }
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if (j < i) F[i * n + j] = r[j];
                // M_aa >= delta I: positive in exact arithmetic; a relative floor guards rounding
                const double piv = sqrt(fmax(dg, 1e-14 * a_ii));
                F[i * n + i] = piv;
                fd[i] = 1.0 / piv;
            }
        }
        __syncthreads();
        for (int a = wid; a < q; a += kWaves) {
            const double *__restrict__ F = w.F + (size_t)a * n * n;
            const double *__restrict__ fd = w.fd + (size_t)a * n;
            if (fl) {
                // packed factor with 1 / L_kk on the diagonal
                for (int e = ln; e < tri; e += 64) {
                    const int i = tri_row(e), j = e - tix(i, 0);
                    wF[e] = (i == j) ? fd[i] : F[i * n + j];
                }
                wave_sync();
            }
            for (int s = 0; s < 2; ++s) {
                const int c = ln + 64 * s;
                if (c >= q) continue;
                const double dac = (c == a) ? 0.0 : w.dd[(size_t)a * q + c];
                double v[NB];
                if (fl) {
#pragma unroll
                    for (int m = 0; m < NB; ++m) {
                        v[m] = 0.0;
                        if (m < n) {
                            double r = (c == a) ? -w.gv[a * n + m] : dac * (sX[a * XS + m] - sX[c * XS + m]);
#pragma unroll
                            for (int j = 0; j < m; ++j) r -= wF[tix(m, j)] * v[j];
                            v[m] = r * wF[tix(m, m)];
                        }
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < NB; ++m) {
                        v[m] = 0.0;
                        if (m < n) {
                            double r = (c == a) ? -w.gv[a * n + m] : dac * (sX[a * XS + m] - sX[c * XS + m]);
#pragma unroll
                            for (int j = 0; j < m; ++j) r -= F[m * n + j] * v[j];
                            v[m] = r * fd[m];
                        }
                    }
                }
                // stores after the substitution, so that no store stands between the factor's loads
#pragma unroll
                for (int m = 0; m < NB; ++m)
                    if (m < n) w.V[(size_t)(a * n + m) * q + c] = v[m];
            }
            wave_sync();
        }
        // M00's lower triangle in place of d: -(d_ac + d_ca) off the diagonal
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c <= a; c += 64)
                sS[a * ld + c] = (c == a) ? sFl[a] : -(sS[a * ld + c] + sS[c * ld + a]);
        __syncthreads();

        // --- S = M00 - V^T V on the lower triangle: 4 x 4 tiles, the rows of V in kKS groups
        {
            const int T4 = (q + 3) >> 2, LDV = 4 * T4, nt = T4 * (T4 + 1) / 2, K = q * n;
            const int ntask = nt * kKS;
            int tI[2], tJ[2], tg[2];
            bool tv[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int u = t + h * kBT;
                tv[h] = u < ntask;
                const int g = tv[h] ? u / nt : 0, tau = tv[h] ? u - g * nt : 0;
                int I = (int)((sqrtf(8.0f * tau + 1.0f) - 1.0f) * 0.5f);
                while ((I + 1) * (I + 2) / 2 <= tau) ++I;
                while (I * (I + 1) / 2 > tau) --I;
                tI[h] = I;
                tJ[h] = tau - I * (I + 1) / 2;
                tg[h] = g;
            }
            // this thread's slots of a stage: row and column within the stage
            int srow[kPre], scol[kPre];
#pragma unroll
            for (int r = 0; r < kPre; ++r) {
                const int e = t + r * kBT;
                srow[r] = e < kKC * LDV ? e / LDV : kKC;
                scol[r] = e < kKC * LDV ? e - srow[r] * LDV : 0;
            }
            double pre[kPre];
            auto fetch = [&](int ch) {
#pragma unroll
                for (int r = 0; r < kPre; ++r) {
                    const int k = ch * kKC + srow[r];
                    pre[r] = (srow[r] < kKC && k < K && scol[r] < q) ? w.V[(size_t)k * q + scol[r]] : 0.0;
                }
            };
            double acc[2][4][4];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[h][i][j] = 0.0;
            const int nch = (K + kKC - 1) / kKC;
            fetch(0);
            for (int ch = 0; ch < nch; ++ch) {
#pragma unroll
                for (int r = 0; r < kPre; ++r)
                    if (srow[r] < kKC) sW[srow[r] * LDV + scol[r]] = pre[r];
                __syncthreads();
                if (ch + 1 < nch) fetch(ch + 1);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (!tv[h]) continue;
                    const double *pa = sW + tg[h] * (kKC / kKS) * LDV + 4 * tI[h];
                    const double *pb = sW + tg[h] * (kKC / kKS) * LDV + 4 * tJ[h];
#pragma unroll
                    for (int r = 0; r < kKC / kKS; ++r) {
                        const double2 a01 = *reinterpret_cast<const double2 *>(pa + r * LDV);
                        const double2 a23 = *reinterpret_cast<const double2 *>(pa + r * LDV + 2);
                        const double2 b01 = *reinterpret_cast<const double2 *>(pb + r * LDV);
                        const double2 b23 = *reinterpret_cast<const double2 *>(pb + r * LDV + 2);
                        const double av[4] = {a01.x, a01.y, a23.x, a23.y};
                        const double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int j = 0; j < 4; ++j) acc[h][i][j] = fma(av[i], bv[j], acc[h][i][j]);
                    }
                }
                __syncthreads();
            }
            // the kKS partial sums of a tile land one group at a time
            for (int g = 0; g < kKS; ++g) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (!tv[h] || tg[h] != g) continue;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int r = 4 * tI[h] + i, c = 4 * tJ[h] + j;
                            if (r < q && c <= r) sS[r * ld + c] -= acc[h][i][j];
                        }
                }
                __syncthreads();
            }
        }

        // --- S = L D L^T in LDS (L unit lower, stored unscaled: L_ik = S_ik / D_k), one barrier per
        // column.  S is positive definite in exact arithmetic; rounding near the end of the IPM
        // (theta / s spanning many orders) is kept from a non-positive pivot by a relative floor.
        {
            // each thread owns the entries e = t, t + kBT, ... of the packed lower triangle
            int oi[kLE], oj[kLE];
            const int nlow = q * (q + 1) / 2;
#pragma unroll
            for (int r = 0; r < kLE; ++r) {
                const int e = t + r * kBT;
                int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
                while ((i + 1) * (i + 2) / 2 <= e) ++i;
                while (i * (i + 1) / 2 > e) --i;
                oi[r] = e < nlow ? i : -1;
                oj[r] = e - i * (i + 1) / 2;
            }
            for (int k = 0; k < q; ++k) {
                const double dk = fmax(sS[k * ld + k], 1e-14 * sFl[k]);
                const double inv = 1.0 / dk;
                if (t == 0) sDi[k] = inv;
#pragma unroll
                for (int r = 0; r < kLE; ++r)
                    if (oj[r] > k && oi[r] >= 0)
                        sS[oi[r] * ld + oj[r]] -= sS[oi[r] * ld + k] * inv * sS[oj[r] * ld + k];
                __syncthreads();
            }
        }

        // Newton system M d_eta = -r_d + A^T wv with wv = d (-r_p) + r_c / s; r_c the
        // complementarity right-hand side (predictor: -s theta; corrector adds -ds_aff dth_aff + sig mu)
        auto solve = [&](bool corrector, double sigmu) __attribute__((always_inline)) {
            // right-hand side: y part -r_d + (column sum - row sum) of wv, xi part
            // -r_d + sum_c wv_ac (x_a - x_c)
            double c0 = 0.0, c1 = 0.0;
            for (int a = wid; a < q; a += kWaves) {
                double rs = 0.0;
                for (int s = 0; s < 2; ++s) {
                    const int c = ln + 64 * s;
                    double v = 0.0;
                    if (c < q && c != a) {
                        const size_t e = (size_t)a * q + c;
                        const double slv = w.sl[e];
                        double rc = -slv * w.th[e];
                        if (corrector) rc += -w.dsa[e] * w.dta[e] + sigmu;
                        v = -w.dd[e] * w.rp[e] + rc / slv;
                    }
                    if (c < q) rb1[c] = v;
                    if (s == 0) c0 += v; else c1 += v;
                    rs += v;
                }
                rs = wave_sum(rs);
                wave_sync();
                double s1, s2;
                rowvec(a, rb1, nullptr, s1, s2);
                if (ln < n) w.bxi[a * n + ln] = -w.rxi[a * n + ln] + s1;
                if (ln == 0) sRt[a] = rs;
                wave_sync();
            }
            colsum(c0, c1, [&](int c, double cs) { sBy[c] = -w.ry[c] + (cs - sRt[c]); });
            // z_a = M_aa^-1 b_a (one thread per point: the points' dependent chains run side by side)
            for (int a = t; a < q; a += kBT) {
                double z[NB];
#pragma unroll
                for (int m = 0; m < NB; ++m) z[m] = (m < n) ? w.bxi[a * n + m] : 0.0;
                factor_solve<NB>(w.F + (size_t)a * n * n, w.fd + (size_t)a * n, n, z);
#pragma unroll
                for (int m = 0; m < NB; ++m)
                    if (m < n) w.zz[a * n + m] = z[m];
            }
            __syncthreads();
            // r0_c = by_c - sum_a (M0a z_a)_c: d_ac <x_a - x_c, z_a> for a != c, -<g_c, z_c> for a = c
            c0 = 0.0; c1 = 0.0;
            for (int a = wid; a < q; a += kWaves) {
                if (ln < n) rbn[ln] = w.zz[a * n + ln];
                wave_sync();
                double wa = 0.0;
#pragma unroll 4
                for (int m = 0; m < n; ++m) wa += rbn[m] * sX[a * XS + m];
                for (int s = 0; s < 2; ++s) {
                    const int c = ln + 64 * s;
                    if (c >= q || c == a) continue;
                    double v = wa;
#pragma unroll 4
                    for (int m = 0; m < n; ++m) v -= rbn[m] * sX[c * XS + m];
                    v *= w.dd[(size_t)a * q + c];
                    if (s == 0) c0 += v; else c1 += v;
                }
                wave_sync();
            }
            colsum(c0, c1, [&](int c, double cs) {
                double gz = 0.0;
                for (int m = 0; m < n; ++m) gz += w.gv[c * n + m] * w.zz[c * n + m];
                sDy[c] = sBy[c] - cs + gz;
            });
            // dy = S^-1 r0 with L D L^T, in one wave: entries c = ln, ln + 64 in registers
            if (wid == 0) {
                double v0 = ln < q ? sDy[ln] : 0.0, v1 = ln + 64 < q ? sDy[ln + 64] : 0.0;
                // the loads are unconditional (rows clamped into the block) so that the unrolled
                // steps can issue them ahead of the dependent updates
                const int r0 = min(ln, q - 1), r1 = min(ln + 64, q - 1);
#pragma unroll 4
                for (int k = 0; k < q; ++k) {
                    const double s0 = sS[r0 * ld + k], s1 = sS[r1 * ld + k], dik = sDi[k];
                    const double zk = (k < 64 ? read_lane(v0, k) : read_lane(v1, k - 64)) * dik;
                    if (ln > k && ln < q) v0 -= s0 * zk;
                    if (ln + 64 > k && ln + 64 < q) v1 -= s1 * zk;
                }
                const double id0 = ln < q ? sDi[ln] : 0.0, id1 = ln + 64 < q ? sDi[ln + 64] : 0.0;
                v0 *= id0;
                v1 *= id1;
#pragma unroll 4
                for (int k = q - 1; k > 0; --k) {
                    const double s0 = sS[k * ld + r0], s1 = sS[k * ld + r1];
                    const double xk = k < 64 ? read_lane(v0, k) : read_lane(v1, k - 64);
                    if (ln < k) v0 -= s0 * id0 * xk;
                    if (ln + 64 < k) v1 -= s1 * id1 * xk;
                }
                if (ln < q) sDy[ln] = v0;
                if (ln + 64 < q) sDy[ln + 64] = v1;
            }
            __syncthreads();
            // dxi_a = M_aa^-1 (b_a - M0a^T dy), (M0a^T dy) = sum_c d_ac dy_c (x_a - x_c) - g_a dy_a
            for (int a = wid; a < q; a += kWaves) {
                for (int s = 0; s < 2; ++s) {
                    const int c = ln + 64 * s;
                    if (c < q) rb1[c] = (c == a) ? 0.0 : w.dd[(size_t)a * q + c] * sDy[c];
                }
                wave_sync();
                double s1, s2;
                rowvec(a, rb1, nullptr, s1, s2);
                if (ln < n) {
                    const int e = a * n + ln;
                    w.dxi[e] = w.bxi[e] - (s1 - w.gv[e] * sDy[a]);
                }
                wave_sync();
            }
            __syncthreads();
            for (int a = t; a < q; a += kBT) {
                double z[NB];
#pragma unroll
                for (int m = 0; m < NB; ++m) z[m] = (m < n) ? w.dxi[a * n + m] : 0.0;
                factor_solve<NB>(w.F + (size_t)a * n * n, w.fd + (size_t)a * n, n, z);
#pragma unroll
                for (int m = 0; m < NB; ++m)
                    if (m < n) w.dxi[a * n + m] = z[m];
            }
            __syncthreads();
        };
        // slack and multiplier steps of the solved direction; returns the largest step in (0, 1]
        // keeping both positive (before the fraction to the boundary), -1 for a non-finite direction
        auto steps = [&](bool corrector, double sigmu, double *dsl, double *dth) -> double {
            double amax = 1.0, bad = 0.0;
            for (int a = wid; a < q; a += kWaves) {
                if (ln < n) rbn[ln] = w.dxi[a * n + ln];
                wave_sync();
                const double dya = sDy[a];
                for (int s = 0; s < 2; ++s) {
                    const int c = ln + 64 * s;
                    if (c >= q) continue;
                    const size_t e = (size_t)a * q + c;
                    if (c == a) { dsl[e] = 0.0; dth[e] = 0.0; continue; }
                    double adeta = sDy[c] - dya;
#pragma unroll 4
                    for (int m = 0; m < n; ++m) adeta += rbn[m] * (sX[a * XS + m] - sX[c * XS + m]);
                    const double slv = w.sl[e], thv = w.th[e];
                    const double dsv = adeta + w.rp[e];
                    double rc = -slv * thv;
                    if (corrector) rc += -w.dsa[e] * w.dta[e] + sigmu;
                    const double dtv = -w.dd[e] * dsv + rc / slv;
                    dsl[e] = dsv;
                    dth[e] = dtv;
                    if (!isfinite(dsv) || !isfinite(dtv)) bad = 1.0;
                    if (dsv < 0.0) amax = fmin(amax, -slv / dsv);
                    if (dtv < 0.0) amax = fmin(amax, -thv / dtv);
                }
                wave_sync();
            }
            return wg_max(bad, sh) > 0.0 ? -1.0 : wg_min(amax, sh);
        };
        // predictor (affine scaling)
        solve(false, 0.0);
        const double aaff = steps(false, 0.0, w.dsa, w.dta);
        if (aaff < 0.0) break;
        double gaff = 0.0;
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c < q; c += 64) {
                if (c == a) continue;
                const size_t e = (size_t)a * q + c;
                gaff += (w.sl[e] + aaff * w.dsa[e]) * (w.th[e] + aaff * w.dta[e]);
            }
        const double muaff = wg_sum(gaff, sh) / mpairs;
        const double sig = mu > 0.0 ? fmin(1.0, (muaff / mu) * (muaff / mu) * (muaff / mu)) : 0.0;
        // corrector
        solve(true, sig * mu);
        const double amax = steps(true, sig * mu, w.dsv, w.dta);
        if (amax < 1e-12) break;   // no usable step (or a non-finite one): keep the current point
        const double alpha = fmin(1.0, 0.99 * amax);
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c < q; c += 64) {
                if (c == a) continue;
                const size_t e = (size_t)a * q + c;
                w.sl[e] += alpha * w.dsv[e];
                w.th[e] += alpha * w.dta[e];
            }
        for (int e = t; e < q; e += kBT) w.y[e] += alpha * sDy[e];
        for (int e = t; e < q * n; e += kBT) w.xi[e] += alpha * w.dxi[e];
        __syncthreads();
    }
    if (t == 0 && A.iters) A.iters[b] = it;
    if (q > 1) {
        // back to the best point (the point the loop ended on when it converged)
        __syncthreads();
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c < q; c += 64) {
                const size_t e = (size_t)a * q + c;
                w.sl[e] = w.ksl[e];
                w.th[e] = w.kth[e];
            }
        for (int e = t; e < q; e += kBT) w.y[e] = w.ky[e];
        for (int e = t; e < q * n; e += kBT) w.xi[e] = w.kxi[e];
        __syncthreads();
    }

    // the projection out: y, xi, dmy = xi^T x - y (and the rows' objective terms), and the
    // blocks' multipliers into the intra-block entries of lam
    for (int e = t; e < q; e += kBT) {
        const int i = i0 + e;
        double d = 0.0, xsq = 0.0;
        for (int m = 0; m < n; ++m) {
            const double v = w.xi[e * n + m];
            A.xi[(size_t)i * NP + m] = v;
            d += v * A.xhat[(size_t)i * NP + m];
            xsq += v * v;
        }
        A.y[i] = w.y[e];
        A.dmy[i] = d - w.y[e];
        if (A.rowred) {
            const double dy = w.y[e] - A.ybar[i];
            A.rowred[2 * (size_t)i] = dy * dy;
            A.rowred[2 * (size_t)i + 1] = xsq;
        }
    }
    if (A.lam) {
        // the multipliers of the constraints the IPM leaves inactive (slack above multiplier) are
        // theta = mu / s, far below the target: they are written as 0
        for (int a = wid; a < q; a += kWaves)
            for (int c = ln; c < q; c += 64) {
                const size_t e = (size_t)a * q + c;
                A.lam[(size_t)(i0 + a) * A.ld + (i0 + c)] = (a == c || w.th[e] <= w.sl[e]) ? 0.0 : w.th[e];
            }
    }
}

}  // namespace

hipError_t launch_block_project(const Geometry &g, const BlockProjArgs &a, hipStream_t st) {
    if (a.p < 1 || a.p > kMaxBlock || a.n < 1 || a.n > 16 * kMaxMB) return hipErrorInvalidValue;
    const int blocks = (g.N + a.p - 1) / a.p;
    // the smallest compile-time bound NB >= n: the per-point vectors are NB doubles in registers
    if (a.n <= 8)
        hipLaunchKernelGGL(block_ipm_kernel<8>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 12)
        hipLaunchKernelGGL(block_ipm_kernel<12>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 16)
        hipLaunchKernelGGL(block_ipm_kernel<16>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 20)
        hipLaunchKernelGGL(block_ipm_kernel<20>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 24)
        hipLaunchKernelGGL(block_ipm_kernel<24>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 32)
        hipLaunchKernelGGL(block_ipm_kernel<32>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 40)
        hipLaunchKernelGGL(block_ipm_kernel<40>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 48)
        hipLaunchKernelGGL(block_ipm_kernel<48>, dim3(blocks), dim3(kBT), 0, st, a);
    else if (a.n <= 56)
        hipLaunchKernelGGL(block_ipm_kernel<56>, dim3(blocks), dim3(kBT), 0, st, a);
    else
        hipLaunchKernelGGL(block_ipm_kernel<64>, dim3(blocks), dim3(kBT), 0, st, a);
    return hipGetLastError();
}

}  // namespace cr
