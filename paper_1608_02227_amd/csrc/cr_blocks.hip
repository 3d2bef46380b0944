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
// Layout and work split: S (at most kMaxBlock^2 doubles) and the block's locations live in LDS; S is
// factored and its triangular solves run on the whole workgroup; each point's n x n block is
// factored by one thread; V_a = F_a^-1 M0a^T (n x p per point) and the other per-block arrays live
// in a global workspace.  Every loop has a trip count uniform over the workgroup and every barrier
// is reached by all threads.

#include "cr_kernels.h"

#include <hip/hip_runtime.h>

namespace cr {
namespace {

constexpr int kBT = 256;   // threads per workgroup (4 waves)

// Workgroup reductions (all threads call; `sh` holds 4 doubles).
__device__ __forceinline__ double wg_sum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__device__ __forceinline__ double wg_max(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}
__device__ __forceinline__ double wg_min(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
}

// Per-block arrays in the global workspace (q points, n features; P2 = q^2 pair slots, the
// diagonal slots unused).
struct BlockWs {
    double *sl, *th, *dd, *rp, *dsa, *dta, *dsv;   // P2 each: slack, multiplier, theta/s, r_p, affine
                                                   // steps (slack, multiplier), the step's slack change
    double *V;      // q * n * q: V[(a n + m) q + c] = (F_a^-1 M0a^T)[m][c]
    double *F;      // q * n * n: Cholesky factor of M_aa (lower, row-major)
    double *y, *xi, *y0, *xi0, *ry, *rxi, *gv, *by, *bxi, *dy, *dxi, *zz, *r0;
};

__device__ __forceinline__ BlockWs carve(double *W, int q, int n) {
    const size_t P2 = (size_t)q * q, qn = (size_t)q * n;
    BlockWs w;
    w.sl = W; w.th = w.sl + P2; w.dd = w.th + P2; w.rp = w.dd + P2; w.dsa = w.rp + P2; w.dta = w.dsa + P2;
    w.dsv = w.dta + P2;
    w.V = w.dsv + P2;
    w.F = w.V + qn * q;
    w.y = w.F + qn * n; w.xi = w.y + q; w.y0 = w.xi + qn; w.xi0 = w.y0 + q;
    w.ry = w.xi0 + qn; w.rxi = w.ry + q; w.gv = w.rxi + qn; w.by = w.gv + qn; w.bxi = w.by + q;
    w.dy = w.bxi + qn; w.dxi = w.dy + q; w.zz = w.dxi + qn; w.r0 = w.zz + qn;
    return w;
}

}  // namespace

size_t block_ws_doubles(int p, int n) {
    const size_t P2 = (size_t)p * p, qn = (size_t)p * n;
    return 7 * P2 + qn * p + qn * n + 6 * (size_t)p + 8 * qn + 64;
}

namespace {

__global__ __launch_bounds__(kBT) void block_ipm_kernel(BlockProjArgs A) {
    __shared__ double sS[kMaxBlock * kMaxBlock];   // the Schur complement, then its Cholesky factor
    __shared__ double sX[kMaxBlock * 16 * kMaxMB];  // the block's locations, point-major
    __shared__ double sv[kMaxBlock];                // right-hand side / solution of the S system
    __shared__ double sdg[kMaxBlock];               // diagonal of M00 (pivot floor of S)
    __shared__ double sh[4];
    const int b = blockIdx.x, t = threadIdx.x;
    const int i0 = b * A.p;
    const int q = min(A.p, A.N - i0);
    const int n = A.n, NP = A.NP;
    const double delta = A.delta;
    if (q <= 0) return;                       // uniform over the workgroup
    const size_t P2 = (size_t)q * q;
    BlockWs w = carve(A.ws + (size_t)b * A.ws_doubles, q, n);
    auto X = [&](int a, int m) -> double { return sX[a * n + m]; };

    // eta0 in, and the starting point of the IPM: eta = eta0, s = max(A eta0, 1), theta = 1
    for (int e = t; e < q; e += kBT) { w.y0[e] = A.y[i0 + e]; w.y[e] = w.y0[e]; }
    for (int e = t; e < q * n; e += kBT) {
        const int a = e / n, m = e - a * n;
        w.xi0[e] = A.xi[(size_t)(i0 + a) * NP + m];
        w.xi[e] = w.xi0[e];
        sX[e] = A.xhat[(size_t)(i0 + a) * NP + m];
    }
    __syncthreads();
    // s_ac of the current eta
    auto lin = [&](int a, int c) -> double {
        double v = w.y[c] - w.y[a];
        for (int m = 0; m < n; ++m) v += w.xi[a * n + m] * (X(a, m) - X(c, m));
        return v;
    };
    double ysc = 0.0;
    for (int e = t; e < q; e += kBT) ysc = fmax(ysc, fabs(w.y0[e]));
    for (int e = t; e < (int)P2; e += kBT) {
        const int a = e / q, c = e - a * q;
        if (a == c) { w.sl[e] = 1.0; w.th[e] = 0.0; continue; }
        const double v = lin(a, c);
        ysc = fmax(ysc, fabs(v));
        w.sl[e] = fmax(v, 1.0);
        w.th[e] = 1.0;
    }
    const double scale = 1.0 + wg_max(ysc, sh);
    const double tol = A.tol * scale;
    // complementarity target: a weakly active constraint keeps a slack near sqrt(mu), so mu is
    // driven three orders below tol^2-like units of the block's scale
    const double tol_mu = 1e-3 * A.tol * scale * scale;
    const double mpairs = (double)q * (double)(q - 1);

    int it = 0;
    for (; it < A.max_iter && q > 1; ++it) {
        // residuals: r_p = A eta - s, mu = s^T theta / m, d = theta / s
        double rpmax = 0.0, gap = 0.0;
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            if (a == c) { w.rp[e] = 0.0; w.dd[e] = 0.0; continue; }
            const double r = lin(a, c) - w.sl[e];
            w.rp[e] = r;
            rpmax = fmax(rpmax, fabs(r));
            gap += w.sl[e] * w.th[e];
            w.dd[e] = w.th[e] / w.sl[e];
        }
        rpmax = wg_max(rpmax, sh);
        const double mu = wg_sum(gap, sh) / mpairs;
        // r_d = G eta + c - A^T theta: y part (y - y0) - (colsum - rowsum), xi part
        // delta (xi_a - xi0_a) - sum_c theta_ac (x_a - x_c); and g_a = sum_c d_ac (x_a - x_c)
        double rdmax = 0.0;
        for (int e = t; e < q; e += kBT) {
            double cs = 0.0, rs = 0.0;
            for (int c = 0; c < q; ++c) { cs += w.th[(size_t)c * q + e]; rs += w.th[(size_t)e * q + c]; }
            const double r = (w.y[e] - w.y0[e]) - (cs - rs);
            w.ry[e] = r;
            rdmax = fmax(rdmax, fabs(r));
        }
        for (int e = t; e < q * n; e += kBT) {
            const int a = e / n, m = e - a * n;
            double sth = 0.0, sd = 0.0;
            const double xa = X(a, m);
            for (int c = 0; c < q; ++c) {
                const double dx = xa - X(c, m);
                sth += w.th[(size_t)a * q + c] * dx;
                sd += w.dd[(size_t)a * q + c] * dx;
            }
            const double r = delta * (w.xi[e] - w.xi0[e]) - sth;
            w.rxi[e] = r;
            w.gv[e] = sd;
            rdmax = fmax(rdmax, fabs(r));
        }
        rdmax = wg_max(rdmax, sh);
        // uniform: the reductions broadcast
        if (rpmax <= tol && rdmax <= tol && mu <= tol_mu) break;

        // M00 into LDS (I + sum of (d_ac + d_ca)(e_c - e_a)(e_c - e_a)^T) and the xi blocks:
        // M_aa = delta I + sum_c d_ac (x_a - x_c)(x_a - x_c)^T
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            if (a != c) {
                sS[e] = -(w.dd[e] + w.dd[(size_t)c * q + a]);
            } else {
                double s = 1.0;
                for (int j = 0; j < q; ++j) s += w.dd[(size_t)a * q + j] + w.dd[(size_t)j * q + a];
                sS[e] = s;
                sdg[a] = s;
            }
        }
        for (int e = t; e < q * n * n; e += kBT) {
            const int a = e / (n * n), r = e - a * n * n, m1 = r / n, m2 = r - m1 * n;
            if (m2 > m1) continue;
            double s = (m1 == m2) ? delta : 0.0;
            const double xa1 = X(a, m1), xa2 = X(a, m2);
            for (int c = 0; c < q; ++c) s += w.dd[(size_t)a * q + c] * (xa1 - X(c, m1)) * (xa2 - X(c, m2));
            w.F[(size_t)a * n * n + m1 * n + m2] = s;
        }
        __syncthreads();
        // Cholesky of each M_aa, one thread per point (lower triangle, in place)
        for (int a = t; a < q; a += kBT) {
            double *L = w.F + (size_t)a * n * n;
            for (int k = 0; k < n; ++k) {
                double dkk = L[k * n + k];
                const double floor_k = 1e-14 * dkk;           // M_aa >= delta I: positive in exact arithmetic
                for (int j = 0; j < k; ++j) dkk -= L[k * n + j] * L[k * n + j];
                dkk = sqrt(fmax(dkk, floor_k));
                L[k * n + k] = dkk;
                for (int i = k + 1; i < n; ++i) {
                    double v = L[i * n + k];
                    for (int j = 0; j < k; ++j) v -= L[i * n + j] * L[k * n + j];
                    L[i * n + k] = v / dkk;
                }
            }
        }
        __syncthreads();
        // V_a[:, c] = F_a^-1 (M0a^T)[:, c], (M0a^T)[:, c] = d_ac (x_a - x_c) for c != a, -g_a for c = a
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            const double *L = w.F + (size_t)a * n * n;
            double *v = w.V + (size_t)a * n * q + c;          // stride q over m
            const double dac = w.dd[(size_t)a * q + c];
            for (int m = 0; m < n; ++m) {
                double r = (c == a) ? -w.gv[a * n + m] : dac * (X(a, m) - X(c, m));
                for (int j = 0; j < m; ++j) r -= L[m * n + j] * v[(size_t)j * q];
                v[(size_t)m * q] = r / L[m * n + m];
            }
        }
        __syncthreads();
        // S = M00 - sum_a V_a^T V_a
        for (int e = t; e < (int)P2; e += kBT) {
            const int c1 = e / q, c2 = e - c1 * q;
            if (c2 > c1) continue;
            double s = 0.0;
            for (int am = 0; am < q * n; ++am) s += w.V[(size_t)am * q + c1] * w.V[(size_t)am * q + c2];
            sS[e] -= s;
        }
        __syncthreads();
        // Cholesky of S in LDS (lower), the whole workgroup, one column at a time
        for (int k = 0; k < q; ++k) {
            // S is positive definite in exact arithmetic; rounding near the end of the IPM (theta / s
            // spanning many orders) is kept from a non-positive pivot by a relative floor
            if (t == 0) sS[k * q + k] = sqrt(fmax(sS[k * q + k], 1e-14 * sdg[k]));
            __syncthreads();
            const double dkk = sS[k * q + k];
            for (int i = k + 1 + t; i < q; i += kBT) sS[i * q + k] /= dkk;
            __syncthreads();
            const int rem = q - k - 1;
            for (int e = t; e < rem * rem; e += kBT) {
                const int i = k + 1 + e / rem, j = k + 1 + e % rem;
                if (j <= i) sS[i * q + j] -= sS[i * q + k] * sS[j * q + k];
            }
            __syncthreads();
        }

        // Newton system M d_eta = -r_d + A^T wv with wv = d (-r_p) + r_c / s; r_c the
        // complementarity right-hand side (predictor: -s theta; corrector adds -ds_aff dth_aff + sig mu)
        auto solve = [&](bool corrector, double sigmu) {
            // right-hand side by, bxi (A^T wv: y part colsum - rowsum, xi part sum_c wv_ac (x_a - x_c))
            auto wv = [&](int a, int c) -> double {
                const size_t e = (size_t)a * q + c;
                double rc = -w.sl[e] * w.th[e];
                if (corrector) rc += -w.dsa[e] * w.dta[e] + sigmu;
                return -w.dd[e] * w.rp[e] + rc / w.sl[e];
            };
            for (int e = t; e < q; e += kBT) {
                double cs = 0.0, rs = 0.0;
                for (int c = 0; c < q; ++c) {
                    if (c == e) continue;
                    cs += wv(c, e);
                    rs += wv(e, c);
                }
                w.by[e] = -w.ry[e] + (cs - rs);
            }
            for (int e = t; e < q * n; e += kBT) {
                const int a = e / n, m = e - a * n;
                double s = 0.0;
                const double xa = X(a, m);
                for (int c = 0; c < q; ++c)
                    if (c != a) s += wv(a, c) * (xa - X(c, m));
                w.bxi[e] = -w.rxi[e] + s;
            }
            __syncthreads();
            // z_a = M_aa^-1 b_a
            for (int a = t; a < q; a += kBT) {
                const double *L = w.F + (size_t)a * n * n;
                double *z = w.zz + (size_t)a * n;
                for (int m = 0; m < n; ++m) {
                    double r = w.bxi[a * n + m];
                    for (int j = 0; j < m; ++j) r -= L[m * n + j] * z[j];
                    z[m] = r / L[m * n + m];
                }
                for (int m = n - 1; m >= 0; --m) {
                    double r = z[m];
                    for (int j = m + 1; j < n; ++j) r -= L[j * n + m] * z[j];
                    z[m] = r / L[m * n + m];
                }
            }
            __syncthreads();
            // r0_c = by_c - sum_a (M0a z_a)_c
            for (int c = t; c < q; c += kBT) {
                double s = 0.0;
                for (int a = 0; a < q; ++a) {
                    double v = 0.0;
                    if (a == c) {
                        for (int m = 0; m < n; ++m) v -= w.gv[a * n + m] * w.zz[a * n + m];
                    } else {
                        const double dac = w.dd[(size_t)a * q + c];
                        for (int m = 0; m < n; ++m) v += (X(a, m) - X(c, m)) * w.zz[a * n + m];
                        v *= dac;
                    }
                    s += v;
                }
                w.r0[c] = w.by[c] - s;
            }
            __syncthreads();
            // dy = S^-1 r0: forward then backward substitution with the LDS factor, in LDS
            for (int e = t; e < q; e += kBT) sv[e] = w.r0[e];
            __syncthreads();
            for (int k = 0; k < q; ++k) {
                const double xk = sv[k] / sS[k * q + k];
                for (int i = k + 1 + t; i < q; i += kBT) sv[i] -= sS[i * q + k] * xk;
                __syncthreads();
                if (t == 0) sv[k] = xk;
                __syncthreads();
            }
            for (int k = q - 1; k >= 0; --k) {
                const double xk = sv[k] / sS[k * q + k];
                for (int i = t; i < k; i += kBT) sv[i] -= sS[k * q + i] * xk;
                __syncthreads();
                if (t == 0) sv[k] = xk;
                __syncthreads();
            }
            for (int e = t; e < q; e += kBT) w.dy[e] = sv[e];
            __syncthreads();
            // dxi_a = M_aa^-1 (b_a - M0a^T dy)
            for (int a = t; a < q; a += kBT) {
                const double *L = w.F + (size_t)a * n * n;
                double *z = w.dxi + (size_t)a * n;
                for (int m = 0; m < n; ++m) {
                    double s = -w.gv[a * n + m] * w.dy[a];
                    const double xa = X(a, m);
                    for (int c = 0; c < q; ++c)
                        if (c != a) s += w.dd[(size_t)a * q + c] * (xa - X(c, m)) * w.dy[c];
                    z[m] = w.bxi[a * n + m] - s;
                }
                for (int m = 0; m < n; ++m) {
                    double r = z[m];
                    for (int j = 0; j < m; ++j) r -= L[m * n + j] * z[j];
                    z[m] = r / L[m * n + m];
                }
                for (int m = n - 1; m >= 0; --m) {
                    double r = z[m];
                    for (int j = m + 1; j < n; ++j) r -= L[j * n + m] * z[j];
                    z[m] = r / L[m * n + m];
                }
            }
            __syncthreads();
        };
        // slack and multiplier steps of the solved direction; returns the largest step in (0, 1]
        // keeping both positive (before the fraction to the boundary)
        auto steps = [&](bool corrector, double sigmu, double *dsl, double *dth) -> double {
            double amax = 1.0, bad = 0.0;
            for (int e = t; e < (int)P2; e += kBT) {
                const int a = e / q, c = e - a * q;
                if (a == c) { dsl[e] = 0.0; dth[e] = 0.0; continue; }
                double adeta = w.dy[c] - w.dy[a];
                for (int m = 0; m < n; ++m) adeta += w.dxi[a * n + m] * (X(a, m) - X(c, m));
                const double dsv = adeta + w.rp[e];
                double rc = -w.sl[e] * w.th[e];
                if (corrector) rc += -w.dsa[e] * w.dta[e] + sigmu;
                const double dtv = -w.dd[e] * dsv + rc / w.sl[e];
                dsl[e] = dsv;
                dth[e] = dtv;
                if (!isfinite(dsv) || !isfinite(dtv)) bad = 1.0;
                if (dsv < 0.0) amax = fmin(amax, -w.sl[e] / dsv);
                if (dtv < 0.0) amax = fmin(amax, -w.th[e] / dtv);
            }
            // a direction with a non-finite entry ends the iteration (returned as -1)
            return wg_max(bad, sh) > 0.0 ? -1.0 : wg_min(amax, sh);
        };
        // predictor (affine scaling)
        solve(false, 0.0);
        const double aaff = steps(false, 0.0, w.dsa, w.dta);
        if (aaff < 0.0) break;
        double gaff = 0.0;
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            if (a == c) continue;
            gaff += (w.sl[e] + aaff * w.dsa[e]) * (w.th[e] + aaff * w.dta[e]);
        }
        const double muaff = wg_sum(gaff, sh) / mpairs;
        const double sig = mu > 0.0 ? fmin(1.0, (muaff / mu) * (muaff / mu) * (muaff / mu)) : 0.0;
        // corrector
        solve(true, sig * mu);
        const double amax = steps(true, sig * mu, w.dsv, w.dta);
        if (amax < 1e-12) break;   // no usable step (or a non-finite one): keep the current point
        const double alpha = fmin(1.0, 0.99 * amax);
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            if (a == c) continue;
            w.sl[e] += alpha * w.dsv[e];
            w.th[e] += alpha * w.dta[e];
        }
        for (int e = t; e < q; e += kBT) w.y[e] += alpha * w.dy[e];
        for (int e = t; e < q * n; e += kBT) w.xi[e] += alpha * w.dxi[e];
        __syncthreads();
    }
    if (t == 0 && A.iters) A.iters[b] = it;

    // the projection out: y, xi, dmy = xi^T x - y (and the rows' objective terms), and the
    // blocks' multipliers into the intra-block entries of lam
    for (int e = t; e < q; e += kBT) {
        const int i = i0 + e;
        double d = 0.0, xsq = 0.0;
        for (int m = 0; m < n; ++m) {
            const double v = w.xi[e * n + m];
            A.xi[(size_t)i * NP + m] = v;
            d += v * X(e, m);
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
        for (int e = t; e < (int)P2; e += kBT) {
            const int a = e / q, c = e - a * q;
            A.lam[(size_t)(i0 + a) * A.ld + (i0 + c)] = (a == c || w.th[e] <= w.sl[e]) ? 0.0 : w.th[e];
        }
    }
}

}  // namespace

hipError_t launch_block_project(const Geometry &g, const BlockProjArgs &a, hipStream_t st) {
    if (a.p < 1 || a.p > kMaxBlock || a.n < 1 || a.n > 16 * kMaxMB) return hipErrorInvalidValue;
    const int blocks = (g.N + a.p - 1) / a.p;
    hipLaunchKernelGGL(block_ipm_kernel, dim3(blocks), dim3(kBT), 0, st, a);
    return hipGetLastError();
}

}  // namespace cr
