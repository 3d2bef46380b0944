// gfx950 kernels for the dual-smoothing (P-APG) convex-regression fit.
//
// The hot loop is one sweep over all N^2 pairs per iteration (pass_kernel, mode PASS_STEP).
// A workgroup owns 64 rows i (four waves of 16) and one chunk of columns j.  For every tile of
// 16 columns a wave
//   1. forms the transposed residual tile S^T = X_J Xi_I^T with FP64 (or FP32) MFMA 16x16x4,
//      so each lane holds 4 consecutive columns j of one row i;
//   2. reads lam^{k-1} and lam^{k-2} for those 4 pairs (32 contiguous bytes in FP64), forms
//      lam~^k, s_ij = y_j - y_i + xi_i^T x_i - xi_i^T x_j, the projected step lam^k and the
//      next extrapolated point lam~^{k+1}, and writes lam^k over lam^{k-2};
//   3. feeds lam~^{k+1} straight back into a second MFMA, (Lam~ Xhat)_I += Lam~_IJ Xhat_J,
//      where Xhat carries a column of ones so that the same product yields the row sums;
//   4. reduces the column sums of the tile across the 16 lanes of each lane group.
// The multipliers are therefore read twice and written once per iteration (the HBM floor
// of a two-state momentum method); X tiles are staged once per workgroup in LDS.  Column
// sums and (Lam X) rows leave the workgroup as partials that finalize_kernel reduces in a
// fixed order, so every iteration is bitwise reproducible.

#include "cr_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace cr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---- multiplier storage -------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// Round-to-nearest-even; values here are finite and non-negative.
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename LT, typename T> struct Store;
template <typename T> struct Store<double, T> {
    __device__ __forceinline__ static T quant(T v) { return v; }
    __device__ __forceinline__ static void load4(const double *p, T v[4]) {
        const d4 q = *reinterpret_cast<const d4 *>(p);
        v[0] = (T)q[0]; v[1] = (T)q[1]; v[2] = (T)q[2]; v[3] = (T)q[3];
    }
    __device__ __forceinline__ static void store4(double *p, const T v[4]) {
        d4 q = {(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
        *reinterpret_cast<d4 *>(p) = q;
    }
};
template <typename T> struct Store<float, T> {
    __device__ __forceinline__ static T quant(T v) { return (T)(float)v; }
    __device__ __forceinline__ static void load4(const float *p, T v[4]) {
        const f4 q = *reinterpret_cast<const f4 *>(p);
        v[0] = (T)q[0]; v[1] = (T)q[1]; v[2] = (T)q[2]; v[3] = (T)q[3];
    }
    __device__ __forceinline__ static void store4(float *p, const T v[4]) {
        f4 q = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        *reinterpret_cast<f4 *>(p) = q;
    }
};
template <typename T> struct Store<bf16_t, T> {
    __device__ __forceinline__ static T quant(T v) { return (T)bf16_to_float(float_to_bf16((float)v)); }
    __device__ __forceinline__ static void load4(const bf16_t *p, T v[4]) {
        const uint2 q = *reinterpret_cast<const uint2 *>(p);
        v[0] = (T)bf16_to_float((uint16_t)(q.x & 0xFFFFu));
        v[1] = (T)bf16_to_float((uint16_t)(q.x >> 16));
        v[2] = (T)bf16_to_float((uint16_t)(q.y & 0xFFFFu));
        v[3] = (T)bf16_to_float((uint16_t)(q.y >> 16));
    }
    __device__ __forceinline__ static void store4(bf16_t *p, const T v[4]) {
        uint2 q;
        q.x = (uint32_t)float_to_bf16((float)v[0]) | ((uint32_t)float_to_bf16((float)v[1]) << 16);
        q.y = (uint32_t)float_to_bf16((float)v[2]) | ((uint32_t)float_to_bf16((float)v[3]) << 16);
        *reinterpret_cast<uint2 *>(p) = q;
    }
};

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, 64); }

// ---- the pair sweep -----------------------------------------------------------------------
template <typename T, typename LT, int MODE, int MB>
__global__ __launch_bounds__(256) void pass_kernel(PassArgs a, Geometry g) {
    constexpr int NP = 16 * MB;
    constexpr int SX = NP + 1;                       // LDS row stride (elements)
    constexpr bool kAdjoint = (MODE == PASS_STEP || MODE == PASS_ADJ || MODE == PASS_POWER);
    constexpr bool kResidual = (MODE != PASS_ADJ);
    constexpr bool kStoreS = (MODE == PASS_RESID);
    typedef typename Vec4<T>::type V4;

    __shared__ T sX[kSuper * SX];
    __shared__ T sY[kSuper];
    __shared__ T sCol[kWaves * kSuper];
    __shared__ int sArg[MODE == PASS_REPAIR ? kWaves * kSuper : 1];
    __shared__ double sRed[kWaves * kRed];

    const T *xhat = static_cast<const T *>(a.xhat);
    const T *xi = static_cast<const T *>(a.xi);
    const T *yv = static_cast<const T *>(a.yv);
    const T *dmy = static_cast<const T *>(a.dmy);
    const LT *lam_a = static_cast<const LT *>(a.lam_a);
    LT *lam_b = static_cast<LT *>(a.lam_b);

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, lr = l & 15, lq = l >> 4;
    const int chunk = blockIdx.x % g.chunks;        // consecutive workgroups: one chunk per XCD
    const int strip = blockIdx.x / g.chunks;
    const int i = strip * kRows + w * 16 + lr;      // < Nr always
    const bool row_ok = i < g.N;
    const int cbeg = chunk * g.chunk_cols;
    const int cend = min(g.ld, cbeg + g.chunk_cols);
    const T bp = (T)a.beta_prev, bn = (T)a.beta_next, invL = (T)a.inv_L;
    // Output rows of the 16x16x4 MFMA: the FP32 form gives lane group lq rows 4 lq + v, the FP64
    // form rows 4 v + lq.  Feeding A-row rho from source row perm(rho) = 4 (rho % 4) + rho / 4
    // in the FP64 case makes both end with rows 4 lq + v (four consecutive columns per lane).
    const int arow = (sizeof(T) == 8) ? (((lr & 3) << 2) | (lr >> 2)) : lr;

    // Row-constant operands: B of the residual contraction is Xi[i][4s + lq].
    T bxi[4 * MB];
#pragma unroll
    for (int s = 0; s < 4 * MB; ++s)
        bxi[s] = (kResidual && s < g.ks1) ? xi[(size_t)i * NP + 4 * s + lq] : (T)0;
    const T dmy_i = kResidual ? dmy[i] : (T)0;

    V4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = V4{0, 0, 0, 0};
    double red0 = 0.0, red1 = 0.0, red2 = 0.0, red3 = 0.0;

    const size_t rowoff = (size_t)i * g.ld;

    for (int cst = cbeg; cst < cend; cst += kSuper) {
        __syncthreads();
        if ((kAdjoint || MODE == PASS_REPAIR) && cst > cbeg && tid < kSuper) {
            const int j = cst - kSuper + tid;
            if (MODE == PASS_REPAIR) {
                double best = (double)sCol[tid];
                int arg = sArg[tid];
                for (int ww = 1; ww < kWaves; ++ww) {
                    const double v = (double)sCol[ww * kSuper + tid];
                    if (v < best) { best = v; arg = sArg[ww * kSuper + tid]; }
                }
                a.part_min[(size_t)strip * g.ld + j] = best;
                a.part_arg[(size_t)strip * g.ld + j] = arg;
            } else {
                T v = sCol[tid];
                for (int ww = 1; ww < kWaves; ++ww) v += sCol[ww * kSuper + tid];
                static_cast<T *>(a.part_col)[(size_t)strip * g.ld + j] = v;
            }
        }
        for (int e = tid; e < kSuper * NP; e += 256) {
            const int jj = e / NP, m = e - jj * NP;
            sX[jj * SX + m] = xhat[(size_t)(cst + jj) * NP + m];
        }
        if (tid < kSuper) sY[tid] = kResidual ? yv[cst + tid] : (T)0;
        __syncthreads();

#pragma unroll
        for (int t = 0; t < kSuper / 16; ++t) {
            const int jl = t * 16;
            const int jc = jl + 4 * lq;              // local column of r = 0
            const int j0 = cst + jc;                 // global column of r = 0

            V4 S = V4{0, 0, 0, 0};
            if (kResidual) {
#pragma unroll
                for (int s = 0; s < 4 * MB; ++s)
                    if (s < g.ks1) S = mfma16(sX[(jl + arow) * SX + 4 * s + lq], bxi[s], S);
            }

            T P[4] = {0, 0, 0, 0}, Q[4] = {0, 0, 0, 0};
            if (MODE == PASS_STEP || MODE == PASS_ADJ || MODE == PASS_KKT)
                Store<LT, T>::load4(lam_a + rowoff + j0, P);
            if (MODE == PASS_STEP) Store<LT, T>::load4(lam_b + rowoff + j0, Q);

            T out[4];
            T newlam[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + r;
                const bool ok = row_ok && (j < g.N) && (j != i);
                const T s = (sY[jc + r] + dmy_i) - S[r];
                if (MODE == PASS_STEP) {
                    const T lt = P[r] + bp * (P[r] - Q[r]);            // lam~^k
                    T ln = lt - s * invL;                              // Step 2
                    ln = ln > (T)0 ? ln : (T)0;
                    ln = ok ? ln : (T)0;
                    ln = Store<LT, T>::quant(ln);                      // value as stored
                    newlam[r] = ln;
                    const T nx = ln + bn * (ln - P[r]);                // Step 4
                    out[r] = ok ? nx : (T)0;
                } else if (MODE == PASS_ADJ) {
                    out[r] = ok ? P[r] : (T)0;
                } else if (MODE == PASS_POWER) {
                    const T z = ok ? s : (T)0;
                    out[r] = z;
                    red0 += (double)z * (double)z;
                } else if (MODE == PASS_KKT) {
                    if (ok) {
                        const double ds = (double)s, dl = (double)P[r];
                        const double mn = fabs(dl < ds ? dl : ds);
                        red0 = red0 > mn ? red0 : mn;
                        red1 = red1 > -ds ? red1 : -ds;
                        const double ng = ds < 0.0 ? ds : 0.0;
                        red2 += ng * ng;
                        red3 += dl * ds;
                    }
                    out[r] = (T)0;
                } else if (MODE == PASS_REPAIR) {
                    out[r] = ok ? s : (T)INFINITY;
                } else {  // PASS_RESID
                    newlam[r] = ok ? s : (T)0;
                    out[r] = (T)0;
                }
            }
            if (MODE == PASS_STEP || kStoreS) Store<LT, T>::store4(lam_b + rowoff + j0, newlam);

            if (kAdjoint) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[mb] = mfma16(sX[(jc + r) * SX + 16 * mb + arow], out[r], acc[mb]);
                T c[4] = {out[0], out[1], out[2], out[3]};
#pragma unroll
                for (int m = 1; m < 16; m <<= 1)
#pragma unroll
                    for (int r = 0; r < 4; ++r) c[r] += shfl_xor(c[r], m);
                if (lr == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sCol[w * kSuper + jc + r] = c[r];
                }
            } else if (MODE == PASS_REPAIR) {
                // column minimum over the 16 rows of this wave, lowest row on ties
                T v[4] = {out[0], out[1], out[2], out[3]};
                int arg[4] = {i, i, i, i};
#pragma unroll
                for (int m = 1; m < 16; m <<= 1)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const T ov = shfl_xor(v[r], m);
                        const int oa = __shfl_xor(arg[r], m, 64);
                        if (ov < v[r] || (ov == v[r] && oa < arg[r])) { v[r] = ov; arg[r] = oa; }
                    }
                if (lr == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        sCol[w * kSuper + jc + r] = v[r];
                        sArg[w * kSuper + jc + r] = arg[r];
                    }
                }
            }
        }
    }

    // last super tile's column partials
    __syncthreads();
    if ((kAdjoint || MODE == PASS_REPAIR) && tid < kSuper && cend > cbeg) {
        const int j = cend - kSuper + tid;
        if (MODE == PASS_REPAIR) {
            double best = (double)sCol[tid];
            int arg = sArg[tid];
            for (int ww = 1; ww < kWaves; ++ww) {
                const double v = (double)sCol[ww * kSuper + tid];
                if (v < best) { best = v; arg = sArg[ww * kSuper + tid]; }
            }
            a.part_min[(size_t)strip * g.ld + j] = best;
            a.part_arg[(size_t)strip * g.ld + j] = arg;
        } else {
            T v = sCol[tid];
            for (int ww = 1; ww < kWaves; ++ww) v += sCol[ww * kSuper + tid];
            static_cast<T *>(a.part_col)[(size_t)strip * g.ld + j] = v;
        }
    }

    if (kAdjoint) {
        // D layout: lane (lr, lq) holds rows m = 16 mb + 4 lq + r of (Lam Xhat)^T for row i.
        T *pacc = static_cast<T *>(a.part_acc) + ((size_t)chunk * g.Nr + i) * NP;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            T v[4] = {acc[mb][0], acc[mb][1], acc[mb][2], acc[mb][3]};
            if (sizeof(T) == 8) {
                *reinterpret_cast<d4 *>(reinterpret_cast<double *>(pacc) + 16 * mb + 4 * lq) =
                    d4{(double)v[0], (double)v[1], (double)v[2], (double)v[3]};
            } else {
                *reinterpret_cast<f4 *>(reinterpret_cast<float *>(pacc) + 16 * mb + 4 * lq) =
                    f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
            }
        }
    }

    if (MODE == PASS_KKT || MODE == PASS_POWER) {
        for (int m = 32; m >= 1; m >>= 1) {
            red0 = (MODE == PASS_KKT) ? fmax(red0, __shfl_xor(red0, m, 64)) : red0 + __shfl_xor(red0, m, 64);
            red1 = fmax(red1, __shfl_xor(red1, m, 64));
            red2 += __shfl_xor(red2, m, 64);
            red3 += __shfl_xor(red3, m, 64);
        }
        if (l == 0) {
            sRed[w * kRed + 0] = red0;
            sRed[w * kRed + 1] = red1;
            sRed[w * kRed + 2] = red2;
            sRed[w * kRed + 3] = red3;
        }
        __syncthreads();
        if (tid < kRed) {
            double v = sRed[tid];
            for (int ww = 1; ww < kWaves; ++ww) {
                const double o = sRed[ww * kRed + tid];
                if (MODE == PASS_KKT && tid < 2) v = fmax(v, o);
                else v += o;
            }
            a.part_red[(size_t)blockIdx.x * kRed + tid] = v;
        }
    }
}

Geometry make_geometry(int N, int n) {
    Geometry g;
    g.N = N;
    g.n = n;
    g.MB = (n + 1 + 15) / 16;
    g.NP = 16 * g.MB;
    g.ks1 = (n + 3) / 4;
    g.Nr = ((N + kRows - 1) / kRows) * kRows;
    g.ld = g.Nr;
    g.strips = g.Nr / kRows;
    const int supers = g.ld / kSuper;
    int chunks = supers < 8 ? supers : 8;
    int per = (supers + chunks - 1) / chunks;
    g.chunk_cols = per * kSuper;
    g.chunks = (g.ld + g.chunk_cols - 1) / g.chunk_cols;
    return g;
}

template <typename T, typename LT, int MODE>
static hipError_t launch_mb(const Geometry &g, const PassArgs &a, hipStream_t st) {
    dim3 grid(g.grid()), block(256);
    switch (g.MB) {
    case 1: hipLaunchKernelGGL((pass_kernel<T, LT, MODE, 1>), grid, block, 0, st, a, g); break;
    case 2: hipLaunchKernelGGL((pass_kernel<T, LT, MODE, 2>), grid, block, 0, st, a, g); break;
    case 3: hipLaunchKernelGGL((pass_kernel<T, LT, MODE, 3>), grid, block, 0, st, a, g); break;
    case 4: hipLaunchKernelGGL((pass_kernel<T, LT, MODE, 4>), grid, block, 0, st, a, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pass(const Geometry &g, PassMode mode, bool fp32, LamType lt, const PassArgs &a,
                       hipStream_t st) {
    if (g.MB < 1 || g.MB > kMaxMB) return hipErrorInvalidValue;
    switch (mode) {
    case PASS_STEP:
        if (!fp32 && lt == LAM_F64) return launch_mb<double, double, PASS_STEP>(g, a, st);
        if (fp32 && lt == LAM_F32) return launch_mb<float, float, PASS_STEP>(g, a, st);
        if (fp32 && lt == LAM_BF16) return launch_mb<float, bf16_t, PASS_STEP>(g, a, st);
        return hipErrorInvalidValue;
    case PASS_ADJ:
        if (fp32) return hipErrorInvalidValue;
        if (lt == LAM_F64) return launch_mb<double, double, PASS_ADJ>(g, a, st);
        if (lt == LAM_F32) return launch_mb<double, float, PASS_ADJ>(g, a, st);
        return launch_mb<double, bf16_t, PASS_ADJ>(g, a, st);
    case PASS_KKT:
        if (fp32) return hipErrorInvalidValue;
        if (lt == LAM_F64) return launch_mb<double, double, PASS_KKT>(g, a, st);
        if (lt == LAM_F32) return launch_mb<double, float, PASS_KKT>(g, a, st);
        return launch_mb<double, bf16_t, PASS_KKT>(g, a, st);
    case PASS_POWER:
        if (fp32) return hipErrorInvalidValue;
        return launch_mb<double, double, PASS_POWER>(g, a, st);
    case PASS_REPAIR:
        if (fp32) return hipErrorInvalidValue;
        return launch_mb<double, double, PASS_REPAIR>(g, a, st);
    case PASS_RESID:
        if (fp32 || lt != LAM_F64) return hipErrorInvalidValue;
        return launch_mb<double, double, PASS_RESID>(g, a, st);
    }
    return hipErrorInvalidValue;
}

// ---- finalize: partial sums -> primal point ------------------------------------------------
// 16 threads per row; thread t handles features m = 16 mb + t.
template <typename T, int MB>
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a, Geometry g) {
    constexpr int NP = 16 * MB;
    const int t = threadIdx.x & 15;
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4);   // grid covers Nr exactly
    const T *pacc = static_cast<const T *>(a.part_acc);
    const T *pcol = static_cast<const T *>(a.part_col);

    double lx[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        double s = 0.0;
        for (int c = 0; c < g.chunks; ++c) s += (double)pacc[((size_t)c * g.Nr + i) * NP + 16 * mb + t];
        lx[mb] = s;
    }
    // row sum = (Lam Xhat)_{i, n}
    double mine = 0.0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
        if (16 * mb + t == g.n) mine = lx[mb];
    double rsum = mine;
    for (int m = 1; m < 16; m <<= 1) rsum += __shfl_xor(rsum, m, 16);
    // column sum over strips, split across the 16 threads then combined (fixed order)
    double csum = 0.0;
    for (int s = t; s < g.strips; s += 16) csum += (double)pcol[(size_t)s * g.ld + i];
    for (int m = 1; m < 16; m <<= 1) csum += __shfl_xor(csum, m, 16);

    const bool valid = i < g.N;
    const double u = csum - rsum;
    const double yi = valid ? (a.power ? u : a.ybar[i] + u) : 0.0;
    double xv[MB];
    double d = 0.0, xsq = 0.0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int m = 16 * mb + t;
        double v = 0.0;
        if (valid && m < g.n) {
            const double xm = a.xf[(size_t)i * NP + m];
            v = rsum * xm - lx[mb];
            if (!a.power) v *= a.inv_delta;
            d += v * xm;
            xsq += v * v;
        }
        xv[mb] = v;
    }
    for (int m = 1; m < 16; m <<= 1) {
        d += __shfl_xor(d, m, 16);
        xsq += __shfl_xor(xsq, m, 16);
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        a.xi[(size_t)i * NP + 16 * mb + t] = xv[mb];
        if (a.xi32) a.xi32[(size_t)i * NP + 16 * mb + t] = (float)xv[mb];
    }
    if (t == 0) {
        a.y[i] = yi;
        a.dmy[i] = valid ? d - yi : 0.0;
        if (a.y32) a.y32[i] = (float)yi;
        if (a.dmy32) a.dmy32[i] = valid ? (float)(d - yi) : 0.f;
        if (a.rowred) {
            const double dy = a.power ? yi : (valid ? yi - a.ybar[i] : 0.0);
            a.rowred[2 * (size_t)i] = dy * dy;
            a.rowred[2 * (size_t)i + 1] = xsq;
        }
    }
}

hipError_t launch_finalize(const Geometry &g, bool fp32, const FinalizeArgs &a, hipStream_t st) {
    dim3 grid(g.Nr / 16), block(256);
#define CR_FIN(T, MBV) hipLaunchKernelGGL((finalize_kernel<T, MBV>), grid, block, 0, st, a, g)
    if (fp32) {
        switch (g.MB) { case 1: CR_FIN(float, 1); break; case 2: CR_FIN(float, 2); break;
                        case 3: CR_FIN(float, 3); break; case 4: CR_FIN(float, 4); break;
                        default: return hipErrorInvalidValue; }
    } else {
        switch (g.MB) { case 1: CR_FIN(double, 1); break; case 2: CR_FIN(double, 2); break;
                        case 3: CR_FIN(double, 3); break; case 4: CR_FIN(double, 4); break;
                        default: return hipErrorInvalidValue; }
    }
#undef CR_FIN
    return hipGetLastError();
}

// ---- small reductions -------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(const double *part, int blocks, int stride,
                                                     int nmax, int nout, double *out) {
    __shared__ double sh[256];
    for (int q = 0; q < nout; ++q) {
        const bool isMax = q < nmax;
        double v = isMax ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < blocks; b += 256) {
            const double p = part[(size_t)b * stride + q];
            v = isMax ? fmax(v, p) : v + p;
        }
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] = isMax ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                                         : sh[threadIdx.x] + sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sh[0];
        __syncthreads();
    }
}

hipError_t launch_reduce(const double *part, int blocks, int stride, int nmax, int nout, double *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, st, part, blocks, stride, nmax, nout, out);
    return hipGetLastError();
}

__global__ void normalize_kernel(double *y, double *xi, double *dmy, const double *sq, int Nr, int NP) {
    const double f = 1.0 / sqrt(sq[0] + sq[1]);
    const size_t tot = (size_t)Nr * NP;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        xi[e] *= f;
        if (e < (size_t)Nr) { y[e] *= f; dmy[e] *= f; }
    }
}

hipError_t launch_normalize(const Geometry &g, double *y, double *xi, double *dmy, const double *sq,
                            hipStream_t st) {
    const int blocks = (int)(((size_t)g.Nr * g.NP + 255) / 256);
    hipLaunchKernelGGL(normalize_kernel, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, st, y, xi,
                       dmy, sq, g.Nr, g.NP);
    return hipGetLastError();
}

// ---- conversions and packing ------------------------------------------------------------------
__device__ __forceinline__ double load_lam(const void *p, LamType t, size_t e) {
    if (t == LAM_F64) return static_cast<const double *>(p)[e];
    if (t == LAM_F32) return (double)static_cast<const float *>(p)[e];
    return (double)bf16_to_float(static_cast<const uint16_t *>(p)[e]);
}
__device__ __forceinline__ void store_lam(void *p, LamType t, size_t e, double v) {
    if (t == LAM_F64) static_cast<double *>(p)[e] = v;
    else if (t == LAM_F32) static_cast<float *>(p)[e] = (float)v;
    else static_cast<uint16_t *>(p)[e] = float_to_bf16((float)v);
}

__global__ void convert_kernel(const void *src, LamType stt, void *dst, LamType dt, size_t tot) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x)
        store_lam(dst, dt, e, load_lam(src, stt, e));
}

hipError_t launch_convert(const Geometry &g, const void *src, LamType stt, void *dst, LamType dt,
                          hipStream_t st) {
    const size_t tot = (size_t)g.Nr * g.ld;
    hipLaunchKernelGGL(convert_kernel, dim3(8192), dim3(256), 0, st, src, stt, dst, dt, tot);
    return hipGetLastError();
}

__global__ void pack_kernel(const double *dense, void *dst, LamType lt, int N, int Nr, int ld) {
    const size_t tot = (size_t)Nr * ld;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), j = (int)(e - (size_t)i * ld);
        double v = 0.0;
        if (i < N && j < N && i != j) v = dense[(size_t)i * N + j];
        store_lam(dst, lt, e, v);
    }
}

__global__ void unpack_kernel(const void *src, LamType lt, double *dense, int N, int ld) {
    const size_t tot = (size_t)N * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
        dense[e] = (i == j) ? 0.0 : load_lam(src, lt, (size_t)i * ld + j);
    }
}

hipError_t launch_pack_lambda(const Geometry &g, const double *dense, void *dst, LamType lt, hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(8192), dim3(256), 0, st, dense, dst, lt, g.N, g.Nr, g.ld);
    return hipGetLastError();
}

hipError_t launch_unpack_lambda(const Geometry &g, const void *src, LamType lt, double *dense, hipStream_t st) {
    hipLaunchKernelGGL(unpack_kernel, dim3(8192), dim3(256), 0, st, src, lt, dense, g.N, g.ld);
    return hipGetLastError();
}

__global__ void prepare_kernel(const double *x, const double *ybar, const double *mu, double *xhat64,
                               float *xhat32, double *ybar_pad, int N, int n, int Nr, int NP) {
    const size_t tot = (size_t)Nr * NP;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / NP), m = (int)(e - (size_t)i * NP);
        double v = 0.0;
        if (i < N) {
            if (m < n) v = mu ? x[(size_t)i * n + m] - mu[m] : x[(size_t)i * n + m];
            else if (m == n) v = 1.0;
        }
        xhat64[e] = v;
        if (xhat32) xhat32[e] = (float)v;
        if (ybar_pad && m == 0) ybar_pad[i] = (i < N) ? ybar[i] : 0.0;
    }
}

hipError_t launch_prepare(const Geometry &g, const double *x, const double *ybar, const double *mu,
                          double *xhat64, float *xhat32, double *ybar_pad, hipStream_t st) {
    const int blocks = (int)(((size_t)g.Nr * g.NP + 255) / 256);
    hipLaunchKernelGGL(prepare_kernel, dim3(blocks < 8192 ? blocks : 8192), dim3(256), 0, st, x, ybar, mu,
                       xhat64, xhat32, ybar_pad, g.N, g.n, g.Nr, g.NP);
    return hipGetLastError();
}

// One thread per padded row; thread-local sums only.
__global__ void power_init_kernel(const double *xhat64, double *y, double *xi, double *dmy, int N, int n,
                                  int Nr, int NP, double inv_norm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nr) return;
    double vy = 0.0, d = 0.0;
    if (i < N) {
        vy = (N > 1 ? -1.0 + 2.0 * (double)i / (double)(N - 1) : 0.0) * inv_norm;
        for (int m = 0; m < n; ++m) d += inv_norm * xhat64[(size_t)i * NP + m];
    }
    for (int m = 0; m < NP; ++m) xi[(size_t)i * NP + m] = (i < N && m < n) ? inv_norm : 0.0;
    y[i] = vy;
    dmy[i] = d - vy;
}

hipError_t launch_power_init(const Geometry &g, const double *xhat64, double *y, double *xi, double *dmy,
                             hipStream_t st) {
    // ||v||^2 = sum_l (-1 + 2l/(N-1))^2 + N n, summed on the host in a fixed order
    double s = 0.0;
    for (int l = 0; l < g.N; ++l) {
        const double v = g.N > 1 ? -1.0 + 2.0 * (double)l / (double)(g.N - 1) : 0.0;
        s += v * v;
    }
    s += (double)g.N * (double)g.n;
    hipLaunchKernelGGL(power_init_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, xhat64, y, xi, dmy, g.N,
                       g.n, g.Nr, g.NP, 1.0 / sqrt(s));
    return hipGetLastError();
}

__global__ void pad_primal_kernel(const double *y_in, const double *xi_in, const double *xhat64, double *y,
                                  double *xi, double *dmy, int N, int n, int Nr, int NP) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nr) return;
    double d = 0.0;
    for (int m = 0; m < NP; ++m) {
        const double v = (i < N && m < n) ? xi_in[(size_t)i * n + m] : 0.0;
        xi[(size_t)i * NP + m] = v;
        if (m < n) d += v * xhat64[(size_t)i * NP + m];
    }
    const double yy = i < N ? y_in[i] : 0.0;
    y[i] = yy;
    dmy[i] = i < N ? d - yy : 0.0;
}

hipError_t launch_pad_primal(const Geometry &g, const double *y_in, const double *xi_in, const double *xhat64,
                             double *y, double *xi, double *dmy, hipStream_t st) {
    hipLaunchKernelGGL(pad_primal_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, y_in, xi_in, xhat64, y, xi,
                       dmy, g.N, g.n, g.Nr, g.NP);
    return hipGetLastError();
}

// Column j: minimum over strips (ascending strip order, strictly smaller wins, so the lowest
// row index is kept on ties); the piece is j itself unless the minimum is negative.
__global__ void repair_finish_kernel(const double *part_min, const int *part_arg, const double *y,
                                     const double *xi, const double *ybar, double *y_rep, double *xi_rep,
                                     double *rowred, int N, int Nr, int ld, int strips, int NP) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Nr) return;
    if (j >= N) {
        y_rep[j] = 0.0;
        for (int m = 0; m < NP; ++m) xi_rep[(size_t)j * NP + m] = 0.0;
        rowred[2 * (size_t)j] = 0.0;
        rowred[2 * (size_t)j + 1] = 0.0;
        return;
    }
    double best = INFINITY;
    int arg = j;
    for (int s = 0; s < strips; ++s) {
        const double v = part_min[(size_t)s * ld + j];
        if (v < best) { best = v; arg = part_arg[(size_t)s * ld + j]; }
    }
    const double shift = best < 0.0 ? best : 0.0;
    const int piece = best < 0.0 ? arg : j;
    const double yr = y[j] - shift;
    y_rep[j] = yr;
    double xsq = 0.0;
    for (int m = 0; m < NP; ++m) {
        const double v = xi[(size_t)piece * NP + m];
        xi_rep[(size_t)j * NP + m] = v;
        xsq += v * v;
    }
    const double dy = yr - ybar[j];
    rowred[2 * (size_t)j] = dy * dy;
    rowred[2 * (size_t)j + 1] = xsq;
}

hipError_t launch_repair_finish(const Geometry &g, const double *part_min, const int *part_arg, const double *y,
                                const double *xi, const double *ybar, double *y_rep, double *xi_rep,
                                double *rowred, hipStream_t st) {
    hipLaunchKernelGGL(repair_finish_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, part_min, part_arg, y, xi,
                       ybar, y_rep, xi_rep, rowred, g.N, g.Nr, g.ld, g.strips, g.NP);
    return hipGetLastError();
}

__global__ void unpad_kernel(const double *y, const double *xi, double *y_out, double *xi_out, int N, int n, int NP) {
    const size_t tot = (size_t)N * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), m = (int)(e - (size_t)i * n);
        xi_out[e] = xi[(size_t)i * NP + m];
        if (m == 0) y_out[i] = y[i];
    }
}

hipError_t launch_unpad_primal(const Geometry &g, const double *y, const double *xi, double *y_out,
                               double *xi_out, hipStream_t st) {
    const size_t tot = (size_t)g.N * g.n;
    const int blocks = (int)((tot + 255) / 256);
    hipLaunchKernelGGL(unpad_kernel, dim3(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096), dim3(256), 0, st, y,
                       xi, y_out, xi_out, g.N, g.n, g.NP);
    return hipGetLastError();
}

__global__ void combine_kernel(const double *ya, const double *xia, const double *yb, const double *xib,
                               const double *xhat64, double b, double *y, double *xi, double *dmy, float *y32,
                               float *xi32, float *dmy32, int N, int n, int Nr, int NP) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nr) return;
    double d = 0.0;
    for (int m = 0; m < NP; ++m) {
        const size_t e = (size_t)i * NP + m;
        const double v = (1.0 + b) * xia[e] - b * xib[e];
        xi[e] = v;
        if (xi32) xi32[e] = (float)v;
        if (m < n) d += v * xhat64[e];
    }
    const double yy = (1.0 + b) * ya[i] - b * yb[i];
    y[i] = yy;
    dmy[i] = i < N ? d - yy : 0.0;
    if (y32) y32[i] = (float)yy;
    if (dmy32) dmy32[i] = i < N ? (float)(d - yy) : 0.f;
}

hipError_t launch_combine(const Geometry &g, const double *ya, const double *xia, const double *yb,
                          const double *xib, const double *ybar, const double *xhat64, double b, double *y,
                          double *xi, double *dmy, float *y32, float *xi32, float *dmy32, hipStream_t st) {
    (void)ybar;
    hipLaunchKernelGGL(combine_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, ya, xia, yb, xib, xhat64, b, y,
                       xi, dmy, y32, xi32, dmy32, g.N, g.n, g.Nr, g.NP);
    return hipGetLastError();
}

}  // namespace cr
