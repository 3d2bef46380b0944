// gfx950 kernels for the dual-smoothing (P-APG) convex-regression fit.
//
// The hot loop is one sweep over all N^2 pairs per iteration (pass_kernel).  A workgroup owns
// 128 rows i (eight waves of 16) and one chunk of columns j.  For every tile of 16 rows x 16
// (FP64 state) or 32 (split state) columns a wave
//   1. forms the transposed residual tile S^T = X_J Xi_I^T with FP64 (or FP32) MFMA 16x16x4, the
//      accumulator starting at y_j + d_i - y_i so that it ends as s_ij; each lane holds 4 (or 8)
//      consecutive columns j of one row i;
//   2. reads the stored iterates for those pairs (whole 128-byte lines per lane group), forms
//      lam~^k, the projected step(s) and the next extrapolated point, and writes lam^k over the
//      older iterate;
//   3. feeds the result straight back into a second MFMA, (Lam~ Xhat)_I += Lam~_IJ Xhat_J,
//      where Xhat carries a column of ones so that the same product yields the row sums;
//   4. reduces the column sums of the tile across the 16 lanes of each lane group.
// The multipliers are therefore read twice and written once per iteration (the HBM floor
// of a two-state momentum method); X tiles are staged once per workgroup in LDS.  Column
// sums and (Lam X) rows leave the workgroup as partials that the finalize kernels reduce in a
// fixed order, so every iteration is bitwise reproducible.  The adaptive step's trial passes
// (PASS_TRIAL, PASS_TRIAL_NS, PASS_ADV) evaluate two candidate steps per sweep the same way.

#include "cr_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <type_traits>

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

// BF16 MFMA with K = 32: lane l holds A[l % 16][8 (l / 16) + q] and B[8 (l / 16) + q][l % 16],
// q < 8, and receives C[4 (l / 16) + v][l % 16], v < 4 (the output layout of the FP32 16x16x4 form).
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma16_bf16(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// x = hi + lo + O(2^-16 |x|) with hi, lo in BF16; a product of two such splits taken as
// hi*hi + hi*lo + lo*hi (three BF16 MFMAs, FP32 accumulation) has relative error ~3 * 2^-16.
__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// Two values at once: hi = RNE(x) in BF16 (one packed conversion for the pair), lo = RNE(x - hi);
// the same numbers as split_bf16 on each.  hp, lp receive the pair packed (first value low).
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16_pair(float x0, float x1, uint32_t &hp, uint32_t &lp) {
    hp = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{x0, x1}, b2));
    const float h0 = __uint_as_float(hp << 16), h1 = __uint_as_float(hp & 0xFFFF0000u);
    lp = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{x0 - h0, x1 - h1}, b2));
}

// FP16 MFMA with K = 16: lane l holds A[l % 16][4 (l / 16) + q] and B[4 (l / 16) + q][l % 16],
// q < 4, and receives C[4 (l / 16) + v][l % 16] (the output layout of the FP32 16x16x4 form).
// (Only this K: a chain in which a K = 16 FP16 MFMA took a K = 32 one's result as its accumulator
// gave wrong sums on this toolchain and device, and K = 16 alone is as fast here.)
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 mfma16_h16(h4 a, h4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
// x = hi + lo with hi = RNE(x) and lo = RNE(x - hi) in FP16: 22 significant bits, so for |x| < 1
// the split holds x to 2^-24 (absolute; lo leaves FP16's normal range only for |x| < 2^-3, where
// its absolute spacing is 2^-24).  Products of two splits are taken as hi*lo + lo*hi + hi*hi
// (lo*lo ~ 2^-24 dropped), each exact in FP32 and accumulated in FP32: the FP32 MFMA's accuracy
// relative to the operands' scale.
__device__ __forceinline__ void split_f16(float x, _Float16 &hi, _Float16 &lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
}
// 2^-e with 2^(e-1) <= m < 2^e (m > 0; 1 for m = 0), e clamped to [-40, 40]: scales a vector whose
// largest magnitude is m into [0.5, 1) exactly.
__device__ __forceinline__ float pow2_scale(float m) {
    if (!(m > 0.f)) return 1.f;
    int e;
    (void)frexpf(m, &e);
    e = e < -40 ? -40 : (e > 40 ? 40 : e);
    return ldexpf(1.f, -e);
}

// ---- multiplier storage -------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// Round-to-nearest-even of a finite float to BF16.
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ d4 ld_d4(const double *p) { return *reinterpret_cast<const d4 *>(p); }
__device__ __forceinline__ f4 ld_f4(const float *p) { return *reinterpret_cast<const f4 *>(p); }
__device__ __forceinline__ uint2 ld_u2(const uint16_t *p) { return *reinterpret_cast<const uint2 *>(p); }

// Raw registers of one lane's pairs of a tile (CPL consecutive columns), per representation.
// REP_F64 lanes hold 4 columns (32 bytes per matrix); the split forms hold 8 columns so that every
// row segment a lane group reads is a whole 128-byte line in each array.
template <int REP> struct Raw;
template <> struct Raw<REP_F64> {
    static constexpr int CPL = 4;
    d4 p, q;
};
template <> struct Raw<REP_SPLIT_F32> {
    static constexpr int CPL = 8;
    f4 h[2], a[2], b[2];
};
template <> struct Raw<REP_SPLIT_BF16> {
    static constexpr int CPL = 8;
    uint4 h;
    f4 a[2], b[2];
};

__device__ __forceinline__ uint32_t u4_at(const uint4 &v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
__device__ __forceinline__ void u4_set(uint4 &v, int k, uint32_t x) {
    if (k == 0) v.x = x; else if (k == 1) v.y = x; else if (k == 2) v.z = x; else v.w = x;
}

template <int REP> __device__ __forceinline__ float hi_at(const Raw<REP> &t, int c);
template <> __device__ __forceinline__ float hi_at<REP_SPLIT_F32>(const Raw<REP_SPLIT_F32> &t, int c) {
    return t.h[c >> 2][c & 3];
}
template <> __device__ __forceinline__ float hi_at<REP_SPLIT_BF16>(const Raw<REP_SPLIT_BF16> &t, int c) {
    const uint32_t w = u4_at(t.h, c >> 1);
    return bf16_to_float((uint16_t)((c & 1) ? (w >> 16) : (w & 0xFFFFu)));
}
template <int REP> __device__ __forceinline__ void hi_set(Raw<REP> &t, int c, float v);
template <> __device__ __forceinline__ void hi_set<REP_SPLIT_F32>(Raw<REP_SPLIT_F32> &t, int c, float v) {
    t.h[c >> 2][c & 3] = v;
}
template <> __device__ __forceinline__ void hi_set<REP_SPLIT_BF16>(Raw<REP_SPLIT_BF16> &t, int c, float v) {
    const uint32_t hv = float_to_bf16(v);
    uint32_t w = u4_at(t.h, c >> 1);
    w = (c & 1) ? ((w & 0xFFFFu) | (hv << 16)) : ((w & 0xFFFF0000u) | hv);
    u4_set(t.h, c >> 1, w);
}

template <typename T> __device__ __forceinline__ T shfl_xor(T v, int m) { return __shfl_xor(v, m, 64); }

// v as seen from another lane of the same 16-lane row, selected by the DPP control CTRL (a row
// shift reads 0 where the source lane lies outside the row).
template <int CTRL> __device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over each row of 16 lanes with DPP row shifts (pure VALU, no LDS): after shifts by 1, 2, 4
// and 8, lane 15 of every row holds the row total.
template <typename T> __device__ __forceinline__ T row16_sum(T v) {
    v += dpp_move<0x111>(v);   // row_shr:1
    v += dpp_move<0x112>(v);   // row_shr:2
    v += dpp_move<0x114>(v);   // row_shr:4
    v += dpp_move<0x118>(v);   // row_shr:8
    return v;
}

// ---- the pair sweep -----------------------------------------------------------------------
// KT: residual K-steps dropped at the end (4 MB - KT steps of 4 features); the launcher passes
// KT > 0 only when every dropped step lies beyond feature n - 1, where Xi is zero.
// `bid` is the workgroup's index within the fit's own grid (blockIdx.x for a single fit; the
// grouped launch below maps its workgroups onto several fits).
template <typename T, int REP, int MODE, int MB, int KT>
__device__ __forceinline__ void pass_body(const PassArgs &a, const Geometry &g, const int bid) {
    constexpr int NP = 16 * MB;
    constexpr int KS = 4 * MB - KT;                  // residual K-steps
    static_assert(KT >= 0 && KS >= 1, "at least one residual step");
    constexpr int SX = NP + 1;                       // LDS row stride (elements): odd, no bank aliasing
    constexpr int BUF = kSuper * SX;
    constexpr int NT = 64 * kWaves;                  // threads per workgroup
    constexpr int XR = kSuper * NP / NT;             // staged X elements per thread
    static_assert(XR * NT == kSuper * NP, "the X tile must split evenly over the threads");
    constexpr int CPL = Raw<REP>::CPL;               // consecutive columns per lane
    constexpr int NB = CPL / 4;                      // 16x16 MFMA blocks per tile
    constexpr int TW = 4 * CPL;                      // tile width (columns)
    constexpr int TPS = kSuper / TW;                 // tiles per super tile
    constexpr bool kSplit = (REP != REP_F64);
    constexpr bool kAdv = (MODE == PASS_ADV);
    constexpr bool kStoreCand = (MODE == PASS_TRIAL);
    static_assert(!(kStoreCand && REP != REP_F64), "only the FP64 trial pass stores its candidates");
    constexpr bool kTrial = (MODE == PASS_TRIAL || MODE == PASS_TRIAL_NS || kAdv);
    constexpr bool kAdjoint = (MODE == PASS_STEP || MODE == PASS_ADJ || MODE == PASS_POWER || MODE == PASS_REBASE ||
                               kTrial);
    // Split-form trial passes take the two adjoints of the candidate differences D on BF16 MFMA with
    // split operands (D and Xhat each as hi + lo BF16; three products per pair of operands): D only
    // enters the step test and the update eta(lam~) + C^T D, where ~1e-5 relative error is harmless,
    // and the FP32 form's cost would make these passes compute-bound.  The residual stays FP32.
    constexpr bool kBfAdj = kTrial && kSplit;
    constexpr int XTS = kSuper + 8;                  // BF16 transposed tile: row stride (elements)
    constexpr bool kResidual = (MODE != PASS_ADJ && MODE != PASS_REBASE);
    // Split-form passes with a residual (the trial passes and the constant step's pass) form it on
    // FP16 matrix cores: both operands scaled by powers of
    // two into [0.5, 1) (each row of Xi by its largest entry, the locations by the fit's largest
    // |Xhat|, PassArgs::x_scale) and split into hi + lo halves (split_f16), three products per pair
    // of operands in K chunks of 16 -- the FP32 16x16x4 form's accuracy at under half of its matrix
    // cycles.  The scales are exact: the accumulator starts at (y_j + d_i - y_i) c_i (c_i = row
    // scale x location scale) and the step sizes are divided by c_i, so the epilogue's products
    // s c_i * (1 / (s_a c_i)) equal the unscaled ones bit for bit.
    constexpr bool kHalfRes = kSplit && kResidual && sizeof(T) == 4 && (kTrial || MODE == PASS_STEP);
    constexpr bool kX32 = !kHalfRes || !kBfAdj;      // the FP32 location tile (FP32 adjoint MFMAs)
    constexpr int HC16 = (4 * KS + 15) / 16;         // K = 16 chunks covering the residual's features
    constexpr int XH = NP + 4;                       // FP16 tile row stride (halves; 8-byte rows)
    constexpr bool kColRed = kAdjoint || MODE == PASS_REPAIR;
    constexpr bool kReadA = (MODE == PASS_STEP || MODE == PASS_ADJ || MODE == PASS_KKT || MODE == PASS_REBASE ||
                             kTrial);
    constexpr bool kReadB = (MODE == PASS_STEP || MODE == PASS_REBASE || kTrial);
    constexpr bool kReadH = kSplit && kReadA;
    constexpr bool kLoads = kReadA || kReadB;
    typedef typename Vec4<T>::type V4;

    __shared__ T sX[kX32 ? 2 * BUF : 1];
    // FP16 hi / lo splits of the scaled location tile (column-major: a column's features adjacent)
    __shared__ __attribute__((aligned(16))) _Float16 sXH[kHalfRes ? 2 * kSuper * XH : 8];
    __shared__ __attribute__((aligned(16))) _Float16 sXL[kHalfRes ? 2 * kSuper * XH : 8];
    __shared__ T sY[2 * kSuper];
    __shared__ T sYo[kAdv ? 2 * kSuper : 1];
    // transposed BF16 hi / lo copies of the staged Xhat tile (feature-major), for the BF16 adjoint
    __shared__ __attribute__((aligned(16))) __bf16 sXTh[kBfAdj ? 2 * NP * XTS : 8];
    __shared__ __attribute__((aligned(16))) __bf16 sXTl[kBfAdj ? 2 * NP * XTS : 8];
    __shared__ T sCol[kColRed ? 2 * kWaves * kSuper : 1];
    __shared__ T sCol2[kTrial ? 2 * kWaves * kSuper : 1];
    __shared__ int sArg[MODE == PASS_REPAIR ? 2 * kWaves * kSuper : 1];
    __shared__ double sRed[kWaves * kRed];

    const T *xhat = static_cast<const T *>(a.xhat);
    const T *xi = static_cast<const T *>(a.xi);
    const T *yv = static_cast<const T *>(a.yv);
    const T *dmy = static_cast<const T *>(a.dmy);

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, lr = l & 15, lq = l >> 4;
    const int chunk = bid % g.chunks;               // consecutive workgroups: one chunk per XCD
    const int strip = bid / g.chunks;
    const int i = strip * kRows + w * 16 + lr;      // < Nr always
    const bool row_ok = i < g.N;
    const int blk = a.blk > 1 ? a.blk : 1;          // pairs of one block are not dualized
    const int iblk = i / blk;
    const int cbeg = chunk * g.chunk_cols;
    const int cend = min(g.ld, cbeg + g.chunk_cols);
    const int nsup = (cend - cbeg) / kSuper;
    // first column of the s-th super tile in walking order (a.rev: from the end of the chunk back)
    const bool rev = a.rev != 0;
    auto sup_col = [&](int s) { return cbeg + (rev ? nsup - 1 - s : s) * kSuper; };
    const T bp = (T)a.beta_prev, bn = (T)a.beta_next, invL = (T)a.inv_L, invL2 = (T)a.inv_L2;
    // Split trial passes: rows 8..15 of each wave evaluate the candidates in the order (b, a), so
    // that the first exchange of the column-sum reduce-scatter needs no selects (every lane keeps
    // `out` and sends `out2`); their trial sums and adjoint accumulators are swapped back at the end.
    const bool cswap = kBfAdj && ((lr >> 3) & 1);
    T invA = cswap ? invL2 : invL, invB = cswap ? invL : invL2;
    T invLo = (T)a.inv_Lo;
    const bool rebase_lam = (MODE == PASS_REBASE) && a.rebase_lam != 0;
    // Output rows of the 16x16x4 MFMA: lane group g, item v receives row 4 g + v in the FP32 form
    // and row 4 v + g in the FP64 form.  A-row rho is therefore fed the source that lane group
    // g(rho), item v(rho) must see: feature 16 mb + 4 g + v in the adjoint contraction, column
    // CPL g + 4 bb + v of block bb in the residual contraction.
    const int rg = (sizeof(T) == 8) ? (lr & 3) : (lr >> 2);
    const int rv = (sizeof(T) == 8) ? (lr >> 2) : (lr & 3);
    const int arow = 4 * rg + rv;                    // feature row fed by this lane
    const int acol = CPL * rg + rv;                  // tile column fed by this lane (block 0)

    // Row-constant operands: B of the residual contraction is -Xi[i][4s + lq]; the accumulator
    // starts at y_j + d_i - y_i, so the product leaves s_ij itself (no separate subtraction).
    T bxi[kHalfRes ? 1 : 4 * MB];
#pragma unroll
    for (int s = 0; s < (kHalfRes ? 1 : 4 * MB); ++s)
        bxi[s] = (kResidual && !kHalfRes) ? -xi[(size_t)i * NP + 4 * s + lq] : (T)0;
    const T dmy_i = kResidual ? dmy[i] : (T)0;
    const T roff_i = (MODE == PASS_REPAIR && a.row_off) ? (T)a.row_off[i] : (T)0;
    // PASS_ADV: the previous trial's row operands (re-forming its accepted candidate)
    const T *xio = static_cast<const T *>(a.xi_o);
    const T *yvo = static_cast<const T *>(a.yv_o);
    T bxio[kAdv && !kHalfRes ? 4 * MB : 1];
#pragma unroll
    for (int s = 0; s < (kAdv && !kHalfRes ? 4 * MB : 1); ++s)
        bxio[s] = (kAdv && !kHalfRes) ? -xio[(size_t)i * NP + 4 * s + lq] : (T)0;
    const T dmyo_i = kAdv ? static_cast<const T *>(a.dmy_o)[i] : (T)0;
    // FP16 row operands: B[k][row lr] = -Xi[i][k] c, lane (lr, lq) holding features 16 c + 4 lq + q
    // of chunk c; rsc / rsco = c_i of the new and of the previous trial's point
    constexpr int H16 = kHalfRes ? HC16 : 1, O16 = kAdv ? H16 : 1;
    h4 rh16[H16], rl16[H16], oh16[O16], ol16[O16];
    T rsc = (T)1, rsco = (T)1;
    if constexpr (kHalfRes) {
        auto load_row = [&](const T *src, h4 *h16, h4 *l16) -> T {
            float v16[H16][4];
            float mx = 0.f;
#pragma unroll
            for (int c = 0; c < HC16; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    v16[c][q] = (float)src[(size_t)i * NP + 16 * c + 4 * lq + q];
                    mx = fmaxf(mx, fabsf(v16[c][q]));
                }
            mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
            mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
            const float al = pow2_scale(mx);
#pragma unroll
            for (int c = 0; c < HC16; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    _Float16 hh, ll;
                    split_f16(-v16[c][q] * al, hh, ll);
                    h16[c][q] = hh;
                    l16[c][q] = ll;
                }
            return (T)(al * a.x_scale);
        };
        rsc = load_row(xi, rh16, rl16);
        if constexpr (kAdv) rsco = load_row(xio, oh16, ol16);
        invA *= (T)1 / rsc;
        invB *= (T)1 / rsc;
        invLo *= (T)1 / rsco;
    }
    const T dmyc_i = dmy_i * rsc, dmyoc_i = dmyo_i * rsco;

    V4 acc[MB];
    V4 acc2[kTrial ? MB : 1];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = V4{0, 0, 0, 0};
#pragma unroll
    for (int mb = 0; mb < (kTrial ? MB : 1); ++mb) acc2[mb] = V4{0, 0, 0, 0};
    double red0 = 0.0, red1 = 0.0, red2 = 0.0, red3 = 0.0;

    const size_t rowoff = (size_t)i * g.ld;
    const double *pa64 = static_cast<const double *>(a.lam_a);
    double *pb64 = static_cast<double *>(a.lam_b);
    float *pa32 = static_cast<float *>(const_cast<void *>(a.lam_a));
    float *pb32 = static_cast<float *>(a.lam_b);
    float *phf = static_cast<float *>(a.lam_h);
    uint16_t *phb = static_cast<uint16_t *>(a.lam_h);
    double *pc64 = static_cast<double *>(a.lam_c);
    double *pd64 = static_cast<double *>(a.lam_d);

    auto load_tile = [&](int j0, Raw<REP> &t) {
        const size_t e = rowoff + j0;
        if constexpr (REP == REP_F64) {
            if (kReadA) t.p = ld_d4(pa64 + e);
            if (kReadB) t.q = ld_d4(pb64 + e);
        } else {
            if constexpr (REP == REP_SPLIT_F32) {
                if (kReadH) { t.h[0] = ld_f4(phf + e); t.h[1] = ld_f4(phf + e + 4); }
            } else {
                if (kReadH) t.h = *reinterpret_cast<const uint4 *>(phb + e);
            }
            if (kReadA) { t.a[0] = ld_f4(pa32 + e); t.a[1] = ld_f4(pa32 + e + 4); }
            if (kReadB) { t.b[0] = ld_f4(pb32 + e); t.b[1] = ld_f4(pb32 + e + 4); }
        }
    };

    // stage super tile 0 and prefetch the first two tiles' multipliers
    const int c0 = sup_col(0);
    if (nsup > 0) {
        for (int e = tid; e < kSuper * NP; e += NT) {
            const int jj = e / NP, m = e - jj * NP;
            const T v = xhat[(size_t)(c0 + jj) * NP + m];
            if constexpr (kHalfRes) split_f16((float)v * a.x_scale, sXH[jj * XH + m], sXL[jj * XH + m]);
            if constexpr (kX32) sX[jj * SX + m] = v;
            if constexpr (kBfAdj) split_bf16((float)v, sXTh[m * XTS + jj], sXTl[m * XTS + jj]);
        }
        if (tid < kSuper) sY[tid] = kResidual ? yv[c0 + tid] : (T)0;
        if (kAdv && tid < kSuper) sYo[tid] = yvo[c0 + tid];
    }
    static_assert(TPS % 2 == 0, "the two-deep prefetch ring needs an even number of tiles per super tile");
    Raw<REP> pf[2];
    if (kLoads && nsup > 0) {
        load_tile(c0 + CPL * lq, pf[0]);
        load_tile(c0 + TW + CPL * lq, pf[1]);
    }
    __syncthreads();

    for (int st = 0; st < nsup; ++st) {
        const int cst = sup_col(st);
        const int b = st & 1;
        const T *sXb = kX32 ? sX + b * BUF : sX;
        const T *sYb = sY + b * kSuper;
        const bool more = st + 1 < nsup;

        // register prefetch of the next super tile's locations (the last super tile re-reads its
        // own rows instead, so the loads need no branch)
        const int cnx = more ? sup_col(st + 1) : cst;
        T xr[XR];
#pragma unroll
        for (int q = 0; q < XR; ++q) xr[q] = xhat[(size_t)cnx * NP + tid + q * NT];
        const T yr = kResidual ? yv[cnx + (tid & (kSuper - 1))] : (T)0;
        const T yro = kAdv ? yvo[cnx + (tid & (kSuper - 1))] : (T)0;
        __builtin_amdgcn_sched_barrier(0);

#pragma unroll
        for (int t = 0; t < TPS; ++t) {
            const int jl = t * TW;                   // local first column of the tile
            const int jc = jl + CPL * lq;            // local column of c = 0 for this lane
            const int j0 = cst + jc;                 // global column of c = 0
            Raw<REP> cur = pf[t & 1];
            if (kLoads) {
                // two tiles ahead in walking order (possibly in the next super tile); past the last
                // tile the current one is re-read instead, so the load needs no branch
                const int sn = st + (t + 2) / TPS;
                const int jn = sn < nsup ? sup_col(sn) + ((t + 2) % TPS) * TW + CPL * lq : j0;
                load_tile(jn, pf[t & 1]);
            }
            // keep the prefetch ahead of this tile's work (the scheduler would otherwise sink the
            // loads below the epilogue, which then waits for them)
            __builtin_amdgcn_sched_barrier(0);

            const T *sYob = sYo + (kAdv ? b * kSuper : 0);
            V4 S[NB];
            V4 So[kAdv ? NB : 1];
#pragma unroll
            for (int bb = 0; bb < NB; ++bb) {
                // output item v of block bb is column jc + 4 bb + v of row i
                const int jb = jc + 4 * bb;
                if constexpr (kHalfRes) {
                    // scaled start (y_j + d_i - y_i) c_i, one rounding as unscaled (c_i a power of 2)
                    S[bb] = V4{fma(sYb[jb], rsc, dmyc_i), fma(sYb[jb + 1], rsc, dmyc_i), fma(sYb[jb + 2], rsc, dmyc_i),
                               fma(sYb[jb + 3], rsc, dmyc_i)};
                    if constexpr (kAdv)
                        So[bb] = V4{fma(sYob[jb], rsco, dmyoc_i), fma(sYob[jb + 1], rsco, dmyoc_i),
                                    fma(sYob[jb + 2], rsco, dmyoc_i), fma(sYob[jb + 3], rsco, dmyoc_i)};
                    const _Float16 *ph = sXH + b * kSuper * XH + (jl + acol + 4 * bb) * XH;
                    const _Float16 *pl = sXL + b * kSuper * XH + (jl + acol + 4 * bb) * XH;
#pragma unroll
                    for (int c = 0; c < HC16; ++c) {
                        const int f0 = 16 * c + 4 * lq;
                        const h4 ah = *reinterpret_cast<const h4 *>(ph + f0);
                        const h4 al = *reinterpret_cast<const h4 *>(pl + f0);
                        S[bb] = mfma16_h16(ah, rl16[c], S[bb]);
                        S[bb] = mfma16_h16(al, rh16[c], S[bb]);
                        S[bb] = mfma16_h16(ah, rh16[c], S[bb]);
                        if constexpr (kAdv) {
                            So[bb] = mfma16_h16(ah, ol16[c], So[bb]);
                            So[bb] = mfma16_h16(al, oh16[c], So[bb]);
                            So[bb] = mfma16_h16(ah, oh16[c], So[bb]);
                        }
                    }
                    continue;
                }
                S[bb] = kResidual ? V4{sYb[jb] + dmy_i, sYb[jb + 1] + dmy_i, sYb[jb + 2] + dmy_i, sYb[jb + 3] + dmy_i}
                                  : V4{0, 0, 0, 0};
                if (kAdv)
                    So[bb] = V4{sYob[jb] + dmyo_i, sYob[jb + 1] + dmyo_i, sYob[jb + 2] + dmyo_i, sYob[jb + 3] + dmyo_i};
                if (kResidual) {
                    // a fixed KS steps: Xi is zero beyond column n - 1, so padded steps add zero
                    // and the loop carries no branch (which would make the compiler drain the
                    // prefetch queue at every join)
#pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const T xa = sXb[(jl + acol + 4 * bb) * SX + 4 * s + lq];
                        S[bb] = mfma16(xa, bxi[s], S[bb]);
                        if constexpr (kAdv) So[bb] = mfma16(xa, bxio[s], So[bb]);
                    }
                }
            }

            T out[CPL];
            T out2[kTrial ? CPL : 1];
            T cand_a[kTrial ? CPL : 1], cand_b[kTrial ? CPL : 1];
            // Pair validity (i != j, both real points, and under a K-block partition i and j in
            // different blocks) only varies inside tiles that touch the diagonal (the diagonal
            // blocks) or the padding; every other tile takes the unmasked path.  The branch is
            // uniform over the wave and holds no memory operation.
            const int i0w = strip * kRows + w * 16;
            const int jt0 = cst + jl;
            const bool interior = (i0w + 16 <= g.N) && (jt0 + TW <= g.N) &&
                                  ((i0w + 15) / blk < jt0 / blk || (jt0 + TW - 1) / blk < i0w / blk);
            // split forms: trial sums of this tile in FP32, folded into the FP64 totals once per tile
            T tr0 = (T)0, tr1 = (T)0, tr2 = (T)0, tr3 = (T)0;
            auto epilogue = [&](auto masked) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = j0 + c;
                const bool ok = masked ? (row_ok && (j < g.N) && (j != i) && (j / blk != iblk)) : true;
                const T s = S[c >> 2][c & 3];                          // s_ij
                if constexpr (MODE == PASS_STEP && REP == REP_F64) {
                    const T P = (T)cur.p[c], Q = (T)cur.q[c];
                    const T lt = P + bp * (P - Q);                       // lam~^k
                    T ln = lt - s * invL;                                // Step 2
                    ln = fmax(ln, (T)0);
                    ln = ok ? ln : (T)0;
                    cur.q[c] = (double)ln;                               // lam^k (stored below)
                    const T nx = ln + bn * (ln - P);                     // Step 4
                    out[c] = ok ? nx : (T)0;
                } else if constexpr (MODE == PASS_STEP) {
                    // lam = H + l: only the low parts move between re-basings
                    const T H = (T)hi_at<REP>(cur, c);
                    const T l1 = (T)cur.a[c >> 2][c & 3], l2 = (T)cur.b[c >> 2][c & 3];
                    const T lt = l1 + bp * (l1 - l2);                    // low part of lam~^k
                    T l0 = lt - s * invA;                                // Step 2 ...
                    l0 = fmax(l0, -H);                                   // ... projected: H + l0 >= 0
                    l0 = ok ? l0 : (T)0;
                    cur.b[c >> 2][c & 3] = (float)l0;
                    const T nx = l0 + bn * (l0 - l1);                    // low part of lam~^{k+1}
                    out[c] = ok ? nx : (T)0;
                } else if constexpr (kAdv && REP == REP_F64) {
                    const T P = (T)cur.p[c], Q = (T)cur.q[c];
                    // re-form the accepted candidate of the previous trial: lam^k
                    const T lto = P + bp * (P - Q);
                    const T so = So[c >> 2][c & 3];
                    T z = fmax(lto - so * invLo, (T)0);
                    z = ok ? z : (T)0;
                    cur.q[c] = (double)z;                                // stored over lam^{k-2}
                    // trial from (lam^k, lam^{k-1})
                    const T lt = z + bn * (z - P);                       // lam~^{k+1}
                    T ta = fmax(lt - s * invL, (T)0);
                    T tb = fmax(lt - s * invL2, (T)0);
                    ta = ok ? ta : (T)0;
                    tb = ok ? tb : (T)0;
                    out[c] = ok ? ta - lt : (T)0;                        // D_a
                    out2[c] = ok ? tb - lt : (T)0;                       // D_b
                    red0 += out[c] * out[c];
                    red1 += out2[c] * out2[c];
                    red2 += out[c] * (ta - z);                           // <D_a, cand_a - lam^k>
                    red3 += out2[c] * (tb - z);
                } else if constexpr ((MODE == PASS_TRIAL || MODE == PASS_TRIAL_NS) && REP == REP_F64) {
                    const T P = (T)cur.p[c], Q = (T)cur.q[c];
                    const T lt = P + bp * (P - Q);                       // lam~^k
                    T ta = fmax(lt - s * invL, (T)0);                    // candidate with 1 / s_a
                    T tb = fmax(lt - s * invL2, (T)0);                   // candidate with 1 / s_b
                    ta = ok ? ta : (T)0;
                    tb = ok ? tb : (T)0;
                    cand_a[c] = ta;
                    cand_b[c] = tb;
                    out[c] = ok ? ta - lt : (T)0;                        // D_a
                    out2[c] = ok ? tb - lt : (T)0;                       // D_b
                    red0 += out[c] * out[c];
                    red1 += out2[c] * out2[c];
                    red2 += out[c] * (ta - P);                           // <D_a, cand_a - lam^k>
                    red3 += out2[c] * (tb - P);
                } else if constexpr (kAdv) {
                    const T H = (T)hi_at<REP>(cur, c);
                    const T l1 = (T)cur.a[c >> 2][c & 3], l2 = (T)cur.b[c >> 2][c & 3];
                    // re-form the accepted candidate of the previous trial: lam^k (low part)
                    const T lto = l1 + bp * (l1 - l2);
                    const T so = So[c >> 2][c & 3];
                    T z = fmax(lto - so * invLo, -H);
                    z = ok ? z : (T)0;
                    cur.b[c >> 2][c & 3] = (float)z;                     // stored over lam^{k-2}
                    // trial from (lam^k, lam^{k-1})
                    const T m = z - l1;
                    const T lt = z + bn * m;
                    T la = fmax(lt - s * invA, -H);                    // (b for swapped rows)
                    T lb = fmax(lt - s * invB, -H);
                    la = ok ? la : (T)0;
                    lb = ok ? lb : (T)0;
                    out[c] = ok ? la - lt : (T)0;
                    out2[c] = ok ? lb - lt : (T)0;
                    tr0 += out[c] * out[c];
                    tr1 += out2[c] * out2[c];
                    // cand - lam^k = D + beta m: <D, cand - lam^k> = ||D||^2 + beta <D, m>
                    tr2 += out[c] * m;
                    tr3 += out2[c] * m;
                } else if constexpr (MODE == PASS_TRIAL || MODE == PASS_TRIAL_NS) {
                    const T H = (T)hi_at<REP>(cur, c);
                    const T l1 = (T)cur.a[c >> 2][c & 3], l2 = (T)cur.b[c >> 2][c & 3];
                    const T m = l1 - l2;
                    const T lt = l1 + bp * m;                            // low part of lam~^k
                    T la = fmax(lt - s * invA, -H);                    // (b for swapped rows)
                    T lb = fmax(lt - s * invB, -H);
                    la = ok ? la : (T)0;
                    lb = ok ? lb : (T)0;
                    out[c] = ok ? la - lt : (T)0;
                    out2[c] = ok ? lb - lt : (T)0;
                    tr0 += out[c] * out[c];
                    tr1 += out2[c] * out2[c];
                    // cand - lam^k = D + beta m: <D, cand - lam^k> = ||D||^2 + beta <D, m>
                    tr2 += out[c] * m;
                    tr3 += out2[c] * m;
                } else if constexpr (MODE == PASS_ADJ) {
                    T v;
                    if constexpr (REP == REP_F64) v = (T)cur.p[c];
                    else v = (T)((double)hi_at<REP>(cur, c) + (double)cur.a[c >> 2][c & 3]);
                    out[c] = ok ? v : (T)0;
                } else if constexpr (MODE == PASS_REBASE) {
                    const double H = (double)hi_at<REP>(cur, c);
                    const double lam0 = H + (double)cur.a[c >> 2][c & 3];   // lam^k
                    const double lam1 = H + (double)cur.b[c >> 2][c & 3];   // lam^{k-1}
                    float hn = (float)lam0;
                    if (REP == REP_SPLIT_BF16) hn = bf16_to_float(float_to_bf16(hn));
                    const double Hn = ok ? (double)hn : 0.0;
                    cur.a[c >> 2][c & 3] = ok ? (float)(lam0 - Hn) : 0.f;
                    cur.b[c >> 2][c & 3] = ok ? (float)(lam1 - Hn) : 0.f;
                    hi_set<REP>(cur, c, (float)Hn);
                    // the adjoint of H' (cached for the constant step) or of lam^k as now stored
                    out[c] = rebase_lam ? (T)(Hn + (double)cur.a[c >> 2][c & 3]) : (T)Hn;
                } else if constexpr (MODE == PASS_POWER) {
                    const T z = ok ? s : (T)0;
                    out[c] = z;
                    red0 += (double)z * (double)z;
                } else if constexpr (MODE == PASS_KKT) {
                    double dl;
                    if constexpr (REP == REP_F64) dl = cur.p[c];
                    else dl = (double)hi_at<REP>(cur, c) + (double)cur.a[c >> 2][c & 3];
                    if (ok) {
                        const double ds = (double)s;
                        const double mn = fabs(dl < ds ? dl : ds);
                        red0 = red0 > mn ? red0 : mn;
                        red1 = red1 > -ds ? red1 : -ds;
                        const double ng = ds < 0.0 ? ds : 0.0;
                        red2 += ng * ng;
                        red3 += dl * ds;
                    }
                    out[c] = (T)0;
                } else if constexpr (MODE == PASS_REPAIR) {
                    out[c] = ok ? s - roff_i : (T)INFINITY;
                } else {  // PASS_RESID (REP_F64)
                    cur.q[c] = ok ? (double)s : 0.0;
                    out[c] = (T)0;
                }
            }
            };
            if (interior) epilogue(std::false_type{});
            else epilogue(std::true_type{});
            if constexpr (kTrial && kSplit) {
                // tr2, tr3 hold <D, m>; beta is that of the extrapolation the candidates start from
                const double bm = kAdv ? a.beta_next : a.beta_prev;
                red0 += (double)tr0;
                red1 += (double)tr1;
                red2 += (double)tr0 + bm * (double)tr2;
                red3 += (double)tr1 + bm * (double)tr3;
            }
            {
                const size_t e = rowoff + j0;
                if constexpr (kStoreCand) {
                    *reinterpret_cast<d4 *>(pc64 + e) = d4{(double)cand_a[0], (double)cand_a[1],
                                                           (double)cand_a[2], (double)cand_a[3]};
                    *reinterpret_cast<d4 *>(pd64 + e) = d4{(double)cand_b[0], (double)cand_b[1],
                                                           (double)cand_b[2], (double)cand_b[3]};
                } else if constexpr (REP == REP_F64) {
                    if (MODE == PASS_STEP || MODE == PASS_RESID || kAdv) *reinterpret_cast<d4 *>(pb64 + e) = cur.q;
                } else {
                    if (MODE == PASS_STEP || MODE == PASS_REBASE || kAdv) {
                        *reinterpret_cast<f4 *>(pb32 + e) = cur.b[0];
                        *reinterpret_cast<f4 *>(pb32 + e + 4) = cur.b[1];
                    }
                    if (MODE == PASS_REBASE) {
                        *reinterpret_cast<f4 *>(pa32 + e) = cur.a[0];
                        *reinterpret_cast<f4 *>(pa32 + e + 4) = cur.a[1];
                        if constexpr (REP == REP_SPLIT_F32) {
                            *reinterpret_cast<f4 *>(phf + e) = cur.h[0];
                            *reinterpret_cast<f4 *>(phf + e + 4) = cur.h[1];
                        } else {
                            *reinterpret_cast<uint4 *>(phb + e) = cur.h;
                        }
                    }
                }
            }

            if constexpr (kBfAdj) {
                static_assert(CPL == 8, "the BF16 adjoint takes a lane's 8 consecutive columns as its K slice");
                // A[m][k] = Xhat[column jl + 8 lq + k][feature 16 mb + lr]; B[k][n] = D[row lr][column
                // jl + 8 lq + k]
                uint4 dhu, dlu, ehu, elu;
#pragma unroll
                for (int c2 = 0; c2 < 4; ++c2) {
                    uint32_t hp, lp;
                    split_bf16_pair((float)out[2 * c2], (float)out[2 * c2 + 1], hp, lp);
                    u4_set(dhu, c2, hp);
                    u4_set(dlu, c2, lp);
                    split_bf16_pair((float)out2[2 * c2], (float)out2[2 * c2 + 1], hp, lp);
                    u4_set(ehu, c2, hp);
                    u4_set(elu, c2, lp);
                }
                const bf8 dh = __builtin_bit_cast(bf8, dhu), dl = __builtin_bit_cast(bf8, dlu);
                const bf8 eh = __builtin_bit_cast(bf8, ehu), el = __builtin_bit_cast(bf8, elu);
                const __bf16 *xth = sXTh + b * NP * XTS + jl + 8 * lq;
                const __bf16 *xtl = sXTl + b * NP * XTS + jl + 8 * lq;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const bf8 ah = *reinterpret_cast<const bf8 *>(xth + (16 * mb + lr) * XTS);
                    const bf8 al = *reinterpret_cast<const bf8 *>(xtl + (16 * mb + lr) * XTS);
                    f4 x = *reinterpret_cast<f4 *>(&acc[mb]);
                    x = mfma16_bf16(ah, dh, x);
                    x = mfma16_bf16(ah, dl, x);
                    x = mfma16_bf16(al, dh, x);
                    acc[mb] = *reinterpret_cast<V4 *>(&x);
                    f4 z = *reinterpret_cast<f4 *>(&acc2[mb]);
                    z = mfma16_bf16(ah, eh, z);
                    z = mfma16_bf16(ah, el, z);
                    z = mfma16_bf16(al, eh, z);
                    acc2[mb] = *reinterpret_cast<V4 *>(&z);
                }
            }
            if constexpr (kBfAdj) {
                // Column sums of both differences over the wave's 16 rows as a reduce-scatter: the
                // 16 sums (8 columns x 2 candidates) halve at each exchange (lane partners l ^ 8,
                // l ^ 7, l ^ 2, l ^ 1, a basis of the 16 lanes), and lane lr of each lane group ends
                // with candidate lr / 8, column lr % 8.
                const bool h3 = (lr >> 3) & 1, h2 = (lr >> 2) & 1, h1 = (lr >> 1) & 1, h0 = lr & 1;
                T v8[8], v4[4], v2[2];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    v8[q] = out[q] + dpp_move<0x128>(out2[q]);    // row_ror:8 (rows 8..15 hold b in `out`)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v4[q] = (h2 ? v8[4 + q] : v8[q]) + dpp_move<0x141>(h2 ? v8[q] : v8[4 + q]);  // row_half_mirror
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    v2[q] = (h1 ? v4[2 + q] : v4[q]) + dpp_move<0x4E>(h1 ? v4[q] : v4[2 + q]);   // lane ^ 2
                const T v1 = (h0 ? v2[1] : v2[0]) + dpp_move<0xB1>(h0 ? v2[0] : v2[1]);         // lane ^ 1
                (h3 ? sCol2 : sCol)[(b * kWaves + w) * kSuper + jc + (lr & 7)] = v1;
            } else if (kAdjoint) {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int c = 0; c < CPL; ++c)
                        acc[mb] = mfma16(sXb[(jc + c) * SX + 16 * mb + arow], out[c], acc[mb]);
                T cs[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) cs[c] = row16_sum(out[c]);
                if (lr == 15) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) sCol[(b * kWaves + w) * kSuper + jc + c] = cs[c];
                }
                if constexpr (kTrial) {
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            acc2[mb] = mfma16(sXb[(jc + c) * SX + 16 * mb + arow], out2[c], acc2[mb]);
#pragma unroll
                    for (int c = 0; c < CPL; ++c) cs[c] = row16_sum(out2[c]);
                    if (lr == 15) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c) sCol2[(b * kWaves + w) * kSuper + jc + c] = cs[c];
                    }
                }
            } else if (MODE == PASS_REPAIR) {
                // column minimum over the 16 rows of this wave, lowest row on ties
                T v[CPL];
                int arg[CPL];
#pragma unroll
                for (int c = 0; c < CPL; ++c) { v[c] = out[c]; arg[c] = i; }
#pragma unroll
                for (int m = 1; m < 16; m <<= 1)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const T ov = shfl_xor(v[c], m);
                        const int oa = __shfl_xor(arg[c], m, 64);
                        if (ov < v[c] || (ov == v[c] && oa < arg[c])) { v[c] = ov; arg[c] = oa; }
                    }
                if (lr == 0) {
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        sCol[(b * kWaves + w) * kSuper + jc + c] = v[c];
                        sArg[(b * kWaves + w) * kSuper + jc + c] = arg[c];
                    }
                }
            }
        }

        // the next super tile's locations go to the other buffer
        if (more) {
            T *sXn = kX32 ? sX + (b ^ 1) * BUF : sX;
#pragma unroll
            for (int q = 0; q < XR; ++q) {
                const int e = tid + q * NT;
                const int jj = e / NP, m = e - jj * NP;
                if constexpr (kHalfRes) {
                    const int o = (b ^ 1) * kSuper * XH + jj * XH + m;
                    split_f16((float)xr[q] * a.x_scale, sXH[o], sXL[o]);
                }
                if constexpr (kX32) sXn[jj * SX + m] = xr[q];
                if constexpr (kBfAdj) {
                    const int o = (b ^ 1) * NP * XTS + m * XTS + jj;
                    split_bf16((float)xr[q], sXTh[o], sXTl[o]);
                }
            }
            if (tid < kSuper) sY[(b ^ 1) * kSuper + tid] = yr;
            if (kAdv && tid < kSuper) sYo[(b ^ 1) * kSuper + tid] = yro;
        }
        __syncthreads();
        // column partials of this super tile (buffer b is not written again before the next barrier)
        if (kColRed && tid < kSuper) {
            const int j = cst + tid;
            const int base = b * kWaves * kSuper;
            if (MODE == PASS_REPAIR) {
                double best = (double)sCol[base + tid];
                int arg = sArg[base + tid];
                for (int ww = 1; ww < kWaves; ++ww) {
                    const double v = (double)sCol[base + ww * kSuper + tid];
                    if (v < best) { best = v; arg = sArg[base + ww * kSuper + tid]; }
                }
                a.part_min[(size_t)strip * g.ld + j] = best;
                a.part_arg[(size_t)strip * g.ld + j] = arg;
            } else {
                T v = sCol[base + tid];
                for (int ww = 1; ww < kWaves; ++ww) v += sCol[base + ww * kSuper + tid];
                static_cast<T *>(a.part_col)[(size_t)strip * g.ld + j] = v;
                if constexpr (kTrial) {
                    T v2 = sCol2[base + tid];
                    for (int ww = 1; ww < kWaves; ++ww) v2 += sCol2[base + ww * kSuper + tid];
                    static_cast<T *>(a.part_col2)[(size_t)strip * g.ld + j] = v2;
                }
            }
        }
    }

    if (kAdjoint) {
        // D layout: lane (lr, lq) holds rows m = 16 mb + 4 lq + r of (Lam Xhat)^T for row i.
        // swapped rows accumulated candidate b in acc and a in acc2
        T *pacc = static_cast<T *>(cswap ? a.part_acc2 : a.part_acc) + ((size_t)chunk * g.Nr + i) * NP;
        T *pacc2 = kTrial ? static_cast<T *>(cswap ? a.part_acc : a.part_acc2) + ((size_t)chunk * g.Nr + i) * NP
                          : nullptr;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            if (sizeof(T) == 8) {
                *reinterpret_cast<d4 *>(reinterpret_cast<double *>(pacc) + 16 * mb + 4 * lq) =
                    d4{(double)acc[mb][0], (double)acc[mb][1], (double)acc[mb][2], (double)acc[mb][3]};
            } else {
                *reinterpret_cast<f4 *>(reinterpret_cast<float *>(pacc) + 16 * mb + 4 * lq) =
                    f4{(float)acc[mb][0], (float)acc[mb][1], (float)acc[mb][2], (float)acc[mb][3]};
            }
            if constexpr (kTrial) {
                if (sizeof(T) == 8) {
                    *reinterpret_cast<d4 *>(reinterpret_cast<double *>(pacc2) + 16 * mb + 4 * lq) =
                        d4{(double)acc2[mb][0], (double)acc2[mb][1], (double)acc2[mb][2], (double)acc2[mb][3]};
                } else {
                    *reinterpret_cast<f4 *>(reinterpret_cast<float *>(pacc2) + 16 * mb + 4 * lq) =
                        f4{(float)acc2[mb][0], (float)acc2[mb][1], (float)acc2[mb][2], (float)acc2[mb][3]};
                }
            }
        }
    }

    if (MODE == PASS_KKT || MODE == PASS_POWER || kTrial) {
        if (cswap) {
            const double t0 = red0, t2 = red2;
            red0 = red1; red1 = t0;
            red2 = red3; red3 = t2;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            red0 = (MODE == PASS_KKT) ? fmax(red0, __shfl_xor(red0, m, 64)) : red0 + __shfl_xor(red0, m, 64);
            red1 = kTrial ? red1 + __shfl_xor(red1, m, 64) : fmax(red1, __shfl_xor(red1, m, 64));
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
                else if (MODE == PASS_POWER && tid == 1) v = fmax(v, o);
                else v += o;
            }
            a.part_red[(size_t)bid * kRed + tid] = v;
        }
    }
}

template <typename T, int REP, int MODE, int MB, int KT = 0>
__global__ __launch_bounds__(64 * kWaves) void pass_kernel(PassArgs a, Geometry g) {
    pass_body<T, REP, MODE, MB, KT>(a, g, blockIdx.x);
}

// Grouped pass: the workgroups of several fits (same template parameters) in one launch; fit f
// owns workgroups [off[f], off[f + 1]).  Each fit's tiles, reductions and outputs are those of its
// own launch, so its results are bitwise the same grouped or alone.
template <typename T, int REP, int MODE, int MB, int KT = 0>
__global__ __launch_bounds__(64 * kWaves) void pass_group_kernel(PassGroup G) {
    int f = 0;
    while (f + 1 < G.nfit && (int)blockIdx.x >= G.off[f + 1]) ++f;
    pass_body<T, REP, MODE, MB, KT>(G.a[f], G.g[f], (int)blockIdx.x - G.off[f]);
}

static int env_int(const char *name, int def) {
    const char *v = getenv(name);
    return v ? atoi(v) : def;
}

Geometry make_geometry(int N, int n, int slots) {
    Geometry g;
    g.N = N;
    g.n = n;
    g.MB = (n + 1 + 15) / 16;
    g.NP = 16 * g.MB;
    g.ks1 = (n + 3) / 4;
    g.Nr = ((N + kRows - 1) / kRows) * kRows;
    g.Nr = ((g.Nr + kSuper - 1) / kSuper) * kSuper;
    g.ld = g.Nr;
    g.strips = g.Nr / kRows;
    const int supers = g.ld / kSuper;
    if (slots <= 0) slots = 256;
    int best = 1;
    double best_eff = -1.0;
    const int forced = env_int("CR_CHUNKS", 0);
    for (int c = 1; c <= 16 && c <= supers; ++c) {
        const int per = (supers + c - 1) / c;
        const int chunks = (supers + per - 1) / per;
        if (chunks != c) continue;                      // same split as a smaller count
        const long wgs = (long)g.strips * chunks;
        const long rounds = (wgs + slots - 1) / slots;
        // balance: the last column chunk may be shorter than the others
        const double col_eff = (double)supers / ((double)chunks * per);
        const double eff = (double)wgs / ((double)rounds * slots) * col_eff;
        if (eff > best_eff + 0.02) { best_eff = eff; best = c; }
    }
    if (forced > 0) best = forced < supers ? forced : supers;
    const int per = (supers + best - 1) / best;
    g.chunk_cols = per * kSuper;
    g.chunks = (g.ld + g.chunk_cols - 1) / g.chunk_cols;
    return g;
}

template <typename T, int REP, int MODE, int KT>
static void launch_kt(const Geometry &g, const PassArgs &a, hipStream_t st) {
    dim3 grid(g.grid()), block(64 * kWaves);
    switch (g.MB) {
    case 1: hipLaunchKernelGGL((pass_kernel<T, REP, MODE, 1, KT>), grid, block, 0, st, a, g); break;
    case 2: hipLaunchKernelGGL((pass_kernel<T, REP, MODE, 2, KT>), grid, block, 0, st, a, g); break;
    case 3: hipLaunchKernelGGL((pass_kernel<T, REP, MODE, 3, KT>), grid, block, 0, st, a, g); break;
    default: hipLaunchKernelGGL((pass_kernel<T, REP, MODE, 4, KT>), grid, block, 0, st, a, g); break;
    }
}

// The per-iteration modes drop the two last residual K-steps when they hold no feature
// (4 MB - ceil(n / 4) >= 2, e.g. n = 40: 10 of 12 steps); the other modes keep all 4 MB.
template <typename T, int REP, int MODE>
static hipError_t launch_mb(const Geometry &g, const PassArgs &a, hipStream_t st) {
    if (g.MB < 1 || g.MB > kMaxMB) return hipErrorInvalidValue;
    constexpr bool kHot = (MODE == PASS_STEP || MODE == PASS_TRIAL || MODE == PASS_TRIAL_NS || MODE == PASS_ADV);
    if (kHot && 4 * g.MB - g.ks1 >= 2) launch_kt<T, REP, MODE, kHot ? 2 : 0>(g, a, st);
    else launch_kt<T, REP, MODE, 0>(g, a, st);
    return hipGetLastError();
}

hipError_t launch_pass(const Geometry &g, PassMode mode, bool fp32, LamRep rep, const PassArgs &a,
                       hipStream_t st) {
    if (g.MB < 1 || g.MB > kMaxMB) return hipErrorInvalidValue;
    switch (mode) {
    case PASS_STEP:
        if (!fp32 && rep == REP_F64) return launch_mb<double, REP_F64, PASS_STEP>(g, a, st);
        if (fp32 && rep == REP_SPLIT_F32) return launch_mb<float, REP_SPLIT_F32, PASS_STEP>(g, a, st);
        if (fp32 && rep == REP_SPLIT_BF16) return launch_mb<float, REP_SPLIT_BF16, PASS_STEP>(g, a, st);
        return hipErrorInvalidValue;
    case PASS_ADJ:
        if (fp32) return hipErrorInvalidValue;
        if (rep == REP_F64) return launch_mb<double, REP_F64, PASS_ADJ>(g, a, st);
        if (rep == REP_SPLIT_F32) return launch_mb<double, REP_SPLIT_F32, PASS_ADJ>(g, a, st);
        return launch_mb<double, REP_SPLIT_BF16, PASS_ADJ>(g, a, st);
    case PASS_KKT:
        if (fp32) return hipErrorInvalidValue;
        if (rep == REP_F64) return launch_mb<double, REP_F64, PASS_KKT>(g, a, st);
        if (rep == REP_SPLIT_F32) return launch_mb<double, REP_SPLIT_F32, PASS_KKT>(g, a, st);
        return launch_mb<double, REP_SPLIT_BF16, PASS_KKT>(g, a, st);
    case PASS_REBASE:
        if (fp32) return hipErrorInvalidValue;
        if (rep == REP_SPLIT_F32) return launch_mb<double, REP_SPLIT_F32, PASS_REBASE>(g, a, st);
        if (rep == REP_SPLIT_BF16) return launch_mb<double, REP_SPLIT_BF16, PASS_REBASE>(g, a, st);
        return hipErrorInvalidValue;
    case PASS_POWER:   // reads no multipliers: REP_F64 only sets the tile shape
        if (fp32) return launch_mb<float, REP_F64, PASS_POWER>(g, a, st);
        return launch_mb<double, REP_F64, PASS_POWER>(g, a, st);
    case PASS_REPAIR:
        if (fp32) return hipErrorInvalidValue;
        return launch_mb<double, REP_F64, PASS_REPAIR>(g, a, st);
    case PASS_RESID:
        if (fp32 || rep != REP_F64) return hipErrorInvalidValue;
        return launch_mb<double, REP_F64, PASS_RESID>(g, a, st);
    case PASS_TRIAL:   // the storing trial pass (FP64); the split forms re-form instead
        if (!fp32 && rep == REP_F64) return launch_mb<double, REP_F64, PASS_TRIAL>(g, a, st);
        return hipErrorInvalidValue;
    case PASS_TRIAL_NS:
        if (!fp32 && rep == REP_F64) return launch_mb<double, REP_F64, PASS_TRIAL_NS>(g, a, st);
        if (fp32 && rep == REP_SPLIT_F32) return launch_mb<float, REP_SPLIT_F32, PASS_TRIAL_NS>(g, a, st);
        if (fp32 && rep == REP_SPLIT_BF16) return launch_mb<float, REP_SPLIT_BF16, PASS_TRIAL_NS>(g, a, st);
        return hipErrorInvalidValue;
    case PASS_ADV:
        if (!fp32 && rep == REP_F64) return launch_mb<double, REP_F64, PASS_ADV>(g, a, st);
        if (fp32 && rep == REP_SPLIT_F32) return launch_mb<float, REP_SPLIT_F32, PASS_ADV>(g, a, st);
        if (fp32 && rep == REP_SPLIT_BF16) return launch_mb<float, REP_SPLIT_BF16, PASS_ADV>(g, a, st);
        return hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

int pass_group_key(const Geometry &g, PassMode mode, bool fp32, LamRep rep) {
    constexpr int kHotTrim = 2;
    const bool hot = (mode == PASS_STEP || mode == PASS_TRIAL || mode == PASS_TRIAL_NS || mode == PASS_ADV);
    const int kt = (hot && 4 * g.MB - g.ks1 >= kHotTrim) ? kHotTrim : 0;
    return (((int)mode * 2 + (fp32 ? 1 : 0)) * 4 + (int)rep) * 64 + g.MB * 8 + kt;
}

template <typename T, int REP, int MODE, int KT>
static void launch_group_kt(const PassGroup &G, int MB, hipStream_t st) {
    dim3 grid(G.off[G.nfit]), block(64 * kWaves);
    switch (MB) {
    case 1: hipLaunchKernelGGL((pass_group_kernel<T, REP, MODE, 1, KT>), grid, block, 0, st, G); break;
    case 2: hipLaunchKernelGGL((pass_group_kernel<T, REP, MODE, 2, KT>), grid, block, 0, st, G); break;
    case 3: hipLaunchKernelGGL((pass_group_kernel<T, REP, MODE, 3, KT>), grid, block, 0, st, G); break;
    default: hipLaunchKernelGGL((pass_group_kernel<T, REP, MODE, 4, KT>), grid, block, 0, st, G); break;
    }
}

template <typename T, int REP, int MODE>
static hipError_t launch_group_mb(const PassGroup &G, hipStream_t st) {
    const Geometry &g = G.g[0];
    if (g.MB < 1 || g.MB > kMaxMB) return hipErrorInvalidValue;
    if (4 * g.MB - g.ks1 >= 2) launch_group_kt<T, REP, MODE, 2>(G, g.MB, st);
    else launch_group_kt<T, REP, MODE, 0>(G, g.MB, st);
    return hipGetLastError();
}

// The grouped forms of the per-iteration trial passes (the adaptive step's sweeps).
hipError_t launch_pass_group(PassMode mode, bool fp32, LamRep rep, const PassGroup &G, hipStream_t st) {
    if (G.nfit < 1 || G.nfit > kGroupMax) return hipErrorInvalidValue;
    const int key = pass_group_key(G.g[0], mode, fp32, rep);
    for (int f = 1; f < G.nfit; ++f)
        if (pass_group_key(G.g[f], mode, fp32, rep) != key) return hipErrorInvalidValue;
    switch (mode) {
    case PASS_TRIAL:
        if (!fp32 && rep == REP_F64) return launch_group_mb<double, REP_F64, PASS_TRIAL>(G, st);
        return hipErrorInvalidValue;
    case PASS_TRIAL_NS:
        if (!fp32 && rep == REP_F64) return launch_group_mb<double, REP_F64, PASS_TRIAL_NS>(G, st);
        if (fp32 && rep == REP_SPLIT_F32) return launch_group_mb<float, REP_SPLIT_F32, PASS_TRIAL_NS>(G, st);
        if (fp32 && rep == REP_SPLIT_BF16) return launch_group_mb<float, REP_SPLIT_BF16, PASS_TRIAL_NS>(G, st);
        return hipErrorInvalidValue;
    case PASS_ADV:
        if (!fp32 && rep == REP_F64) return launch_group_mb<double, REP_F64, PASS_ADV>(G, st);
        if (fp32 && rep == REP_SPLIT_F32) return launch_group_mb<float, REP_SPLIT_F32, PASS_ADV>(G, st);
        if (fp32 && rep == REP_SPLIT_BF16) return launch_group_mb<float, REP_SPLIT_BF16, PASS_ADV>(G, st);
        return hipErrorInvalidValue;
    default:
        return hipErrorInvalidValue;
    }
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
    double u = csum - rsum;
    if (a.ubase) u += a.ubase[i];
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
            if (a.wbase) v += a.wbase[(size_t)i * NP + m];
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

__global__ void normalize_kernel(double *y, double *xi, double *dmy, float *y32, float *xi32, float *dmy32,
                                 const double *sq, int Nr, int NP) {
    const double f = 1.0 / sqrt(sq[0] + sq[1]);
    const size_t tot = (size_t)Nr * NP;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const double v = xi[e] * f;
        xi[e] = v;
        if (xi32) xi32[e] = (float)v;
        if (e < (size_t)Nr) {
            const double a = y[e] * f, d = dmy[e] * f;
            y[e] = a;
            dmy[e] = d;
            if (y32) { y32[e] = (float)a; dmy32[e] = (float)d; }
        }
    }
}

hipError_t launch_normalize(const Geometry &g, double *y, double *xi, double *dmy, float *y32, float *xi32,
                            float *dmy32, const double *sq, hipStream_t st) {
    const int blocks = (int)(((size_t)g.Nr * g.NP + 255) / 256);
    hipLaunchKernelGGL(normalize_kernel, dim3(blocks < 4096 ? blocks : 4096), dim3(256), 0, st, y, xi,
                       dmy, y32, xi32, dmy32, sq, g.Nr, g.NP);
    return hipGetLastError();
}

// ---- representation changes -------------------------------------------------------------------
__device__ __forceinline__ double hi_load(const void *p, LamRep rep, size_t e) {
    if (rep == REP_SPLIT_F32) return (double)static_cast<const float *>(p)[e];
    return (double)bf16_to_float(static_cast<const uint16_t *>(p)[e]);
}

__global__ void merge_kernel(LamRep rep, const void *hi, const float *lo, double *dst, size_t tot) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = hi_load(hi, rep, e) + (double)lo[e];
}

hipError_t launch_merge(const Geometry &g, LamRep rep, const void *hi, const float *lo, double *dst, hipStream_t st) {
    if (rep == REP_F64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(merge_kernel, dim3(8192), dim3(256), 0, st, rep, hi, lo, dst, (size_t)g.Nr * g.ld);
    return hipGetLastError();
}

__global__ void pack_kernel(const double *dense, LamRep rep, void *main, float *lo, int N, int Nr, int ld) {
    const size_t tot = (size_t)Nr * ld;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / ld), j = (int)(e - (size_t)i * ld);
        double v = 0.0;
        if (i < N && j < N && i != j) v = dense[(size_t)i * N + j];
        if (rep == REP_F64) {
            static_cast<double *>(main)[e] = v;
        } else {
            float h = (float)v;
            if (rep == REP_SPLIT_BF16) {
                const uint16_t hb = float_to_bf16(h);
                static_cast<uint16_t *>(main)[e] = hb;
                h = bf16_to_float(hb);
            } else {
                static_cast<float *>(main)[e] = h;
            }
            lo[e] = (float)(v - (double)h);
        }
    }
}

__global__ void unpack_kernel(LamRep rep, const void *main, const float *lo, double *dense, int N, int ld) {
    const size_t tot = (size_t)N * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
        const size_t f = (size_t)i * ld + j;
        double v;
        if (rep == REP_F64) v = static_cast<const double *>(main)[f];
        else v = hi_load(main, rep, f) + (double)lo[f];
        dense[e] = (i == j) ? 0.0 : v;
    }
}

__global__ void unpack_rows_kernel(LamRep rep, const void *main, const float *lo, double *dense, int N, int ld,
                                   int row0, int nrows) {
    const size_t tot = (size_t)nrows * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / N), j = (int)(e - (size_t)r * N);
        const int i = row0 + r;
        const size_t f = (size_t)i * ld + j;
        double v;
        if (rep == REP_F64) v = static_cast<const double *>(main)[f];
        else v = hi_load(main, rep, f) + (double)lo[f];
        dense[e] = (i == j) ? 0.0 : v;
    }
}

hipError_t launch_unpack_rows(const Geometry &g, LamRep rep, const void *main, const float *lo, int row0, int nrows,
                              double *dense, hipStream_t st) {
    hipLaunchKernelGGL(unpack_rows_kernel, dim3(1024), dim3(256), 0, st, rep, main, lo, dense, g.N, g.ld, row0, nrows);
    return hipGetLastError();
}

hipError_t launch_pack_lambda(const Geometry &g, const double *dense, LamRep rep, void *main, float *lo,
                              hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3(8192), dim3(256), 0, st, dense, rep, main, lo, g.N, g.Nr, g.ld);
    return hipGetLastError();
}

hipError_t launch_unpack_lambda(const Geometry &g, LamRep rep, const void *main, const float *lo, double *dense,
                                hipStream_t st) {
    hipLaunchKernelGGL(unpack_kernel, dim3(8192), dim3(256), 0, st, rep, main, lo, dense, g.N, g.ld);
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
__global__ void power_init_kernel(const double *xhat64, double *y, double *xi, double *dmy, float *y32,
                                  float *xi32, float *dmy32, int N, int n, int Nr, int NP, double inv_norm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nr) return;
    double vy = 0.0, d = 0.0;
    if (i < N) {
        vy = (N > 1 ? -1.0 + 2.0 * (double)i / (double)(N - 1) : 0.0) * inv_norm;
        for (int m = 0; m < n; ++m) d += inv_norm * xhat64[(size_t)i * NP + m];
    }
    for (int m = 0; m < NP; ++m) {
        const double v = (i < N && m < n) ? inv_norm : 0.0;
        xi[(size_t)i * NP + m] = v;
        if (xi32) xi32[(size_t)i * NP + m] = (float)v;
    }
    y[i] = vy;
    dmy[i] = d - vy;
    if (y32) { y32[i] = (float)vy; dmy32[i] = (float)(d - vy); }
}

hipError_t launch_power_init(const Geometry &g, const double *xhat64, double *y, double *xi, double *dmy,
                             float *y32, float *xi32, float *dmy32, hipStream_t st) {
    // ||v||^2 = sum_l (-1 + 2l/(N-1))^2 + N n, summed on the host in a fixed order
    double s = 0.0;
    for (int l = 0; l < g.N; ++l) {
        const double v = g.N > 1 ? -1.0 + 2.0 * (double)l / (double)(g.N - 1) : 0.0;
        s += v * v;
    }
    s += (double)g.N * (double)g.n;
    hipLaunchKernelGGL(power_init_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, xhat64, y, xi, dmy, y32, xi32,
                       dmy32, g.N, g.n, g.Nr, g.NP, 1.0 / sqrt(s));
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
                                     double *rowred, double xspan, int N, int Nr, int ld, int strips,
                                     int NP) {
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
    // j keeps its own slope unless another piece exceeds it by more than the rounding scale
    // (ties at the optimum are decided by rounding; switching slopes there would inflate the gap)
    double xi1 = 0.0;
    for (int m = 0; m < NP; ++m) xi1 += fabs(xi[(size_t)j * NP + m]);
    const double tau = 1e-10 * (1.0 + fabs(y[j]) + xi1 * xspan);
    const double shift = best < 0.0 ? best : 0.0;
    const int piece = best < -tau ? arg : j;
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

__global__ __launch_bounds__(256) void relax_finish_kernel(const double *part_min, const double *c_in,
                                                          double *c_out, const double *y, const double *xi,
                                                          const double *ybar, double xspan, double *rowred,
                                                          double *changed, int N, int Nr, int ld, int strips,
                                                          int NP) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    int grew = 0;
    if (j < N) {
        double m = INFINITY;
        for (int s = 0; s < strips; ++s) m = fmin(m, part_min[(size_t)s * ld + j]);
        const double c0 = c_in[j];
        const double c1 = fmax(c0, -m);
        double xi1 = 0.0;
        for (int q = 0; q < NP; ++q) xi1 += fabs(xi[(size_t)j * NP + q]);
        const double tau = 1e-10 * (1.0 + fabs(y[j]) + xi1 * xspan);
        grew = c1 > c0 + tau ? 1 : 0;
        c_out[j] = c1;
        const double dy = y[j] + c1 - ybar[j];
        rowred[2 * (size_t)j] = dy * dy;
        rowred[2 * (size_t)j + 1] = 0.0;
    } else if (j < Nr) {
        c_out[j] = 0.0;
        rowred[2 * (size_t)j] = 0.0;
        rowred[2 * (size_t)j + 1] = 0.0;
    }
    __shared__ int sh[256];
    sh[threadIdx.x] = grew;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) changed[blockIdx.x] = (double)sh[0];
}

hipError_t launch_relax_finish(const Geometry &g, const double *part_min, const double *c_in, double *c_out,
                               const double *y, const double *xi, const double *ybar, double xspan,
                               double *rowred, double *changed, hipStream_t st) {
    hipLaunchKernelGGL(relax_finish_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, part_min, c_in, c_out, y, xi,
                       ybar, xspan, rowred, changed, g.N, g.Nr, g.ld, g.strips, g.NP);
    return hipGetLastError();
}

hipError_t launch_repair_finish(const Geometry &g, const double *part_min, const int *part_arg, const double *y,
                                const double *xi, const double *ybar, double *y_rep, double *xi_rep,
                                double *rowred, double xspan, hipStream_t st) {
    hipLaunchKernelGGL(repair_finish_kernel, dim3((g.Nr + 255) / 256), dim3(256), 0, st, part_min, part_arg, y, xi,
                       ybar, y_rep, xi_rep, rowred, xspan, g.N, g.Nr, g.ld, g.strips, g.NP);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint4 *p, size_t n16, uint8_t *tail, int ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n16; e += stride) p[e] = uint4{0, 0, 0, 0};
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16;
    const int ntail = (int)(bytes - n16 * 16);
    const size_t blocks = std::min<size_t>(4096, std::max<size_t>(1, (n16 + 255) / 256));
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<uint4 *>(p), n16,
                       static_cast<uint8_t *>(p) + n16 * 16, ntail);
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

// 16 threads per row (features m = t, t + 16, ...), 16 rows per 256-thread block: row segments
// are read and written as whole 128-byte lines.
__global__ __launch_bounds__(256) void lincomb_kernel(const double *ya, const double *xia, const double *yb,
                                                     const double *xib, double cya, double cyb, double cxa,
                                                     double cxb, const double *xhat64, double *y, double *xi,
                                                     double *dmy, float *y32, float *xi32, float *dmy32, int N, int n,
                                                     int Nr, int NP) {
    const int t = threadIdx.x & 15;
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4);   // grid covers Nr exactly
    double d = 0.0;
    for (int m = t; m < NP; m += 16) {
        const size_t e = (size_t)i * NP + m;
        const double v = cxa * xia[e] + cxb * xib[e];
        xi[e] = v;
        if (xi32) xi32[e] = (float)v;
        if (m < n) d += v * xhat64[e];
    }
    for (int s = 1; s < 16; s <<= 1) d += __shfl_xor(d, s, 16);
    if (t == 0) {
        const double yy = cya * ya[i] + cyb * yb[i];
        y[i] = yy;
        dmy[i] = i < N ? d - yy : 0.0;
        if (y32) y32[i] = (float)yy;
        if (dmy32) dmy32[i] = i < N ? (float)(d - yy) : 0.f;
    }
}

hipError_t launch_lincomb(const Geometry &g, const double *ya, const double *xia, const double *yb,
                          const double *xib, double cya, double cyb, double cxa, double cxb, const double *xhat64,
                          double *y, double *xi, double *dmy, float *y32, float *xi32, float *dmy32, hipStream_t st) {
    hipLaunchKernelGGL(lincomb_kernel, dim3(g.Nr / 16), dim3(256), 0, st, ya, xia, yb, xib, cya, cyb, cxa, cxb, xhat64,
                       y, xi, dmy, y32, xi32, dmy32, g.N, g.n, g.Nr, g.NP);
    return hipGetLastError();
}

// Accepted adaptive step: eta(lam^{k+1}) = eta(lam~^{k+1}) + (A1^T D, A2^T D / delta) into
// (ye, xie, dmye), then the next extrapolated point (1 + beta) eta(lam^{k+1}) - beta eta(lam^k) into
// the pass arrays (y, xi, dmy and their FP32 copies).  (yt, xit) hold eta(lam~^{k+1}); they may be
// the same arrays as (y, xi).
// With `decision` set, the candidate (0 or 1; negative: none, the kernel does nothing) and beta
// are read from decision[0], decision[1] as the trial reduction left them, and uD / wD point at
// the two candidates' adjoints; otherwise candidate 0 and the `beta` argument are used.
__device__ __forceinline__ void accept_body(const AcceptArgs &a, const int bid) {
    const double *uD = a.uD0, *wD = a.wD0;
    double beta = a.beta;
    if (a.decision) {
        const double acc = a.decision[0];
        if (acc < 0.0) return;
        beta = a.decision[1];
        if (acc > 0.5) { uD = a.uD1; wD = a.wD1; }
    }
    const int NP = a.NP;
    const int t = threadIdx.x & 15;
    const int i = bid * 16 + (threadIdx.x >> 4);
    double dn = 0.0, dp = 0.0;
    for (int m = t; m < NP; m += 16) {
        const size_t e = (size_t)i * NP + m;
        const double xn = a.xit[e] + wD[e] * a.inv_delta;
        const double xp = (1.0 + beta) * xn - beta * a.xik[e];
        a.xie[e] = xn;
        a.xi[e] = xp;
        if (a.xi32) a.xi32[e] = (float)xp;
        if (m < a.n) {
            dn += xn * a.xhat64[e];
            dp += xp * a.xhat64[e];
        }
    }
    for (int s = 1; s < 16; s <<= 1) {
        dn += __shfl_xor(dn, s, 16);
        dp += __shfl_xor(dp, s, 16);
    }
    if (t == 0) {
        const bool valid = i < a.N;
        const double yn = a.yt[i] + uD[i];
        const double yp = (1.0 + beta) * yn - beta * a.yk[i];
        a.ye[i] = yn;
        a.dmye[i] = valid ? dn - yn : 0.0;
        a.y[i] = yp;
        a.dmy[i] = valid ? dp - yp : 0.0;
        if (a.y32) a.y32[i] = (float)yp;
        if (a.dmy32) a.dmy32[i] = valid ? (float)(dp - yp) : 0.f;
    }
}

__global__ __launch_bounds__(256) void accept_kernel(AcceptArgs a) { accept_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void accept_group_kernel(AcceptGroup G) {
    int f = 0;
    while (f + 1 < G.nfit && (int)blockIdx.x >= G.off[f + 1]) ++f;
    accept_body(G.a[f], (int)blockIdx.x - G.off[f]);
}

AcceptArgs make_accept_args(const Geometry &g, const double *yt, const double *xit, double *y, double *xi,
                            double *dmy, const double *const uD[2], const double *const wD[2], const double *yk,
                            const double *xik, double *ye, double *xie, double *dmye, float *y32, float *xi32,
                            float *dmy32, const double *xhat64, double inv_delta, double beta,
                            const double *decision) {
    AcceptArgs a;
    a.yt = yt; a.xit = xit; a.y = y; a.xi = xi; a.dmy = dmy;
    a.uD0 = uD[0]; a.uD1 = uD[1]; a.wD0 = wD[0]; a.wD1 = wD[1];
    a.yk = yk; a.xik = xik; a.ye = ye; a.xie = xie; a.dmye = dmye;
    a.y32 = y32; a.xi32 = xi32; a.dmy32 = dmy32; a.xhat64 = xhat64;
    a.inv_delta = inv_delta; a.beta = beta; a.decision = decision;
    a.N = g.N; a.n = g.n; a.NP = g.NP;
    return a;
}

hipError_t launch_accept(const Geometry &g, const double *yt, const double *xit, double *y, double *xi, double *dmy,
                         const double *const uD[2], const double *const wD[2], const double *yk, const double *xik,
                         double *ye, double *xie, double *dmye, float *y32, float *xi32, float *dmy32,
                         const double *xhat64, double inv_delta, double beta, const double *decision, hipStream_t st) {
    const AcceptArgs a = make_accept_args(g, yt, xit, y, xi, dmy, uD, wD, yk, xik, ye, xie, dmye, y32, xi32, dmy32,
                                          xhat64, inv_delta, beta, decision);
    hipLaunchKernelGGL(accept_kernel, dim3(g.Nr / 16), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_accept_args(const Geometry &g, const AcceptArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(accept_kernel, dim3(g.Nr / 16), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_accept_group(const AcceptGroup &G, hipStream_t st) {
    if (G.nfit < 1 || G.nfit > kGroupMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(accept_group_kernel, dim3(G.off[G.nfit]), dim3(256), 0, st, G);
    return hipGetLastError();
}

// Both candidates of a trial pass: adjoints (A1^T D_q, A2^T D_q) from the pass partials, like the
// power-mode finalize, plus per-block sums of ||A1^T D_q||^2 and ||A2^T D_q||^2 (4 per block).
// The two candidates run in the two halves of the workgroup (threads 0-255 and 256-511).
template <typename T, int MB>
__device__ __forceinline__ void trial_finalize_body(const TrialFinalizeArgs &a, const Geometry &g, const int bid) {
    constexpr int NP = 16 * MB;
    const int q = threadIdx.x >> 8;
    const int t = threadIdx.x & 15;
    const int r = (threadIdx.x & 255) >> 4;
    const int i = bid * 16 + r;
    const bool valid = i < g.N;
    __shared__ double sh[16][4];
    {
        const T *pacc = static_cast<const T *>(q ? a.part_acc[1] : a.part_acc[0]);
        const T *pcol = static_cast<const T *>(q ? a.part_col[1] : a.part_col[0]);
        double lx[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            double s = 0.0;
            for (int c = 0; c < g.chunks; ++c) s += (double)pacc[((size_t)c * g.Nr + i) * NP + 16 * mb + t];
            lx[mb] = s;
        }
        double mine = 0.0;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            if (16 * mb + t == g.n) mine = lx[mb];
        double rsum = mine;
        for (int m = 1; m < 16; m <<= 1) rsum += __shfl_xor(rsum, m, 16);
        double csum = 0.0;
        for (int s = t; s < g.strips; s += 16) csum += (double)pcol[(size_t)s * g.ld + i];
        for (int m = 1; m < 16; m <<= 1) csum += __shfl_xor(csum, m, 16);
        const double u = valid ? csum - rsum : 0.0;
        double wsq = 0.0;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int m = 16 * mb + t;
            double v = 0.0;
            if (valid && m < g.n) v = rsum * a.xf[(size_t)i * NP + m] - lx[mb];
            (q ? a.wD[1] : a.wD[0])[(size_t)i * NP + m] = v;
            wsq += v * v;
        }
        for (int m = 1; m < 16; m <<= 1) wsq += __shfl_xor(wsq, m, 16);
        if (t == 0) {
            (q ? a.uD[1] : a.uD[0])[i] = u;
            sh[r][2 * q] = u * u;
            sh[r][2 * q + 1] = wsq;
        }
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int rr = 0; rr < 16; ++rr) s += sh[rr][threadIdx.x];
        a.block_part[(size_t)bid * 4 + threadIdx.x] = s;
    }
}

template <typename T, int MB>
__global__ __launch_bounds__(512) void trial_finalize_kernel(TrialFinalizeArgs a, Geometry g) {
    trial_finalize_body<T, MB>(a, g, blockIdx.x);
}

template <typename T, int MB>
__global__ __launch_bounds__(512) void trial_finalize_group_kernel(TrialFinalizeGroup G) {
    int f = 0;
    while (f + 1 < G.nfit && (int)blockIdx.x >= G.off[f + 1]) ++f;
    trial_finalize_body<T, MB>(G.a[f], G.g[f], (int)blockIdx.x - G.off[f]);
}

hipError_t launch_trial_finalize_group(bool fp32, int MB, const TrialFinalizeGroup &G, hipStream_t st) {
    if (G.nfit < 1 || G.nfit > kGroupMax) return hipErrorInvalidValue;
    dim3 grid(G.off[G.nfit]), block(512);
#define CR_TFING(T, MBV) hipLaunchKernelGGL((trial_finalize_group_kernel<T, MBV>), grid, block, 0, st, G)
    if (fp32) {
        switch (MB) { case 1: CR_TFING(float, 1); break; case 2: CR_TFING(float, 2); break;
                      case 3: CR_TFING(float, 3); break; case 4: CR_TFING(float, 4); break;
                      default: return hipErrorInvalidValue; }
    } else {
        switch (MB) { case 1: CR_TFING(double, 1); break; case 2: CR_TFING(double, 2); break;
                      case 3: CR_TFING(double, 3); break; case 4: CR_TFING(double, 4); break;
                      default: return hipErrorInvalidValue; }
    }
#undef CR_TFING
    return hipGetLastError();
}

hipError_t launch_trial_finalize(const Geometry &g, bool fp32, const TrialFinalizeArgs &a, hipStream_t st) {
    dim3 grid(g.Nr / 16), block(512);
#define CR_TFIN(T, MBV) hipLaunchKernelGGL((trial_finalize_kernel<T, MBV>), grid, block, 0, st, a, g)
    if (fp32) {
        switch (g.MB) { case 1: CR_TFIN(float, 1); break; case 2: CR_TFIN(float, 2); break;
                        case 3: CR_TFIN(float, 3); break; case 4: CR_TFIN(float, 4); break;
                        default: return hipErrorInvalidValue; }
    } else {
        switch (g.MB) { case 1: CR_TFIN(double, 1); break; case 2: CR_TFIN(double, 2); break;
                        case 3: CR_TFIN(double, 3); break; case 4: CR_TFIN(double, 4); break;
                        default: return hipErrorInvalidValue; }
    }
#undef CR_TFIN
    return hipGetLastError();
}

// The eight trial scalars in one single-workgroup launch, fixed order: out[q] = sum_b pa[b * 4 + q]
// for q < 4 (the finalize's per-block sums), out[4 + q] = sum_b pb[b * kRed + q] (the pass's
// reduction slots).  `out` may be pinned host memory (written once, read after the stream syncs).
//
// It also takes the step test's decision (eq. "eq:adaptive-check" with every pair dualized:
// ||A1^T D||^2 + ||A2^T D||^2 / delta <= s ||D||^2, candidate a first), so that the accept kernel
// queued behind it needs no host round trip: decision[0] = 0 / 1 (candidate), -1 (neither: retry),
// -2 (a non-finite scalar); decision[1] = beta_k, decision[2] = t_{k+1}, decision[3] = 1 if the
// momentum restarts (restart on and <D, candidate - lam^k> < 0).  The same four values follow the
// eight scalars in out[8..11].
__device__ __forceinline__ void trial_reduce_body(const double *pa, int ba, const double *pb, int bb, double *out,
                                                  unsigned long long *seq_out, unsigned long long seq,
                                                  const TrialRule &rule, double *decision) {
    __shared__ double sh[8][256];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double v = 0.0;
        if (q < 4) {
            for (int b = threadIdx.x; b < ba; b += 256) v += pa[(size_t)b * 4 + q];
        } else {
            for (int b = threadIdx.x; b < bb; b += 256) v += pb[(size_t)b * kRed + q - 4];
        }
        sh[q][threadIdx.x] = v;
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
#pragma unroll
            for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) out[q] = sh[q][0];
        double acc = -1.0, rs = 0.0, tt = rule.t;
        bool finite = true;
#pragma unroll
        for (int q = 0; q < 8; ++q) finite = finite && isfinite(sh[q][0]);
        if (!finite) {
            acc = -2.0;
        } else {
            const double curv_a = sh[0][0] + sh[1][0] / rule.delta, curv_b = sh[2][0] + sh[3][0] / rule.delta;
            if (curv_a <= rule.s_a * sh[4][0] * (1.0 + 1e-12)) { acc = 0.0; rs = sh[6][0] < 0.0 ? 1.0 : 0.0; }
            else if (curv_b <= rule.s_b * sh[5][0] * (1.0 + 1e-12)) { acc = 1.0; rs = sh[7][0] < 0.0 ? 1.0 : 0.0; }
        }
        if (!rule.restart) rs = 0.0;
        if (rs != 0.0) tt = 1.0;
        const double t_next = (1.0 + sqrt(1.0 + 4.0 * tt * tt)) / 2.0;
        const double beta_k = rule.momentum ? (tt - 1.0) / t_next : 0.0;
        out[8] = acc; out[9] = beta_k; out[10] = t_next; out[11] = rs;
        if (decision) {
            decision[0] = acc; decision[1] = beta_k; decision[2] = t_next; decision[3] = rs;
        }
        if (seq_out) {
            // the eight values reach system scope before the sequence word that announces them
            __threadfence_system();
            *reinterpret_cast<volatile unsigned long long *>(seq_out) = seq;
        }
    }
}

__global__ __launch_bounds__(256) void trial_reduce_kernel(const double *pa, int ba, const double *pb, int bb,
                                                          double *out, unsigned long long *seq_out,
                                                          unsigned long long seq, TrialRule rule,
                                                          double *decision) {
    trial_reduce_body(pa, ba, pb, bb, out, seq_out, seq, rule, decision);
}

// one workgroup per fit
__global__ __launch_bounds__(256) void trial_reduce_group_kernel(TrialReduceGroup G) {
    const TrialReduceArgs &a = G.a[blockIdx.x];
    trial_reduce_body(a.block_part, a.nblk, a.part_red, a.nred, a.out, a.seq_out, a.seq, a.rule, a.decision);
}

hipError_t launch_trial_reduce_group(const TrialReduceGroup &G, hipStream_t st) {
    if (G.nfit < 1 || G.nfit > kGroupMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(trial_reduce_group_kernel, dim3(G.nfit), dim3(256), 0, st, G);
    return hipGetLastError();
}

hipError_t launch_trial_reduce(const Geometry &g, const double *block_part, const double *part_red, double *out,
                               unsigned long long *seq_out, unsigned long long seq, const TrialRule &rule,
                               double *decision, hipStream_t st) {
    hipLaunchKernelGGL(trial_reduce_kernel, dim3(1), dim3(256), 0, st, block_part, g.Nr / 16, part_red, g.grid(),
                       out, seq_out, seq, rule, decision);
    return hipGetLastError();
}

}  // namespace cr
