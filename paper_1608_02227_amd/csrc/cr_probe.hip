// Memory probes for the roofline of the pair sweep (a separate library, libcr_probe.so; not part
// of the fit path).  They answer one question: how fast can this device move the bytes the
// re-forming trial pass moves -- three 4-byte multiplier arrays read, the third one written back
// in place -- with and without that pass's access pattern and with no arithmetic to speak of.
//
//   cr_probe_stream   : plain grid-stride streams over n floats per array (16-byte accesses):
//                       kind 0 read only, 1 copy, 2 two reads + one write, 3 three reads with the
//                       third written in place (the pass's mix).
//   cr_probe_pattern  : the pass's own access pattern: the same grid (row strips of 128 rows x
//                       column chunks), waves of 16 rows, lanes holding 8 consecutive columns of one
//                       row, 32-column tiles prefetched two ahead in registers, the third array
//                       written in place; optionally one workgroup barrier per 64 columns as in the
//                       pass, and optionally every other launch walking its columns from the end of
//                       the chunk back to its start (so that a launch begins where the previous one
//                       ended, on the lines the last-level cache still holds).  Arithmetic: one fused
//                       multiply-add and one max per element.
// Both time `iters` launches with HIP events on the given stream and return the average ms.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_kernel(int kind, const f4 *a, const f4 *b, f4 *c, size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += stride) {
        const f4 x = a[e];
        if (kind == 0) {
            acc += x;
        } else if (kind == 1) {
            c[e] = x;
        } else if (kind == 2) {
            c[e] = x + b[e];
        } else {
            const f4 y = b[e], z = c[e];
            c[e] = x + 0.5f * (y - z);
        }
    }
    // read-only stream: keep the loads alive with one store per thread that never happens in
    // practice (the sum of finite inputs is never this value)
    if (kind == 0 && acc.x == 1.2345e-38f) c[0] = acc;
}

constexpr int kRows = 128;   // rows per workgroup: 8 waves of 16
constexpr int kSuper = 64;   // columns per barrier interval

template <bool BARRIER>
__global__ __launch_bounds__(512) void pattern_kernel(const float *H, const float *A, float *B, int ld, int chunks,
                                                      int chunk_cols, int rev) {
    __shared__ float sink[512];
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63, lr = l & 15, lq = l >> 4;
    const int chunk = blockIdx.x % chunks;
    const int strip = blockIdx.x / chunks;
    const int i = strip * kRows + w * 16 + lr;
    const int cbeg = chunk * chunk_cols;
    const int cend = min(ld, cbeg + chunk_cols);
    const size_t rowoff = (size_t)i * ld;
    struct Raw { f4 h[2], a[2], b[2]; };
    auto load = [&](int j0, Raw &t) {
        const size_t e = rowoff + j0;
        t.h[0] = *reinterpret_cast<const f4 *>(H + e); t.h[1] = *reinterpret_cast<const f4 *>(H + e + 4);
        t.a[0] = *reinterpret_cast<const f4 *>(A + e); t.a[1] = *reinterpret_cast<const f4 *>(A + e + 4);
        t.b[0] = *reinterpret_cast<const f4 *>(B + e); t.b[1] = *reinterpret_cast<const f4 *>(B + e + 4);
    };
    Raw pf[2];
    const int ntiles = (cend - cbeg) / 32;
    // column of tile number t in the walking order
    auto col = [&](int t) { return cbeg + (rev ? ntiles - 1 - t : t) * 32 + 8 * lq; };
    if (ntiles > 0) load(col(0), pf[0]);
    if (ntiles > 1) load(col(1), pf[1]);
    float keep = 0.f;
    for (int t = 0; t < ntiles; t += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int j0 = col(t + u);
            Raw cur = pf[u];
            load(t + u + 2 < ntiles ? col(t + u + 2) : j0, pf[u]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                f4 z = cur.a[q] + 0.5f * (cur.a[q] - cur.b[q]);
                z = f4{fmaxf(z.x, -cur.h[q].x), fmaxf(z.y, -cur.h[q].y), fmaxf(z.z, -cur.h[q].z),
                       fmaxf(z.w, -cur.h[q].w)};
                *reinterpret_cast<f4 *>(B + rowoff + j0 + 4 * q) = z;
                keep += z.x;
            }
        }
        if (BARRIER) {
            sink[tid] = keep;
            __syncthreads();
            keep += sink[(tid + 64) & 511] * 0.0f;
        }
    }
    if (keep == 1.2345e-38f) B[rowoff] = keep;
}

}  // namespace

extern "C" int cr_probe_stream(int kind, const void *a, const void *b, void *c, size_t n_floats, int iters,
                               void *stream, float *ms_out) {
    if (kind < 0 || kind > 3 || !a || !c || (kind >= 2 && !b) || n_floats % 4 || iters < 1 || !ms_out) return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n4 = n_floats / 4;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -5;
    const dim3 grid(4096), block(256);
    hipLaunchKernelGGL(stream_kernel, grid, block, 0, st, kind, (const f4 *)a, (const f4 *)b, (f4 *)c, n4);
    (void)hipEventRecord(e0, st);
    for (int it = 0; it < iters; ++it)
        hipLaunchKernelGGL(stream_kernel, grid, block, 0, st, kind, (const f4 *)a, (const f4 *)b, (f4 *)c, n4);
    (void)hipEventRecord(e1, st);
    int rc = hipEventSynchronize(e1) == hipSuccess ? 0 : -5;
    float ms = 0.f;
    if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
    *ms_out = ms / iters;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// rows: padded row count (a multiple of 128, = ld); chunks, chunk_cols: the pass's column split
// (chunk_cols a multiple of 64).  Arrays are rows x ld floats.  flags: bit 0 the per-64-column
// barrier, bit 1 every odd-numbered launch walks its columns backwards.
extern "C" int cr_probe_pattern(const void *H, const void *A, void *B, int rows, int ld, int chunks, int chunk_cols,
                                int flags, int iters, void *stream, float *ms_out) {
    if (!H || !A || !B || rows % kRows || chunk_cols % kSuper || chunks < 1 || iters < 1 || !ms_out ||
        (long)chunks * chunk_cols < ld || ld % kSuper || flags < 0 || flags > 3)
        return -1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -5;
    const dim3 grid((rows / kRows) * chunks), block(512);
    int launch = 0;
    auto go = [&]() {
        const int rev = (flags & 2) ? (launch & 1) : 0;
        ++launch;
        if (flags & 1)
            hipLaunchKernelGGL(pattern_kernel<true>, grid, block, 0, st, (const float *)H, (const float *)A,
                               (float *)B, ld, chunks, chunk_cols, rev);
        else
            hipLaunchKernelGGL(pattern_kernel<false>, grid, block, 0, st, (const float *)H, (const float *)A,
                               (float *)B, ld, chunks, chunk_cols, rev);
    };
    go();
    (void)hipEventRecord(e0, st);
    for (int it = 0; it < iters; ++it) go();
    (void)hipEventRecord(e1, st);
    int rc = hipEventSynchronize(e1) == hipSuccess ? 0 : -5;
    float ms = 0.f;
    if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
    *ms_out = ms / iters;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
