// Host side of libcr: argument checks, device state of one fit (cr_solver), the P-APG driver
// loop with its FISTA scalar schedule and stopping tests, and the one-call cr_fit entry
// points.  Every step of the numerical path runs in the kernels of cr_kernels.hip.

#include "cr_internal.h"

#include <dlfcn.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

using namespace cr;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

LamRep rep_of(int precision) {
    return precision == CR_FP64 ? REP_F64 : (precision == CR_MIXED_FP32 ? REP_SPLIT_F32 : REP_SPLIT_BF16);
}

// bytes of the multiplier state per (padded) pair
size_t state_bytes_per_pair(LamRep r, bool adaptive) {
    // FP64 adaptive (storing trial pass): two iterates + two stored candidates; the split forms
    // re-form the accepted candidate instead of storing it
    if (r == REP_F64) return adaptive ? 32 : 16;
    return 8 + (r == REP_SPLIT_F32 ? 4 : 2);
}

bool all_finite(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Phase ranges for profilers (roctx): "cr_fit", "preprocess", "iterate", "stopping_test",
// "certificate".  The roctx library is looked up at run time (libroctx64, or the rocprofiler-sdk
// one); without it the ranges cost nothing.  rocprofv3 --marker-trace records them.
struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};
const Roctx &roctx() {
    static Roctx r;
    static std::once_flag once;
    std::call_once(once, [] {
        for (const char *lib : {"librocprofiler-sdk-roctx.so.1", "libroctx64.so.4", "libroctx64.so"}) {
            void *h = dlopen(lib, RTLD_NOW | RTLD_LOCAL | RTLD_NOLOAD);
            if (!h) h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            auto push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
            auto pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
            if (push && pop) { r.push = push; r.pop = pop; break; }
        }
    });
    return r;
}
struct Range {
    explicit Range(const char *name) { if (roctx().push) roctx().push(name); }
    ~Range() { if (roctx().pop) roctx().pop(); }
};

// Per-test trace (environment CR_TRACE): a path receives one JSON line per stopping test
// (appended); any other value prints a line per test to stderr.
FILE *trace_file() {
    static FILE *f = nullptr;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *v = getenv("CR_TRACE");
        if (v && std::strchr(v, '/')) f = std::fopen(v, "a");
    });
    return f;
}
std::mutex trace_mu;

}  // namespace

#define CR_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return fail_hip(e_, #call); \
    } while (0)

static int fail_hip(hipError_t e, const char *what) {
    if (getenv("CR_DEBUG")) fprintf(stderr, "libcr: %s failed: %s\n", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CR_ENOMEM : CR_EDEVICE;
}

extern "C" void cr_default_options(cr_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = CR_FP64;
    opt->check_every = 50;
    opt->max_iters = 2000000;
    opt->time_budget_s = 0.0;
    opt->L = 0.0;
    opt->power_max_iters = 300;
    opt->power_rtol = 0.0;   // automatic: 1e-8 for the constant step, 1e-2 for the adaptive one
    opt->momentum = 1;
    opt->certificate = 1;
    opt->device = 0;
    opt->stream = nullptr;
    opt->stall_checks = 100;
    opt->step_rule = 1;
    opt->upsilon = 2.0;
    opt->restart = 1;
    opt->check_rule = 1;
    opt->center = 1;
    opt->keep_lambda = 0;
    opt->lambda0 = nullptr;
}

extern "C" const char *cr_strerror(int code) {
    switch (code) {
    case CR_OK: return "ok";
    case CR_EINVAL: return "invalid argument";
    case CR_ENOMEM: return "out of device memory or byte budget";
    case CR_ENOCONV: return "iteration or time budget exhausted before the tolerance";
    case CR_ENUMERIC: return "non-finite value in the iterates";
    case CR_EDEVICE: return "HIP device error or no gfx950 device";
    case CR_EAGAIN: return "request still running";
    case CR_ENOTFOUND: return "unknown request id";
    case CR_ECANCELED: return "request dropped: the serving context was destroyed before it ran";
    default: return "unknown error";
    }
}

extern "C" int cr_device_check(int device) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CR_EDEVICE;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return CR_EDEVICE;
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return CR_EDEVICE;
    return CR_OK;
}

// ---------------------------------------------------------------------------------------------
// Solver state
// ---------------------------------------------------------------------------------------------

int cr_solver::alloc(void **p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ws) {
        // carve a 256-byte aligned piece of the workspace (counting mode only adds up the sizes)
        const size_t at = (ws->off + 255) & ~(size_t)255;
        if (!ws->counting && (at > ws->size || bytes > ws->size - at)) {
            *p = nullptr;
            return CR_ENOMEM;
        }
        *p = ws->counting ? nullptr : ws->base + at;
        ws->last = static_cast<char *>(*p);
        ws->last_off = ws->off;
        ws->off = at + bytes;
        return CR_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? CR_ENOMEM : CR_EDEVICE;
    }
    owned.push_back(*p);
    return CR_OK;
}

void cr_solver::release(void *p) {
    if (!p) return;
    if (ws) {
        // only the latest carve can be given back (temporary staging); anything else stays
        if (p == ws->last) {
            ws->off = ws->last_off;
            ws->last = nullptr;
        }
        return;
    }
    for (size_t k = 0; k < owned.size(); ++k)
        if (owned[k] == p) {
            (void)hipFree(p);
            owned.erase(owned.begin() + (long)k);
            return;
        }
}

cr_solver::~cr_solver() {
    if (device >= 0) (void)hipSetDevice(device);
    if (stream) (void)hipStreamSynchronize(stream);
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
    for (void *p : owned) (void)hipFree(p);
    if (h_scal && h_owned) (void)hipHostFree(h_scal);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

size_t cr_state_bytes(int64_t N, int64_t n, int precision, bool adaptive) {
    Geometry g = make_geometry((int)N, (int)n);
    size_t b = (size_t)g.Nr * g.ld * state_bytes_per_pair(rep_of(precision), adaptive);
    b += (size_t)g.chunks * g.Nr * g.NP * 8 * (adaptive ? 2 : 1) + (size_t)g.strips * g.ld * 12 * (adaptive ? 2 : 1);
    b += (size_t)g.Nr * g.NP * 8 * (adaptive ? 12 : 6) + (size_t)g.Nr * 8 * 24;
    return b;
}

static int validate(int64_t N, int64_t n, double delta, const cr_options *opt) {
    if (N < 1 || n < 1 || !(delta > 0.0) || !std::isfinite(delta)) return CR_EINVAL;
    if (n + 1 > 16 * kMaxMB) return CR_EINVAL;
    if (N > 200000) return CR_EINVAL;
    if (opt) {
        if (opt->precision < CR_FP64 || opt->precision > CR_MIXED_BF16) return CR_EINVAL;
        if (opt->check_every < 1 || opt->max_iters < 0 || opt->power_max_iters < 1) return CR_EINVAL;
        if (opt->L < 0.0 || !std::isfinite(opt->L) || opt->time_budget_s < 0.0) return CR_EINVAL;
        if (!(opt->power_rtol >= 0.0) || !std::isfinite(opt->power_rtol)) return CR_EINVAL;
        if (opt->step_rule < 0 || opt->step_rule > 1) return CR_EINVAL;
        if (opt->step_rule == 1 && !(opt->upsilon > 1.0 && std::isfinite(opt->upsilon))) return CR_EINVAL;
        if (opt->restart < 0 || opt->restart > 1) return CR_EINVAL;
        if (opt->stop_rule < 0 || opt->stop_rule > 1) return CR_EINVAL;
        if (opt->check_rule < 0 || opt->check_rule > 1) return CR_EINVAL;
        if (opt->reform_fp64 < 0 || opt->reform_fp64 > 1) return CR_EINVAL;
        if (opt->center < 0 || opt->center > 1 || opt->keep_lambda < 0 || opt->keep_lambda > 1) return CR_EINVAL;
        // K-block partial dualization: FP64, constant step, blocks of at most kMaxBlock points and
        // at least two blocks
        if (opt->block_size < 0 || opt->block_size > kMaxBlock) return CR_EINVAL;
        if (opt->block_size > 1 &&
            (opt->precision != CR_FP64 || opt->step_rule != 0 || N <= opt->block_size)) return CR_EINVAL;
    }
    return CR_OK;
}

// Every device buffer of a fit, in one list (so that a workspace can be sized by running it in
// counting mode).  Needs g, rep, adaptive and fp32pass set.
int cr_solver::allocate_state(int64_t N, int64_t n) {
    const size_t nr = g.Nr, np = g.NP, rows_np = nr * np;
    const size_t pairs_p = nr * g.ld;
    const size_t lamsz = pairs_p * (rep == REP_F64 ? 8 : 4);
#define CR_ALLOC(ptr, bytes) do { int r_ = alloc((void **)&(ptr), (bytes)); if (r_) return r_; } while (0)
    CR_ALLOC(lam[0], lamsz);
    CR_ALLOC(lam[1], lamsz);
    if (rep == REP_F64 && fp64_buffers() == 4) {
        CR_ALLOC(lam[2], lamsz);
        CR_ALLOC(lam[3], lamsz);
    }
    if (rep != REP_F64) {
        CR_ALLOC(lam_hi, pairs_p * (rep == REP_SPLIT_F32 ? 4 : 2));
        CR_ALLOC(ubase, nr * 8);
        CR_ALLOC(wbase, rows_np * 8);
    }
    CR_ALLOC(xhat64, rows_np * 8);
    CR_ALLOC(ybar64, nr * 8);
    CR_ALLOC(y64, nr * 8);
    CR_ALLOC(xi64, rows_np * 8);
    CR_ALLOC(dmy64, nr * 8);
    CR_ALLOC(yc, nr * 8);
    CR_ALLOC(xic, rows_np * 8);
    CR_ALLOC(dmyc, nr * 8);
    CR_ALLOC(yr, nr * 8);
    CR_ALLOC(xir, rows_np * 8);
    CR_ALLOC(dmyr, nr * 8);
    CR_ALLOC(rowred, nr * 2 * 8);
    CR_ALLOC(part_acc, (size_t)g.chunks * rows_np * 8);
    CR_ALLOC(part_col, (size_t)g.strips * g.ld * 8);
    CR_ALLOC(part_red, (size_t)g.grid() * kRed * 8);
    CR_ALLOC(part_min, (size_t)g.strips * g.ld * 8);
    CR_ALLOC(part_arg, (size_t)g.strips * g.ld * 4);
    CR_ALLOC(scal, 32 * 8);
    CR_ALLOC(cpot[0], nr * 8);
    CR_ALLOC(cpot[1], nr * 8);
    CR_ALLOC(changed, (size_t)((g.Nr + 255) / 256) * 8);
    if (adaptive) {
        CR_ALLOC(part_acc2, (size_t)g.chunks * rows_np * 8);
        CR_ALLOC(part_col2, (size_t)g.strips * g.ld * 8);
        CR_ALLOC(block_part, (size_t)(g.Nr / 16) * 4 * 8);
        CR_ALLOC(decision, 4 * 8);
        CR_ALLOC(trial_out, 16 * 8);
        for (int q = 0; q < 2; ++q) {
            CR_ALLOC(uD[q], nr * 8);
            CR_ALLOC(wD[q], rows_np * 8);
            CR_ALLOC(ye[q], nr * 8);
            CR_ALLOC(xie[q], rows_np * 8);
            CR_ALLOC(dmye[q], nr * 8);
        }
    }
    if (fp32pass) {
        CR_ALLOC(xhat32, rows_np * 4);
        CR_ALLOC(y32, nr * 4);
        CR_ALLOC(xi32, rows_np * 4);
        CR_ALLOC(dmy32, nr * 4);
    }
    if (deferred()) {
        CR_ALLOC(yo64, nr * 8);
        CR_ALLOC(xio64, rows_np * 8);
        CR_ALLOC(dmyo64, nr * 8);
        if (fp32pass) {
            CR_ALLOC(yo32, nr * 4);
            CR_ALLOC(xio32, rows_np * 4);
            CR_ALLOC(dmyo32, nr * 4);
        }
    }
    if (blk > 1) {
        const size_t nblk = (size_t)(N + blk - 1) / blk;
        CR_ALLOC(blk_ws, nblk * block_ws_doubles(blk, (int)n) * 8);
        CR_ALLOC(blk_iters, nblk * 4);
        // no Step 1 yet (a workspace is cleared by a fill kernel at the start of each fit instead)
        if (!ws && hipMemset(blk_iters, 0, nblk * 4) != hipSuccess) return CR_EDEVICE;
    }
    CR_ALLOC(in_x, (size_t)N * n * 8);
    CR_ALLOC(in_y, (size_t)N * 8);
    CR_ALLOC(in_mu, (size_t)n * 8);
#undef CR_ALLOC
    return CR_OK;
}

namespace {
// Tiling and representation of a new solver (no device work).
void configure(cr_solver *s, int64_t N, int64_t n, const cr_options &opt) {
    s->device = opt.device;
    s->opt = opt;
    // workgroups resident at once: one per compute unit at the pass kernel's occupancy
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, opt.device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    s->g = make_geometry((int)N, (int)n, cus);
    s->precision = opt.precision;
    s->rep = rep_of(opt.precision);
    s->adaptive = opt.step_rule == 1;
    s->upsilon = opt.upsilon;
    s->fp32pass = opt.precision != CR_FP64;
    s->blk = opt.block_size > 1 ? opt.block_size : 0;
}
}  // namespace

size_t cr_workspace_bytes(int64_t N, int64_t n, const cr_options *opt_in, int device, bool promotion) {
    cr_options opt;
    if (opt_in) opt = *opt_in; else cr_default_options(&opt);
    opt.device = device;
    if (validate(N, n, 1.0, &opt) != CR_OK || N < 2) return 0;
    cr_solver probe;
    configure(&probe, N, n, opt);
    cr_workspace count;
    count.counting = true;
    probe.ws = &count;
    if (probe.allocate_state(N, n) != CR_OK) return 0;
    probe.ws = nullptr;
    probe.device = -1;
    const size_t state = (count.off + 255) & ~(size_t)255;
    size_t b = state;
    if (promotion && probe.rep != REP_F64)
        b += probe.fp64_buffers() * (((size_t)probe.g.Nr * probe.g.ld * 8 + 255) & ~(size_t)255);
    // a warm start is staged as a dense N x N FP64 matrix right behind the state, before anything
    // else is carved (it fits in the promotion room when there is one)
    if (opt.lambda0) b = std::max(b, state + (size_t)N * N * 8);
    return b;
}

// x, ybar: pointers of kind `on_device` (true: device memory on opt.device).
int cr_solver_create_impl(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                          const cr_options *opt_in, const double *lambda0, bool on_device, cr_solver **out,
                          cr_workspace *ws, double *pinned_scal) {
    if (!out || !x || !ybar) return CR_EINVAL;
    *out = nullptr;
    cr_options opt;
    if (opt_in) opt = *opt_in; else cr_default_options(&opt);
    int rc = validate(N, n, delta, &opt);
    if (rc) return rc;
    if (cr_device_check(opt.device) != CR_OK) return CR_EDEVICE;
    CR_HIP(hipSetDevice(opt.device));

    // host copies for validation and the centring shift
    std::vector<double> hx((size_t)N * n), hy((size_t)N);
    if (on_device) {
        CR_HIP(hipMemcpy(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost));
        CR_HIP(hipMemcpy(hy.data(), ybar, hy.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(hx.data(), x, hx.size() * 8);
        std::memcpy(hy.data(), ybar, hy.size() * 8);
    }
    if (!all_finite(hx.data(), hx.size()) || !all_finite(hy.data(), hy.size())) return CR_EINVAL;

    cr_solver *s = new cr_solver();
    configure(s, N, n, opt);
    s->delta = delta;
    double ymin = hy[0], ymax = hy[0];
    for (double v : hy) { ymin = std::min(ymin, v); ymax = std::max(ymax, v); }
    s->scale = std::max(1.0, ymax - ymin);
    s->yrange = ymax - ymin;
    if (!lambda0) lambda0 = opt.lambda0;
    s->lam_zero = (lambda0 == nullptr);

    auto bail = [&](int code) { delete s; return code; };
    if (opt.stream || ws) {
        // a workspace fit creates no stream: it runs on the caller's (possibly the null stream)
        s->stream = static_cast<hipStream_t>(opt.stream);
        s->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return bail(CR_EDEVICE);
        s->own_stream = true;
    }
    if (pinned_scal) {
        s->h_scal = pinned_scal;
        s->h_pinned = true;
    } else if (ws) {
        s->h_scal = s->h_local;
        s->h_pinned = false;
    } else {
        if (hipHostMalloc((void **)&s->h_scal, 32 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return bail(CR_ENOMEM);
        s->h_pinned = true;
        s->h_owned = true;
    }
    std::memset(s->h_scal, 0, 32 * sizeof(double));
    if (!ws) {
        if (hipEventCreate(&s->ev_a) != hipSuccess || hipEventCreate(&s->ev_b) != hipSuccess) return bail(CR_EDEVICE);
        // a state larger than the free device memory is refused before any O(N^2) allocation
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && cr_state_bytes(N, n, opt.precision, s->adaptive) > fr)
            return bail(CR_ENOMEM);
    } else {
        ws->off = 0;
        ws->counting = false;
        s->ws = ws;
    }
    rc = s->allocate_state(N, n);
    if (rc) return bail(rc);

    const Geometry &g = s->g;
    const size_t nr = g.Nr, np = g.NP, rows_np = nr * np;
    const size_t pairs_p = nr * g.ld;
    const size_t lamsz = pairs_p * (s->rep == REP_F64 ? 8 : 4);

    // Mixed modes work in the frame x - mean(x): every constraint and the adjoint depend only
    // on differences x_i - x_j, so (y, xi, lam) are unchanged while the float residual loses
    // less to cancellation.  The FP64 mode keeps the caller's coordinates.
    std::vector<double> mu((size_t)n, 0.0);
    for (int64_t i = 0; i < N; ++i)
        for (int64_t m = 0; m < n; ++m) mu[m] += hx[(size_t)i * n + m];
    for (int64_t m = 0; m < n; ++m) mu[m] /= (double)N;
    // spread of the centred locations: the rounding scale of the certificate's tie test
    s->xspan = 0.0;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t m = 0; m < n; ++m) s->xspan = std::max(s->xspan, std::fabs(hx[(size_t)i * n + m] - mu[m]));
    // the FP64 mode keeps the caller's frame, and so do the mixed modes with opt.center = 0
    if (!s->fp32pass || !opt.center) std::fill(mu.begin(), mu.end(), 0.0);
    {
        // the FP16 residual's location scale: a power of two taking max |Xhat| (the stored
        // locations and the ones column) into [0.5, 1)
        double xm = 1.0;
        for (int64_t i = 0; i < N; ++i)
            for (int64_t m = 0; m < n; ++m) xm = std::max(xm, std::fabs((double)(float)(hx[(size_t)i * n + m] - mu[m])));
        int e = 0;
        (void)std::frexp(xm, &e);
        s->xscale = (float)std::ldexp(1.0, -std::min(40, std::max(-40, e)));
    }
    int rc2 = CR_OK;
    auto H = [&](hipError_t e) { if (e != hipSuccess && rc2 == CR_OK) rc2 = fail_hip(e, "setup"); };
    // a workspace keeps whatever the previous fit left there: clear all of it first
    if (ws) H(launch_fill_zero(ws->base, ws->off, s->stream));
    H(hipMemcpyAsync(s->in_x, hx.data(), hx.size() * 8, hipMemcpyHostToDevice, s->stream));
    H(hipMemcpyAsync(s->in_y, hy.data(), hy.size() * 8, hipMemcpyHostToDevice, s->stream));
    H(hipMemcpyAsync(s->in_mu, mu.data(), mu.size() * 8, hipMemcpyHostToDevice, s->stream));
    H(launch_prepare(g, s->in_x, s->in_y, s->fp32pass ? s->in_mu : nullptr, s->xhat64, s->xhat32, s->ybar64,
                     s->stream));
    // multipliers: lam^0 in both buffers (lam^{-1} := lam^0 makes the first extrapolation exact)
    if (lambda0) {
        double *dl = nullptr;
        int r = s->alloc((void **)&dl, (size_t)N * N * 8);
        if (r) return bail(r);
        std::vector<double> hl((size_t)N * N);
        if (on_device) H(hipMemcpy(hl.data(), lambda0, hl.size() * 8, hipMemcpyDeviceToHost));
        else std::memcpy(hl.data(), lambda0, hl.size() * 8);
        for (int64_t i = 0; i < N; ++i) hl[(size_t)i * N + i] = 0.0;
        // K-block partial dualization: only the pairs between blocks carry multipliers; the
        // entries inside a block are not variables (Step 1 recomputes the blocks' own)
        if (s->blk > 1)
            for (int64_t i = 0; i < N; ++i)
                for (int64_t j = 0; j < N; ++j)
                    if (i / s->blk == j / s->blk) hl[(size_t)i * N + j] = 0.0;
        for (double v : hl)
            if (!std::isfinite(v) || v < 0.0) { H(hipStreamSynchronize(s->stream)); return bail(CR_EINVAL); }
        H(hipMemcpyAsync(dl, hl.data(), hl.size() * 8, hipMemcpyHostToDevice, s->stream));
        H(launch_pack_lambda(g, dl, s->rep, s->rep == REP_F64 ? s->lam[0] : s->lam_hi, (float *)s->lam[0], s->stream));
        H(hipMemcpyAsync(s->lam[1], s->lam[0], lamsz, hipMemcpyDeviceToDevice, s->stream));
        H(hipStreamSynchronize(s->stream));
        s->release(dl);
    } else if (!ws) {
        H(launch_fill_zero(s->lam[0], lamsz, s->stream));
        H(launch_fill_zero(s->lam[1], lamsz, s->stream));
        if (s->lam_hi) H(launch_fill_zero(s->lam_hi, pairs_p * (s->rep == REP_SPLIT_F32 ? 4 : 2), s->stream));
    }
    if (!ws) {
        if (s->ubase) {
            H(launch_fill_zero(s->ubase, nr * 8, s->stream));
            H(launch_fill_zero(s->wbase, rows_np * 8, s->stream));
        }
        H(launch_fill_zero(s->part_acc, (size_t)g.chunks * rows_np * 8, s->stream));
        H(launch_fill_zero(s->part_col, (size_t)g.strips * g.ld * 8, s->stream));
        if (s->adaptive) {
            H(launch_fill_zero(s->part_acc2, (size_t)g.chunks * rows_np * 8, s->stream));
            H(launch_fill_zero(s->part_col2, (size_t)g.strips * g.ld * 8, s->stream));
        }
    }
    H(hipStreamSynchronize(s->stream));
    s->release(s->in_x);
    s->release(s->in_y);
    s->release(s->in_mu);
    if (rc2) return bail(rc2);
    *out = s;
    return CR_OK;
}

extern "C" int cr_solver_create(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                                const cr_options *opt, const double *lambda0, cr_solver **out) {
    return cr_solver_create_impl(N, n, x, ybar, delta, opt, lambda0, false, out);
}

extern "C" int cr_solver_destroy(cr_solver *s) {
    delete s;
    return CR_OK;
}

// ---- passes ---------------------------------------------------------------------------------

// FP64 adjoint of the stored iterate `idx` -> primal arrays (y, xi, dmy) and optional copies.
int cr_solver::adjoint_to(int idx, double *y, double *xi, double *dmy, bool with_rowred, float *y32_, float *xi32_,
                          float *dmy32_) {
    PassArgs a{};
    a.rev = next_sweep();
    a.x_scale = xscale;
    a.lam_h = lam_hi;
    a.lam_a = lam[idx];
    a.xhat = xhat64;
    a.part_acc = part_acc;
    a.part_col = part_col;
    a.blk = blk;   // under a partition: the dualized multipliers only (the blocks' own are ignored)
    CR_HIP(launch_pass(g, PASS_ADJ, false, rep, a, stream));
    FinalizeArgs f{};
    f.part_acc = part_acc;
    f.part_col = part_col;
    f.xf = xhat64;
    f.ybar = ybar64;
    f.y = y; f.xi = xi; f.dmy = dmy;
    f.y32 = y32_; f.xi32 = xi32_; f.dmy32 = dmy32_;
    f.rowred = with_rowred ? rowred : nullptr;
    f.inv_delta = 1.0 / delta;
    f.power = 0;
    CR_HIP(launch_finalize(g, false, f, stream));
    return CR_OK;
}

// Split representations: fold lam^k's low part into the shared high part (H <- round(H + l_k)),
// re-express both low parts against it and, in the same pass, form an FP64 adjoint: of H for
// the constant step (cached for its next steps), of lam^k itself for the adaptive one (its
// eta(lam^k), with the row terms of the stopping report, lands in yc / xic / dmyc).
// Returns with eta_in_yc telling which.
int cr_solver::rebase(bool *eta_in_yc) {
    if (eta_in_yc) *eta_in_yc = false;
    int rc = materialize();
    if (rc) return rc;
    if (rep == REP_F64) return CR_OK;
    PassArgs a{};
    a.rev = next_sweep();
    a.x_scale = xscale;
    a.lam_h = lam_hi;
    a.lam_a = lam[cur];
    a.lam_b = lam[prv];
    a.xhat = xhat64;
    a.part_acc = part_acc;
    a.part_col = part_col;
    a.rebase_lam = adaptive ? 1 : 0;
    CR_HIP(launch_pass(g, PASS_REBASE, false, rep, a, stream));
    FinalizeArgs f{};
    f.part_acc = part_acc;
    f.part_col = part_col;
    f.xf = xhat64;
    f.ybar = ybar64;
    if (adaptive) {
        f.y = yc; f.xi = xic; f.dmy = dmyc;
        f.rowred = rowred;
        f.inv_delta = 1.0 / delta;
        f.power = 0;
    } else {
        f.y = ubase; f.xi = wbase; f.dmy = dmyr;
        f.inv_delta = 1.0;
        f.power = 1;
    }
    CR_HIP(launch_finalize(g, false, f, stream));
    if (eta_in_yc) *eta_in_yc = adaptive;
    return CR_OK;
}

// eta^{k+1} for the next step from the current multipliers (used before the first iteration
// and after a change of representation or of the pass arrays).
int cr_solver::prime() {
    int rc = rebase();
    if (rc) return rc;
    if (adaptive) {
        rc = refresh_eta(false);
        if (rc) return rc;
        primed = true;
        return CR_OK;
    }
    // lam~^{k+1} = lam^k + beta_k (lam^k - lam^{k-1}) is linear in the stored iterates, so its
    // adjoint is (1 + beta) C^T lam^k - beta C^T lam^{k-1}; at k = 0 (or beta = 0) only lam^k counts.
    if (k == 0 || beta_last == 0.0) {
        rc = adjoint_to(cur, y64, xi64, dmy64, false, y32, xi32, dmy32);
        if (rc) return rc;
    } else {
        rc = adjoint_to(cur, yc, xic, dmyc, false, nullptr, nullptr, nullptr);
        if (rc) return rc;
        rc = adjoint_to(prv, yr, xir, dmyr, false, nullptr, nullptr, nullptr);
        if (rc) return rc;
        const double b = beta_last;
        CR_HIP(launch_lincomb(g, yc, xic, yr, xir, 1.0 + b, -b, 1.0 + b, -b, xhat64, y64, xi64, dmy64, y32, xi32,
                              dmy32, stream));
    }
    if (blk > 1) {
        // Step 1 under the partition: the closed form of lam~ projected block by block
        rc = project_blocks(y64, xi64, dmy64, false, nullptr);
        if (rc) return rc;
    }
    primed = true;
    return CR_OK;
}

// Adaptive step: recompute eta(lam^k) and eta(lam^{k-1}) exactly in FP64 from the stored
// iterates (the running updates between stopping tests add FP32-accurate increments) and the
// next extrapolated point eta(lam~^{k+1}) from them.  have_cur_in_yc: eta(lam^k) is already in
// yc / xic / dmyc (fresh from a stopping test).
int cr_solver::refresh_eta(bool have_cur_in_yc) {
    if (have_cur_in_yc) {
        // take the test's buffers over instead of copying them; yc / xic / dmyc are then scratch
        // until the next test fills them again, so that test's results are no longer reusable
        std::swap(ye[ecur], yc);
        std::swap(xie[ecur], xic);
        std::swap(dmye[ecur], dmyc);
        test_fresh = false;
    } else {
        int rc = adjoint_to(cur, ye[ecur], xie[ecur], dmye[ecur], false, nullptr, nullptr, nullptr);
        if (rc) return rc;
    }
    int rc = adjoint_to(prv, ye[1 - ecur], xie[1 - ecur], dmye[1 - ecur], false, nullptr, nullptr, nullptr);
    if (rc) return rc;
    const double b = opt.momentum ? beta_last : 0.0;
    CR_HIP(launch_lincomb(g, ye[ecur], xie[ecur], ye[1 - ecur], xie[1 - ecur], 1.0 + b, -b, 1.0 + b, -b, xhat64, y64,
                          xi64, dmy64, fp32pass ? y32 : nullptr, fp32pass ? xi32 : nullptr, fp32pass ? dmy32 : nullptr,
                          stream));
    return CR_OK;
}

// Store the accepted candidate of the last trial (split forms with the adaptive step): one
// constant-step-form pass from lam[cur], lam[prv] with the accepted step and that trial's pass
// arrays writes lam^k over lam[prv].
int cr_solver::materialize() {
    if (!pend) return CR_OK;
    PassArgs a{};
    a.rev = next_sweep();
    a.x_scale = xscale;
    a.lam_h = lam_hi;
    a.lam_a = lam[cur];
    a.lam_b = lam[prv];
    a.beta_prev = pend_beta;
    a.beta_next = 0.0;
    a.inv_L = pend_invs;
    if (fp32pass) {
        a.xhat = xhat32; a.xi = xio32; a.yv = yo32; a.dmy = dmyo32;
    } else {
        a.xhat = xhat64; a.xi = xio64; a.yv = yo64; a.dmy = dmyo64;
    }
    a.part_acc = part_acc;
    a.part_col = part_col;
    CR_HIP(launch_pass(g, PASS_STEP, fp32pass, rep, a, stream));
    std::swap(cur, prv);
    pend = false;
    return CR_OK;
}

// One iteration under the adaptive rule of eq. "eq:adaptive-check" (s_0 = L, s_k = s_{k-1}
// upsilon^(l_k - 1), smallest admissible l_k >= 0).  Each fused trial pass evaluates two consecutive
// candidates l and l + 1 from one read of the iterates.  With every pair dualized the dual function
// is exactly quadratic, so the check for D = lam^k - lam~^k reads
//     ||A1^T D||^2 + ||A2^T D||^2 / delta <= s ||D||^2,
// which the pass provides directly (adjoint of D and ||D||^2) without differencing dual values.
int cr_solver::step_adaptive() {
    test_fresh = false;
    lam_zero = false;
    if (!primed) {
        int rc = prime();
        if (rc) return rc;
    }
    const double bk = opt.momentum ? beta_last : 0.0;   // forms lam~^{k+1} from lam^k, lam^{k-1}
    double sa = s_step / upsilon, sb = s_step;
    int accepted = -1;
    double s_new = s_step;
    bool restart_now = false;
    double beta_dev = 0.0, t_next_dev = 1.0;
    const bool defer = deferred();
    for (int attempt = 0; attempt < 64; ++attempt) {
        // split forms: the first attempt also re-forms and stores the previous accepted iterate
        const bool adv = defer && pend;
        PassArgs a{};
        a.rev = next_sweep();
        a.x_scale = xscale;
        a.lam_h = lam_hi;
        a.lam_a = lam[cur];
        a.lam_b = lam[prv];
        if (!defer) {
            a.lam_c = lam[fa];
            a.lam_d = lam[fb];
        }
        a.beta_prev = bk;
        if (adv) {
            a.beta_prev = pend_beta;
            a.inv_Lo = pend_invs;
            a.beta_next = bk;
            if (fp32pass) { a.xi_o = xio32; a.yv_o = yo32; a.dmy_o = dmyo32; }
            else { a.xi_o = xio64; a.yv_o = yo64; a.dmy_o = dmyo64; }
        }
        a.inv_L = 1.0 / sa;
        a.inv_L2 = 1.0 / sb;
        a.part_acc = part_acc;
        a.part_col = part_col;
        a.part_acc2 = part_acc2;
        a.part_col2 = part_col2;
        a.part_red = part_red;
        if (fp32pass) {
            a.xhat = xhat32; a.xi = xi32; a.yv = y32; a.dmy = dmy32;
        } else {
            a.xhat = xhat64; a.xi = xi64; a.yv = y64; a.dmy = dmy64;
        }
        const PassMode mode = adv ? PASS_ADV : (defer ? PASS_TRIAL_NS : PASS_TRIAL);
        TrialFinalizeArgs f{};
        f.part_acc[0] = part_acc; f.part_acc[1] = part_acc2;
        f.part_col[0] = part_col; f.part_col[1] = part_col2;
        f.xf = xhat64;
        f.uD[0] = uD[0]; f.uD[1] = uD[1];
        f.wD[0] = wD[0]; f.wD[1] = wD[1];
        f.block_part = block_part;
        // h_scal (pinned host memory) receives ||A1^T D_a||^2, ||A2^T D_a||^2, the same for D_b,
        // ||D_a||^2, ||D_b||^2, <D_a, lam_a - lam^k>, <D_b, lam_b - lam^k>, then the decision
        // (candidate or -1 / -2, beta_k, t_{k+1}, restart)
        const unsigned long long seq = ++trial_seq;
        // the reduction takes the step test's decision on the device (both candidates, the
        // restart, t_{k+1} and beta_k, in FP64; the host reads that decision back rather than
        // evaluating the test again), and the accepted step's update is queued right behind it:
        // it reads the decision and does nothing on a retry, so no host round trip sits between
        // the test and the update.  Its outputs go to the pass-array set that becomes current on
        // acceptance (split forms keep this trial's set for re-forming the candidate).
        const TrialRule rule{sa, sb, delta, t, opt.restart ? 1 : 0, opt.momentum ? 1 : 0};
        // without pinned host memory the scalars land in device memory and are copied back below
        TrialReduceArgs red{};
        red.block_part = block_part; red.nblk = g.Nr / 16;
        red.part_red = part_red; red.nred = g.grid();
        red.out = h_pinned ? h_scal : trial_out;
        red.seq_out = h_pinned ? h_seq() : nullptr;
        red.seq = seq;
        red.rule = rule;
        red.decision = decision;
        AcceptArgs upd;
        {
            const int en = 1 - ecur;
            double *yn = defer ? yo64 : y64, *xin = defer ? xio64 : xi64, *dmyn = defer ? dmyo64 : dmy64;
            float *y32n = fp32pass ? (defer ? yo32 : y32) : nullptr;
            float *xi32n = fp32pass ? (defer ? xio32 : xi32) : nullptr;
            float *dmy32n = fp32pass ? (defer ? dmyo32 : dmy32) : nullptr;
            upd = make_accept_args(g, y64, xi64, yn, xin, dmyn, uD, wD, ye[ecur], xie[ecur], ye[en], xie[en],
                                   dmye[en], y32n, xi32n, dmy32n, xhat64, 1.0 / delta, 0.0, decision);
        }
        if (batch && h_pinned) {
            // grouped with the other fits iterating now (serving); ordered behind this stream's
            // work by ev_ready, and this stream's later work behind the round by plan.done
            TrialPlan plan;
            plan.g = g; plan.mode = mode; plan.fp32 = fp32pass; plan.rep = rep;
            plan.pass = a; plan.fin = f; plan.red = red; plan.acc = upd;
            plan.ready = ev_ready;
            CR_HIP(hipEventRecord(ev_ready, stream));
            const int rc = cr_batcher_run(batch, &plan);
            if (rc) return rc;
            CR_HIP(hipStreamWaitEvent(stream, plan.done, 0));
        } else {
            // the timed launches are the dominant kind: re-forming trials (split) or storing
            // trials; one in four is sampled
            const bool timed = ev_a && !ev_pending && (adv || !defer) && (timing_tick++ % 4 == 0);
            if (timed) CR_HIP(hipEventRecord(ev_a, stream));
            CR_HIP(launch_pass(g, mode, fp32pass, rep, a, stream));
            if (timed) {
                CR_HIP(hipEventRecord(ev_b, stream));
                ev_pending = true;
                ev_pending_low = fp32pass;
            }
            CR_HIP(launch_trial_finalize(g, fp32pass, f, stream));
            CR_HIP(launch_trial_reduce(g, block_part, part_red, red.out, red.seq_out, seq, rule, decision, stream));
            CR_HIP(launch_accept_args(g, upd, stream));
        }
        if (adv) {
            // lam^k now sits in lam[prv]: it becomes the current iterate
            std::swap(cur, prv);
            pend = false;
            adv_passes += 1.0;
        }
        if (h_pinned) {
            const int rc = wait_trial(seq);
            if (rc) return rc;
        } else {
            CR_HIP(hipMemcpyAsync(h_scal, trial_out, 12 * sizeof(double), hipMemcpyDeviceToHost, stream));
            CR_HIP(hipStreamSynchronize(stream));
        }
        collect_timing();
        trials += 2.0;
        for (int q = 0; q < 8; ++q)
            if (!std::isfinite(h_scal[q])) return CR_ENUMERIC;
        const double acc = h_scal[8];
        if (acc < -1.5) return CR_ENUMERIC;
        if (acc >= 0.0) {
            accepted = acc > 0.5 ? 1 : 0;
            s_new = accepted ? sb : sa;
            restart_now = h_scal[11] != 0.0;
            beta_dev = h_scal[9];
            t_next_dev = h_scal[10];
            break;
        }
        sa = sb * upsilon;
        sb = sa * upsilon;
    }
    if (accepted < 0) return CR_ENUMERIC;   // no admissible step after 2^128-fold growth
    if (defer) {
        // the accepted candidate is re-formed by the next pass from lam[cur], lam[prv]
        pend = true;
        pend_beta = bk;
        pend_invs = 1.0 / s_new;
    } else {
        const int c = cur, p = prv, A = fa, B = fb;
        if (accepted == 0) { cur = A; prv = c; fa = p; fb = B; }
        else { cur = B; prv = c; fa = A; fb = p; }
    }
    // optional gradient restart: the accepted step points against the iterate's own movement
    // (decided on the device: t_{k+1} and beta_k there already start again from t = 1)
    if (restart_now) restarts += 1.0;
    // the queued update has written eta(lam^{k+1}) = eta(lam~^{k+1}) + (A1^T D, A2^T D / delta)
    // into the slot of eta(lam^{k-1}) and the pass arrays (1 + beta_k) eta(lam^{k+1}) -
    // beta_k eta(lam^k) into the other set, which becomes the current one
    const int en = 1 - ecur;
    if (defer) {
        std::swap(y64, yo64); std::swap(xi64, xio64); std::swap(dmy64, dmyo64);
        std::swap(y32, yo32); std::swap(xi32, xio32); std::swap(dmy32, dmyo32);
    }
    ecur = en;
    t = t_next_dev;
    beta_last = beta_dev;
    s_step = s_new;
    ++k;
    if (fp32pass) ++k_low;
    return CR_OK;
}

// Step 1 under a K-block partition: the closed-form point in (y, xi) projected onto every block's
// pair constraints (eq. "subgradient_split"), in place; with lam_out, the blocks' multipliers go to
// the intra-block entries of that FP64 multiplier array.
int cr_solver::project_blocks(double *y, double *xi, double *dmy, bool with_rowred, double *lam_out) {
    BlockProjArgs b{};
    b.xhat = xhat64;
    b.y = y; b.xi = xi; b.dmy = dmy;
    b.ybar = ybar64;
    b.rowred = with_rowred ? rowred : nullptr;
    b.lam = lam_out;
    b.ld = g.ld;
    b.ws = blk_ws;
    b.ws_doubles = block_ws_doubles(blk, g.n);
    b.iters = blk_iters;
    b.delta = delta;
    b.tol = 1e-11;
    b.N = g.N; b.n = g.n; b.NP = g.NP; b.p = blk;
    b.max_iter = 60;
    b.warm = blk_warm ? 1 : 0;
    CR_HIP(launch_block_project(g, b, stream));
    blk_warm = true;
    return CR_OK;
}

int cr_solver::step_once() {
    test_fresh = false;
    lam_zero = false;
    if (!primed) {
        int rc = prime();
        if (rc) return rc;
    }
    const double t_next = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const double beta_k = opt.momentum ? (t - 1.0) / t_next : 0.0;
    PassArgs a{};
    a.rev = next_sweep();
    a.x_scale = xscale;
    a.lam_h = lam_hi;
    a.lam_a = lam[cur];
    a.lam_b = lam[prv];
    a.beta_prev = opt.momentum ? beta_last : 0.0;
    a.beta_next = beta_k;
    a.inv_L = 1.0 / L;
    a.part_acc = part_acc;
    a.part_col = part_col;
    a.blk = blk;
    if (fp32pass) {
        a.xhat = xhat32; a.xi = xi32; a.yv = y32; a.dmy = dmy32;
    } else {
        a.xhat = xhat64; a.xi = xi64; a.yv = y64; a.dmy = dmy64;
    }
    const bool timed = ev_a && !ev_pending;
    if (timed) CR_HIP(hipEventRecord(ev_a, stream));
    CR_HIP(launch_pass(g, PASS_STEP, fp32pass, rep, a, stream));
    if (timed) {
        CR_HIP(hipEventRecord(ev_b, stream));
        ev_pending = true;
        ev_pending_low = fp32pass;
    }
    FinalizeArgs f{};
    f.part_acc = part_acc;
    f.part_col = part_col;
    f.xf = xhat64;
    f.ybar = ybar64;
    f.y = y64; f.xi = xi64; f.dmy = dmy64;
    f.y32 = fp32pass ? y32 : nullptr;
    f.xi32 = fp32pass ? xi32 : nullptr;
    f.dmy32 = fp32pass ? dmy32 : nullptr;
    f.ubase = ubase;
    f.wbase = wbase;
    f.inv_delta = 1.0 / delta;
    CR_HIP(launch_finalize(g, fp32pass, f, stream));
    if (blk > 1) {
        // Step 1 of the next iteration: the closed form of lam~^{k+1}, projected block by block
        const int rc = project_blocks(y64, xi64, dmy64, false, nullptr);
        if (rc) return rc;
    }
    std::swap(cur, prv);
    t = t_next;
    beta_last = beta_k;
    ++k;
    if (fp32pass) ++k_low;
    return CR_OK;
}

// Waits until the trial reduction has announced sequence number `seq` in pinned memory (a spin on
// the host: the decision is needed at once and the round trip is about half that of a stream
// synchronization).  The stream is queried now and then, so a failed launch ends the wait.
int cr_solver::wait_trial(unsigned long long seq) {
    volatile unsigned long long *w = h_seq();
    for (unsigned long spins = 1; *w != seq; ++spins) {
        if ((spins & 1023) == 0) {
            const hipError_t q = hipStreamQuery(stream);
            if (q == hipSuccess) {
                if (*w == seq) break;
                return fail_hip(hipErrorUnknown, "trial scalars not announced");
            }
            if (q != hipErrorNotReady) return fail_hip(q, "trial reduction");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return CR_OK;
}

// Folds the last sampled launch into the averages once its end event has completed (a sample
// still in flight is kept for a later call).
void cr_solver::collect_timing() {
    if (!ev_pending) return;
    if (hipEventQuery(ev_b) == hipErrorNotReady) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_a, ev_b) == hipSuccess) {
        const int q = ev_pending_low ? 0 : 1;
        step_ms_sum[q] += ms;
        step_n[q] += 1.0;
    }
    ev_pending = false;
}

int cr_solver::lipschitz(double *Lout, double *s2out, int32_t *itout) {
    const Range r("preprocess");
    test_fresh = false;   // the power passes reuse scal and the pass arrays
    const double t0 = now_s();
    CR_HIP(hipSetDevice(device));
    // The constant step 1/L needs L itself; the adaptive rule only starts from s_0 = L and checks
    // every step (an estimate a few percent low costs at most one retry pass at the start).
    const double rtol = opt.power_rtol > 0.0 ? opt.power_rtol : (adaptive ? 1e-2 : 1e-8);
    // Mixed modes run the power passes in FP32 when the tolerance is far above FP32 resolution
    // (the FP64 vector is normalized each step and re-rounded, so errors do not accumulate).
    const bool f32 = fp32pass && rtol >= 1e-6;
    CR_HIP(launch_power_init(g, xhat64, y64, xi64, dmy64, f32 ? y32 : nullptr, f32 ? xi32 : nullptr,
                             f32 ? dmy32 : nullptr, stream));
    double est = 0.0;
    int it = 0;
    for (it = 1; it <= opt.power_max_iters; ++it) {
        PassArgs a{};
        if (f32) {
            a.xhat = xhat32; a.xi = xi32; a.yv = y32; a.dmy = dmy32;
        } else {
            a.xhat = xhat64; a.xi = xi64; a.yv = y64; a.dmy = dmy64;
        }
        a.part_acc = part_acc; a.part_col = part_col; a.part_red = part_red;
        a.blk = blk;   // sigma_max of the dualized rows only
        CR_HIP(launch_pass(g, PASS_POWER, f32, REP_F64, a, stream));
        FinalizeArgs f{};
        f.part_acc = part_acc; f.part_col = part_col; f.xf = xhat64; f.ybar = ybar64;
        f.y = y64; f.xi = xi64; f.dmy = dmy64; f.rowred = rowred; f.inv_delta = 1.0; f.power = 1;
        CR_HIP(launch_finalize(g, f32, f, stream));
        CR_HIP(launch_reduce(part_red, g.grid(), kRed, 0, 1, scal, stream));
        CR_HIP(launch_reduce(rowred, g.Nr, 2, 0, 2, scal + 1, stream));
        CR_HIP(launch_normalize(g, y64, xi64, dmy64, f32 ? y32 : nullptr, f32 ? xi32 : nullptr,
                                f32 ? dmy32 : nullptr, scal + 1, stream));
        CR_HIP(hipMemcpyAsync(h_scal, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, stream));
        CR_HIP(hipStreamSynchronize(stream));
        const double nw = h_scal[0];
        if (!std::isfinite(nw)) return CR_ENUMERIC;
        if (h_scal[1] + h_scal[2] == 0.0) { est = nw; break; }
        const bool done = std::fabs(nw - est) <= rtol * nw;
        est = nw;
        if (done) break;
    }
    if (it > opt.power_max_iters) it = opt.power_max_iters;
    sigma2 = est;
    L = est / delta;
    if (!(L > 0.0)) L = 1.0 / delta;   // every x equal and N = 1: any positive step is exact
    s_step = L;
    power_iters = it;
    preprocess_s = now_s() - t0;
    primed = false;
    if (Lout) *Lout = L;
    if (s2out) *s2out = sigma2;
    if (itout) *itout = it;
    return CR_OK;
}

// FP64 stopping test at lam^k; fills rep (without timing fields).  Leaves eta(lam^k) in yc/xic.
int cr_solver::check(cr_report *rep_out, bool certificate) {
    // the certificate right after a test at the same iterate (the end of a fit) reuses that test's
    // adjoint and KKT reductions
    const bool reuse = certificate && test_fresh && checked_k == k && !pend;
    if (!reuse) {
        bool have_eta = false;
        int rc = rebase(&have_eta);
        if (rc) return rc;
        if (!have_eta) {
            rc = adjoint_to(cur, yc, xic, dmyc, true, nullptr, nullptr, nullptr);
            if (rc) return rc;
        }
        if (blk > 1) {
            // eta(lam^k) under the partition, and the blocks' multipliers into lam^k's intra-block
            // entries: the test then reads the whole problem's multipliers, whose closed form is
            // that projection
            rc = project_blocks(yc, xic, dmyc, true, static_cast<double *>(lam[cur]));
            if (rc) return rc;
        }
        PassArgs a{};
        a.rev = next_sweep();
        a.x_scale = xscale;
        a.lam_h = lam_hi;
        a.lam_a = lam[cur];
        a.xhat = xhat64; a.xi = xic; a.yv = yc; a.dmy = dmyc;
        a.part_red = part_red;
        CR_HIP(launch_pass(g, PASS_KKT, false, this->rep, a, stream));
        CR_HIP(launch_reduce(part_red, g.grid(), kRed, 2, 4, scal, stream));
        CR_HIP(launch_reduce(rowred, g.Nr, 2, 0, 2, scal + 4, stream));
    }
    test_fresh = false;
    int nsc = 6;
    if (certificate) {
        PassArgs r{};
        r.xhat = xhat64; r.xi = xic; r.yv = yc; r.dmy = dmyc;
        r.part_min = part_min; r.part_arg = part_arg;
        CR_HIP(launch_pass(g, PASS_REPAIR, false, REP_F64, r, stream));
        CR_HIP(launch_repair_finish(g, part_min, part_arg, yc, xic, ybar64, yr, xir, rowred, xspan, stream));
        CR_HIP(launch_reduce(rowred, g.Nr, 2, 0, 2, scal + 6, stream));
        // own-slope repair: relaxation rounds for the least height potentials c (the first round
        // reuses the column minima above, offsets 0)
        const int nb = (g.Nr + 255) / 256;
        double *cin = cpot[0], *cout = cpot[1];
        CR_HIP(launch_fill_zero(cin, (size_t)g.Nr * 8, stream));
        own_converged = false;
        own_rounds = 0;
        for (int round = 1; round <= kOwnRounds; ++round) {
            if (round > 1) {
                PassArgs q = r;
                q.row_off = cin;
                CR_HIP(launch_pass(g, PASS_REPAIR, false, REP_F64, q, stream));
            }
            CR_HIP(launch_relax_finish(g, part_min, cin, cout, yc, xic, ybar64, xspan, rowred, changed, stream));
            CR_HIP(launch_reduce(changed, nb, 1, 0, 1, scal + 8, stream));
            CR_HIP(hipMemcpyAsync(h_scal + 8, scal + 8, sizeof(double), hipMemcpyDeviceToHost, stream));
            CR_HIP(hipStreamSynchronize(stream));
            own_rounds = round;
            std::swap(cin, cout);
            if (h_scal[8] == 0.0) { own_converged = true; break; }
        }
        if (own_converged) CR_HIP(launch_reduce(rowred, g.Nr, 2, 0, 1, scal + 8, stream));
        nsc = own_converged ? 9 : 8;
    }
    CR_HIP(hipMemcpyAsync(h_scal, scal, nsc * sizeof(double), hipMemcpyDeviceToHost, stream));
    CR_HIP(hipStreamSynchronize(stream));
    collect_timing();
    const double pairs = (double)g.N * (double)g.N - (double)g.N;
    std::memset(rep_out, 0, sizeof(*rep_out));
    rep_out->precision = precision;
    rep_out->iters = k;
    rep_out->iters_low = k_low;
    rep_out->L = L;
    rep_out->sigma2 = sigma2;
    rep_out->power_iters = power_iters;
    rep_out->preprocess_seconds = preprocess_s;
    rep_out->scale = scale;
    rep_out->nat_res_max = h_scal[0] / scale;
    rep_out->max_viol = h_scal[1] / scale;
    rep_out->infeas_rms = pairs > 0 ? std::sqrt(h_scal[2] / pairs) : 0.0;
    rep_out->comp_sum = h_scal[3];
    rep_out->dual_gap_paper = pairs > 0 ? std::fabs(h_scal[3]) / pairs : 0.0;
    rep_out->primal_obj = 0.5 * h_scal[4] + 0.5 * delta * h_scal[5];
    xi_sq = h_scal[5];
    rep_out->dual_obj = rep_out->primal_obj - rep_out->comp_sum;
    // The returned (y, xi) are the FP64 closed form of lam^k, so stationarity holds to rounding.
    rep_out->stat_y = 0.0;
    rep_out->stat_xi = 0.0;
    rep_out->kkt = std::max(rep_out->nat_res_max, std::max(rep_out->stat_y, rep_out->stat_xi));
    if (certificate) {
        // the smaller of the max-affine repair and (if its relaxation converged) the own-slope one
        rep_out->cert_primal = 0.5 * h_scal[6] + 0.5 * delta * h_scal[7];
        if (own_converged) {
            const double own = 0.5 * h_scal[8] + 0.5 * delta * h_scal[5];
            if (own < rep_out->cert_primal) rep_out->cert_primal = own;
        }
        rep_out->cert_gap = rep_out->cert_primal - rep_out->dual_obj;
        rep_out->y_err_bound = std::sqrt(std::max(0.0, 2.0 * rep_out->cert_gap));
    }
    rep_out->step_samples_low = step_n[0];
    rep_out->step_samples_fp64 = step_n[1];
    rep_out->step_ms_low = step_n[0] > 0 ? step_ms_sum[0] / step_n[0] : 0.0;
    rep_out->step_final = adaptive ? s_step : L;
    rep_out->trials = trials;
    rep_out->restarts = restarts;
    rep_out->adv_passes = adv_passes;
    rep_out->step_ms_fp64 = step_n[1] > 0 ? step_ms_sum[1] / step_n[1] : 0.0;
    bool finite = true;
    for (int q = 0; q < nsc; ++q) finite = finite && std::isfinite(h_scal[q]);
    rep_out->status = finite ? CR_OK : CR_ENUMERIC;
    checked_k = k;
    test_fresh = finite;
    return finite ? CR_OK : CR_ENUMERIC;
}

int cr_solver::promote() {
    test_fresh = false;
    if (rep == REP_F64) return CR_OK;
    const size_t bytes = (size_t)g.Nr * g.ld * 8;
    const int nbuf = fp64_buffers();
    // a workspace promotes only if the FP64 copy fits in what is left of it (checked before any
    // work, so that a refusal leaves the split state untouched)
    if (ws && (((ws->off + 255) & ~(size_t)255) + nbuf * ((bytes + 255) & ~(size_t)255) > ws->size))
        return CR_ENOMEM;
    CR_HIP(hipSetDevice(device));
    int rc0 = materialize();
    if (rc0) return rc0;
    void *nb[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int q = 0; q < nbuf; ++q) {
        int rc = alloc(&nb[q], bytes);
        if (rc) {
            for (int p = 0; p < q; ++p) release(nb[p]);
            return rc;
        }
    }
    CR_HIP(launch_merge(g, rep, lam_hi, (const float *)lam[cur], (double *)nb[0], stream));
    CR_HIP(launch_merge(g, rep, lam_hi, (const float *)lam[prv], (double *)nb[1], stream));
    CR_HIP(hipStreamSynchronize(stream));
    for (int q = 0; q < 4; ++q) release(lam[q]);
    release(lam_hi);
    release(ubase);
    release(wbase);
    for (int q = 0; q < 4; ++q) lam[q] = nb[q];
    cur = 0; prv = 1; fa = 2; fb = 3;
    lam_hi = nullptr;
    ubase = nullptr;
    wbase = nullptr;
    rep = REP_F64;
    fp32pass = false;
    primed = false;   // eta^{k+1} is recomputed in FP64 from the promoted multipliers
    return CR_OK;
}

namespace {
// Counts a fit as iterating for its batcher (if any) while in scope: the batcher's rounds wait
// for the fits that are iterating, not for those in a stopping test.
struct Iterating {
    cr_batcher *b;
    explicit Iterating(cr_batcher *b_) : b(b_) { if (b) cr_batcher_active(b, +1); }
    ~Iterating() { if (b) cr_batcher_active(b, -1); }
};
}  // namespace

int cr_solver::solve(double tol, cr_report *rep_out) {
    const double t0 = now_s();
    CR_HIP(hipSetDevice(device));
    if (!(tol > 0.0)) return CR_EINVAL;
    if (!(L > 0.0)) {
        int rc = lipschitz(nullptr, nullptr, nullptr);
        if (rc) return rc;
    }
    cr_report rep;
    std::memset(&rep, 0, sizeof(rep));
    int status = CR_ENOCONV;
    double best = INFINITY;
    int since_best = 0;
    int checks = 0;
    const int64_t kmax = opt.max_iters;
    const bool trace = getenv("CR_TRACE") != nullptr;
    // iteration 0 check: lam^0 may already be optimal (e.g. constant data)
    const bool by_gap = opt.stop_rule == 1;
    double prev_r = -1.0;        // residual and iteration of the previous test (check_rule 1)
    int64_t prev_k = -1;
    for (;;) {
        // At the zero start every pair has s_ij = ybar_j - ybar_i, so the natural residual is
        // (max ybar - min ybar) / scale: when that exceeds tol the test cannot pass and is skipped.
        if (k == 0 && lam_zero && !by_gap && yrange / scale > tol && kmax > 0) {
            int rc = CR_OK;
            if (adaptive && batch && !primed) {
                rc = prime();   // outside the batcher's rounds: the first step would prime itself
                if (rc) return rc;
            }
            const Iterating it(adaptive ? batch : nullptr);
            const Range r("iterate");
            for (int64_t q = 0; q < std::min<int64_t>(opt.check_every, kmax); ++q) {
                rc = adaptive ? step_adaptive() : step_once();
                if (rc) break;
            }
            if (rc == CR_ENUMERIC) { status = CR_ENUMERIC; break; }
            if (rc) return rc;
            continue;
        }
        int rc;
        {
            const Range r("stopping_test");
            rc = check(&rep, by_gap);
        }
        ++checks;
        if (trace && trace_file()) {
            std::lock_guard<std::mutex> lk(trace_mu);
            fprintf(trace_file(),
                    "{\"fit\": \"%p\", \"N\": %d, \"n\": %d, \"k\": %lld, \"t_s\": %.6f, \"kkt\": %.6e, "
                    "\"max_viol\": %.6e, \"infeas_rms\": %.6e, \"dual_gap_paper\": %.6e, \"comp_sum\": %.9e, "
                    "\"dual_obj\": %.15e, \"primal_obj\": %.15e, \"low_precision\": %d, \"step_over_L\": %.6e, "
                    "\"trial_passes\": %.0f, \"restarts\": %.0f}\n",
                    (void *)this, g.N, g.n, (long long)k, now_s() - t0, rep.kkt, rep.max_viol, rep.infeas_rms,
                    rep.dual_gap_paper, rep.comp_sum, rep.dual_obj, rep.primal_obj, fp32pass ? 1 : 0,
                    adaptive ? s_step / L : 1.0, trials / 2.0, restarts);
            fflush(trace_file());
        } else if (trace)
            fprintf(stderr, "cr trace: k=%lld kkt=%.4e viol=%.4e infeas=%.4e dual=%.12e low=%d s/L=%.3e trials=%.0f "
                    "t=%.3f\n", (long long)k, rep.kkt, rep.max_viol, rep.infeas_rms, rep.dual_obj, fp32pass ? 1 : 0,
                    adaptive ? s_step / L : 1.0, trials, now_s() - t0);
        if (rc == CR_ENUMERIC) { status = CR_ENUMERIC; break; }
        if (rc) return rc;
        if ((by_gap ? rep.cert_gap : rep.kkt) <= tol) { status = CR_OK; break; }
        if (k >= kmax) break;
        if (opt.time_budget_s > 0.0 && now_s() - t0 > opt.time_budget_s) break;
        if (fp32pass) {
            // safety net only: the split representation tracks FP64 to ~1e-9 in y, so a switch
            // happens only after `stall_checks` tests without any new lowest residual (a workspace
            // without room for the FP64 copy keeps the split form)
            if (rep.kkt < best) { best = rep.kkt; since_best = 0; }
            else if (++since_best >= opt.stall_checks) {
                rc = promote();
                if (rc && !(rc == CR_ENOMEM && ws)) return rc;
                best = INFINITY;
                since_best = 0;
            }
        }
        if (adaptive && primed) {
            rc = refresh_eta(true);   // exact FP64 eta(lam^k), eta(lam^{k-1}) after the test
            if (rc) return rc;
        }
        int64_t gap = opt.check_every;
        if (opt.check_rule == 1) {
            // after progress, aim the next test at the iteration where the decay seen between the
            // last two tests would reach tol (clamped to [check_every / 5, check_every])
            const double r = by_gap ? rep.cert_gap : rep.kkt;
            if (prev_r > 0.0 && r > 0.0 && r < prev_r && k > prev_k) {
                const double rate = std::log(prev_r / r) / (double)(k - prev_k);
                const double m = std::ceil(std::log(r / tol) / rate);
                const int64_t lo = std::max<int64_t>(1, opt.check_every / 5);
                gap = m < (double)opt.check_every ? std::max<int64_t>(lo, (int64_t)m) : opt.check_every;
            }
            prev_r = r;
            prev_k = k;
        }
        const int64_t todo = std::min<int64_t>(gap, kmax - k);
        if (adaptive && batch && !primed) {
            rc = prime();
            if (rc) return rc;
        }
        const Iterating it(adaptive && todo > 0 ? batch : nullptr);
        const Range r("iterate");
        for (int64_t q = 0; q < todo; ++q) {
            rc = adaptive ? step_adaptive() : step_once();
            if (rc == CR_ENUMERIC) { status = CR_ENUMERIC; break; }
            if (rc) return rc;
        }
        if (status == CR_ENUMERIC) break;
    }
    if (opt.certificate) {
        const Range r("certificate");
        int rc = check(&rep, true);
        if (rc && rc != CR_ENUMERIC) return rc;
        if (rc == CR_ENUMERIC) status = CR_ENUMERIC;
    }
    rep.checks = checks;
    rep.status = status;
    rep.seconds = now_s() - t0;
    last_report = rep;
    if (rep_out) *rep_out = rep;
    return status;
}

// ---- C entry points on the solver -------------------------------------------------------------

extern "C" int cr_solver_lipschitz(cr_solver *s, double *L, double *sigma2, int32_t *iters) {
    if (!s) return CR_EINVAL;
    return s->lipschitz(L, sigma2, iters);
}

extern "C" int cr_solver_set_delta(cr_solver *s, double delta) {
    if (!s || !(delta > 0.0) || !std::isfinite(delta)) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    int rc = s->materialize();
    if (rc) return rc;
    s->delta = delta;
    s->test_fresh = false;
    s->L = s->sigma2 > 0.0 ? s->sigma2 / delta : 0.0;   // L_gamma = sigma_max(C)^2 / gamma
    s->s_step = s->L;
    s->t = 1.0;                                         // a fresh P-APG run from the current lam
    s->beta_last = 0.0;
    s->primed = false;
    return CR_OK;
}

extern "C" int cr_solver_set_L(cr_solver *s, double L) {
    if (!s || !(L > 0.0) || !std::isfinite(L)) return CR_EINVAL;
    s->L = L;
    s->s_step = L;
    s->sigma2 = 0.0;
    return CR_OK;
}

extern "C" int cr_solver_iterate(cr_solver *s, int64_t iters) {
    if (!s || iters < 0) return CR_EINVAL;
    if (hipSetDevice(s->device) != hipSuccess) return CR_EDEVICE;
    if (!(s->L > 0.0)) {
        int rc = s->lipschitz(nullptr, nullptr, nullptr);
        if (rc) return rc;
    }
    for (int64_t q = 0; q < iters; ++q) {
        int rc = s->adaptive ? s->step_adaptive() : s->step_once();
        if (rc) return rc;
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) return CR_EDEVICE;
    s->collect_timing();
    return CR_OK;
}

extern "C" int cr_solver_solve(cr_solver *s, double tol, cr_report *rep) {
    if (!s) return CR_EINVAL;
    return s->solve(tol, rep);
}

extern "C" int cr_solver_promote(cr_solver *s) {
    if (!s) return CR_EINVAL;
    return s->promote();
}

extern "C" int64_t cr_solver_iterations(const cr_solver *s) { return s ? s->k : -1; }

extern "C" int cr_solver_get_lambda(cr_solver *s, double *lambda) {
    if (!s || !lambda) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    int rc0 = s->materialize();
    if (rc0) return rc0;
    double *d = nullptr;
    const size_t bytes = (size_t)s->g.N * s->g.N * 8;
    int rc = s->alloc((void **)&d, bytes);
    if (rc) return rc;
    CR_HIP(launch_unpack_lambda(s->g, s->rep, s->rep == REP_F64 ? s->lam[s->cur] : s->lam_hi,
                                (const float *)s->lam[s->cur], d, s->stream));
    CR_HIP(hipMemcpyAsync(lambda, d, bytes, hipMemcpyDeviceToHost, s->stream));
    CR_HIP(hipStreamSynchronize(s->stream));
    s->release(d);
    return CR_OK;
}

extern "C" int cr_solver_get_lambda_rows(cr_solver *s, int64_t row0, int64_t nrows, double *rows) {
    if (!s || !rows || row0 < 0 || nrows < 1 || row0 + nrows > s->g.N) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    int rc0 = s->materialize();
    if (rc0) return rc0;
    double *d = nullptr;
    const size_t bytes = (size_t)nrows * s->g.N * 8;
    int rc = s->alloc((void **)&d, bytes);
    if (rc) return rc;
    CR_HIP(launch_unpack_rows(s->g, s->rep, s->rep == REP_F64 ? s->lam[s->cur] : s->lam_hi,
                              (const float *)s->lam[s->cur], (int)row0, (int)nrows, d, s->stream));
    CR_HIP(hipMemcpyAsync(rows, d, bytes, hipMemcpyDeviceToHost, s->stream));
    CR_HIP(hipStreamSynchronize(s->stream));
    s->release(d);
    return CR_OK;
}

// A workspace fit copies lam^k to the host in row blocks staged in its column-partial buffer
// (strips x ld doubles, free once the iterations have ended), so it needs no further device memory.
int cr_solver::lambda_rows_via_scratch(double *lambda) {
    const int64_t N = g.N;
    const int64_t rows = std::max<int64_t>(1, ((int64_t)g.strips * g.ld) / N);
    for (int64_t r0 = 0; r0 < N; r0 += rows) {
        const int nr = (int)std::min<int64_t>(rows, N - r0);
        CR_HIP(launch_unpack_rows(g, rep, rep == REP_F64 ? lam[cur] : lam_hi, (const float *)lam[cur], (int)r0, nr,
                                  static_cast<double *>(part_col), stream));
        CR_HIP(hipMemcpyAsync(lambda + r0 * N, part_col, (size_t)nr * N * 8, hipMemcpyDeviceToHost, stream));
        CR_HIP(hipStreamSynchronize(stream));
    }
    return CR_OK;
}

static int primal_out(cr_solver *s, const double *ysrc, const double *xisrc, double *y, double *xi, bool device_out) {
    const size_t N = s->g.N, n = s->g.n;
    double *dy = nullptr, *dxi = nullptr;
    if (device_out) {
        dy = y; dxi = xi;
    } else if (s->ws) {
        // a workspace fit stages the dense copies in its scratch primal buffers (N <= Nr and
        // N n <= Nr NP), which nothing reads after the fit
        dy = s->yr; dxi = s->xir;
    } else {
        int rc = s->alloc((void **)&dy, N * 8);
        if (rc) return rc;
        rc = s->alloc((void **)&dxi, N * n * 8);
        if (rc) return rc;
    }
    CR_HIP(launch_unpad_primal(s->g, ysrc, xisrc, dy, dxi, s->stream));
    if (!device_out) {
        CR_HIP(hipMemcpyAsync(y, dy, N * 8, hipMemcpyDeviceToHost, s->stream));
        CR_HIP(hipMemcpyAsync(xi, dxi, N * n * 8, hipMemcpyDeviceToHost, s->stream));
    }
    CR_HIP(hipStreamSynchronize(s->stream));
    if (!device_out && !s->ws) {
        s->release(dy);
        s->release(dxi);
    }
    return CR_OK;
}

extern "C" int cr_solver_get_primal(cr_solver *s, double *y, double *xi) {
    if (!s || !y || !xi) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    int rc = s->materialize();
    if (rc) return rc;
    rc = s->adjoint_to(s->cur, s->yc, s->xic, s->dmyc, false, nullptr, nullptr, nullptr);
    if (rc) return rc;
    return primal_out(s, s->yc, s->xic, y, xi, false);
}

extern "C" int cr_solver_block_iters(cr_solver *s, int32_t *iters, int64_t cap, int64_t *nblocks) {
    if (!s || !nblocks) return CR_EINVAL;
    const int64_t nb = s->blk > 1 ? (s->g.N + s->blk - 1) / s->blk : 0;
    *nblocks = nb;
    if (nb == 0 || !iters) return CR_OK;
    if (cap < nb) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    CR_HIP(hipStreamSynchronize(s->stream));
    CR_HIP(hipMemcpy(iters, s->blk_iters, (size_t)nb * 4, hipMemcpyDeviceToHost));
    return CR_OK;
}

extern "C" int cr_solver_report(cr_solver *s, cr_report *rep) {
    if (!s || !rep) return CR_EINVAL;
    CR_HIP(hipSetDevice(s->device));
    int rc = s->check(rep, s->opt.certificate != 0);
    rep->checks = 1;
    return rc;
}

// ---- one-call fits --------------------------------------------------------------------------

static int fit_trivial(int64_t N, int64_t n, const double *ybar, double *y, double *xi, double *lambda, cr_report *rep,
                       bool device_out, const cr_options &opt) {
    // N = 1: no pair constraint; the minimizer is y = ybar, xi = 0.
    (void)N;
    if (device_out) {
        if (hipSetDevice(opt.device) != hipSuccess) return CR_EDEVICE;
        CR_HIP(hipMemcpy(y, ybar, 8, hipMemcpyDeviceToDevice));
        CR_HIP(hipMemset(xi, 0, (size_t)n * 8));
        if (lambda) CR_HIP(hipMemset(lambda, 0, 8));
    } else {
        y[0] = ybar[0];
        for (int64_t m = 0; m < n; ++m) xi[m] = 0.0;
        if (lambda) lambda[0] = 0.0;
    }
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->precision = opt.precision;
        rep->scale = 1.0;
    }
    return CR_OK;
}

int cr_fit_impl(int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
                const cr_options *opt_in, double *y, double *xi, double *lambda, cr_report *rep, bool dev,
                cr_workspace *ws, double *pinned_scal, cr_batcher *batch, hipEvent_t ev_ready) {
    const Range range("cr_fit");
    const double t0 = now_s();
    cr_options opt;
    if (opt_in) opt = *opt_in; else cr_default_options(&opt);
    if (!x || !ybar || !y || !xi) return CR_EINVAL;
    int rc = validate(N, n, delta, &opt);
    if (rc) return rc;
    if (!(tol > 0.0) || !std::isfinite(tol)) return CR_EINVAL;
    if (N == 1) return fit_trivial(N, n, ybar, y, xi, lambda, rep, dev, opt);
    cr_solver *s = nullptr;
    rc = cr_solver_create_impl(N, n, x, ybar, delta, &opt, nullptr, dev, &s, ws, pinned_scal);
    if (rc) return rc;
    if (batch && ev_ready && s->h_pinned) {
        s->batch = batch;
        s->ev_ready = ev_ready;
    }
    if (opt.L > 0.0) { s->L = opt.L; s->s_step = opt.L; }
    cr_report r;
    int status = s->solve(tol, &r);
    if (status != CR_OK && status != CR_ENOCONV && status != CR_ENUMERIC) {
        delete s;
        return status;
    }
    // eta(lam^k) is in yc / xic from the last check
    rc = primal_out(s, s->yc, s->xic, y, xi, dev);
    if (rc) { delete s; return rc; }
    if (lambda) {
        rc = s->materialize();
        if (rc) { delete s; return rc; }
        if (dev) {
            if (launch_unpack_lambda(s->g, s->rep, s->rep == REP_F64 ? s->lam[s->cur] : s->lam_hi,
                                     (const float *)s->lam[s->cur], lambda, s->stream) != hipSuccess ||
                hipStreamSynchronize(s->stream) != hipSuccess) { delete s; return CR_EDEVICE; }
        } else if (ws) {
            rc = s->lambda_rows_via_scratch(lambda);
            if (rc) { delete s; return rc; }
        } else {
            rc = cr_solver_get_lambda(s, lambda);
            if (rc) { delete s; return rc; }
        }
    }
    r.seconds = now_s() - t0;
    if (rep) *rep = r;
    delete s;
    return status;
}

extern "C" int cr_fit_continuation(int64_t N, int64_t n, const double *x, const double *ybar,
                                   const cr_cont_params *cp, const cr_options *opt_in, double *y, double *xi,
                                   double *lambda, cr_cont_step *steps, cr_report *rep) {
    const double t0 = now_s();
    if (!cp || !x || !ybar || !y || !xi) return CR_EINVAL;
    if (!(cp->eps0 > 0.0) || !(cp->beta > 1.0) || !(cp->kappa_gamma > 0.0) || !(cp->kappa_delta > 0.0) ||
        !std::isfinite(cp->eps0 * cp->beta * cp->kappa_gamma * cp->kappa_delta) || cp->T < 1 || cp->T > 200)
        return CR_EINVAL;
    cr_options opt;
    if (opt_in) opt = *opt_in; else cr_default_options(&opt);
    opt.stop_rule = 1;   // delta_t-optimality, certified
    auto gamma_at = [&](int t) { return cp->kappa_gamma * cp->eps0 / std::pow(cp->beta, t); };
    auto delta_at = [&](int t) { return cp->kappa_delta * cp->eps0 / std::pow(cp->beta, t); };
    int rc = validate(N, n, gamma_at(1), &opt);
    if (rc) return rc;
    if (N == 1) {
        rc = fit_trivial(N, n, ybar, y, xi, lambda, rep, false, opt);
        if (steps)
            for (int t = 1; t <= cp->T; ++t) {
                std::memset(&steps[t - 1], 0, sizeof(cr_cont_step));
                steps[t - 1].gamma = gamma_at(t);
                steps[t - 1].delta = delta_at(t);
            }
        return rc;
    }
    cr_solver *s = nullptr;
    rc = cr_solver_create_impl(N, n, x, ybar, gamma_at(1), &opt, nullptr, false, &s);
    if (rc) return rc;
    // sigma_max(C)^2 once (an explicit opt.L is read as L at gamma_1)
    if (opt.L > 0.0) { s->sigma2 = opt.L * gamma_at(1); }
    else {
        rc = s->lipschitz(nullptr, nullptr, nullptr);
        if (rc) { delete s; return rc; }
    }
    int first_bad = CR_OK;
    cr_report r{};
    int64_t total = 0;
    for (int t = 1; t <= cp->T; ++t) {
        const double ts = now_s();
        rc = cr_solver_set_delta(s, gamma_at(t));
        if (rc) { delete s; return rc; }
        const int64_t k0 = s->k;
        const int status = s->solve(delta_at(t), &r);
        if (status != CR_OK && status != CR_ENOCONV && status != CR_ENUMERIC) { delete s; return status; }
        if (status != CR_OK && first_bad == CR_OK) first_bad = status;
        total = s->k;
        if (steps) {
            cr_cont_step &st = steps[t - 1];
            std::memset(&st, 0, sizeof(st));
            st.gamma = gamma_at(t);
            st.delta = delta_at(t);
            st.iters = s->k - k0;
            st.status = status;
            st.cert_gap = r.cert_gap;
            st.kkt = r.kkt;
            st.xi_norm = std::sqrt(std::max(0.0, s->xi_sq));
            st.seconds = now_s() - ts;
        }
        if (status == CR_ENUMERIC) break;
    }
    // (y, xi) of the last check, lambda if asked
    rc = primal_out(s, s->yc, s->xic, y, xi, false);
    if (rc) { delete s; return rc; }
    if (lambda) {
        rc = cr_solver_get_lambda(s, lambda);
        if (rc) { delete s; return rc; }
    }
    r.iters = total;
    r.seconds = now_s() - t0;
    if (rep) *rep = r;
    delete s;
    return first_bad;
}

extern "C" int cr_fit(int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
                      const cr_options *opt, double *y, double *xi, double *lambda, cr_report *rep) {
    return cr_fit_impl(N, n, x, ybar, delta, tol, opt, y, xi, lambda, rep, false);
}

extern "C" int cr_fit_device(int64_t N, int64_t n, const double *x, const double *ybar, double delta, double tol,
                             const cr_options *opt, double *y, double *xi, double *lambda, cr_report *rep) {
    return cr_fit_impl(N, n, x, ybar, delta, tol, opt, y, xi, lambda, rep, true);
}

extern "C" int cr_pass_geometry(int64_t N, int64_t n, int device, int32_t *rows, int32_t *chunks,
                                int32_t *chunk_cols, int32_t *workgroups) {
    if (N < 1 || n < 1 || n + 1 > 16 * kMaxMB || N > 200000) return CR_EINVAL;
    hipDeviceProp_t prop;
    int cus = 256;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    const Geometry g = make_geometry((int)N, (int)n, cus);
    if (rows) *rows = g.Nr;
    if (chunks) *chunks = g.chunks;
    if (chunk_cols) *chunk_cols = g.chunk_cols;
    if (workgroups) *workgroups = g.grid();
    return CR_OK;
}

// ---- operators --------------------------------------------------------------------------------

extern "C" int cr_op_residual(int64_t N, int64_t n, const double *x, const double *y, const double *xi, double *s_out,
                              int device) {
    if (N < 1 || n < 1 || n + 1 > 16 * kMaxMB || !x || !y || !xi || !s_out) return CR_EINVAL;
    cr_options opt;
    cr_default_options(&opt);
    opt.device = device;
    if (cr_device_check(device) != CR_OK) return CR_EDEVICE;
    CR_HIP(hipSetDevice(device));
    // a solver with zero observations gives the padded location array and scratch
    std::vector<double> zy((size_t)N, 0.0);
    std::vector<double> hx((size_t)N * n);
    CR_HIP(hipMemcpy(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost));
    cr_solver *s = nullptr;
    int rc = cr_solver_create_impl(N, n, hx.data(), zy.data(), 1.0, &opt, nullptr, false, &s);
    if (rc) return rc;
    rc = CR_OK;
    do {
        if (launch_pad_primal(s->g, y, xi, s->xhat64, s->yc, s->xic, s->dmyc, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        PassArgs a{};
        a.lam_b = s->lam[0];
        a.xhat = s->xhat64; a.xi = s->xic; a.yv = s->yc; a.dmy = s->dmyc;
        if (launch_pass(s->g, PASS_RESID, false, REP_F64, a, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        if (launch_unpack_lambda(s->g, REP_F64, s->lam[0], nullptr, s_out, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        if (hipStreamSynchronize(s->stream) != hipSuccess) rc = CR_EDEVICE;
    } while (0);
    delete s;
    return rc;
}

extern "C" int cr_op_adjoint(int64_t N, int64_t n, const double *x, const double *lam, double *u, double *w, int device) {
    if (N < 1 || n < 1 || n + 1 > 16 * kMaxMB || !x || !lam || !u || !w) return CR_EINVAL;
    cr_options opt;
    cr_default_options(&opt);
    opt.device = device;
    if (cr_device_check(device) != CR_OK) return CR_EDEVICE;
    CR_HIP(hipSetDevice(device));
    std::vector<double> zy((size_t)N, 0.0);
    std::vector<double> hx((size_t)N * n);
    CR_HIP(hipMemcpy(hx.data(), x, hx.size() * 8, hipMemcpyDeviceToHost));
    cr_solver *s = nullptr;
    int rc = cr_solver_create_impl(N, n, hx.data(), zy.data(), 1.0, &opt, nullptr, false, &s);
    if (rc) return rc;
    rc = CR_OK;
    do {
        if (launch_pack_lambda(s->g, lam, REP_F64, s->lam[0], nullptr, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        PassArgs a{};
        a.lam_a = s->lam[0];
        a.xhat = s->xhat64;
        a.part_acc = s->part_acc;
        a.part_col = s->part_col;
        if (launch_pass(s->g, PASS_ADJ, false, REP_F64, a, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        FinalizeArgs f{};
        f.part_acc = s->part_acc; f.part_col = s->part_col; f.xf = s->xhat64; f.ybar = s->ybar64;
        f.y = s->yc; f.xi = s->xic; f.dmy = s->dmyc; f.inv_delta = 1.0; f.power = 1;
        if (launch_finalize(s->g, false, f, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        if (launch_unpad_primal(s->g, s->yc, s->xic, u, w, s->stream) != hipSuccess) { rc = CR_EDEVICE; break; }
        if (hipStreamSynchronize(s->stream) != hipSuccess) rc = CR_EDEVICE;
    } while (0);
    delete s;
    return rc;
}
