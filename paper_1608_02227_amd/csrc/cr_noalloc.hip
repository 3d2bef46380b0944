// Allocation-free fit: cr_fit_device's work in a fixed, library-owned device scratch array.
//
// For callers that cannot allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc).  Every device buffer of the fit -- the multiplier iterates, the
// partial sums of the pair sweep, the O(N n) primal vectors, the trial scalars -- is carved from
// `scratch`, a file-scope device array of kScratchBytes that each GPU the library runs on holds
// until the process ends.  The call allocates no device or pinned host memory and creates no stream
// or event; its device work runs on the caller's stream (opt->stream, which may be the null stream).

#include "cr_internal.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;   // 128 MiB per device
constexpr int kMaxDevices = 64;

// Host code never uses this name as an address: it only names the symbol for hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu[kMaxDevices];        // one allocation-free fit at a time per device
void *g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (set up once)

}  // namespace

extern "C" size_t cr_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" size_t cr_noalloc_required_bytes(int64_t N, int64_t n, const cr_options *opt) {
    cr_options o;
    if (opt) o = *opt; else cr_default_options(&o);
    return N == 1 ? 0 : cr_workspace_bytes(N, n, &o, o.device);
}

extern "C" int cr_fit_device_noalloc(int64_t N, int64_t n, const double *x, const double *ybar, double delta,
                                     double tol, const cr_options *opt_in, double *y, double *xi, double *lambda,
                                     cr_report *rep) {
    cr_options opt;
    if (opt_in) opt = *opt_in; else cr_default_options(&opt);
    if (opt.device < 0 || opt.device >= kMaxDevices) return CR_EINVAL;
    if (N == 1) return cr_fit_impl(N, n, x, ybar, delta, tol, &opt, y, xi, lambda, rep, true);
    const size_t need = cr_workspace_bytes(N, n, &opt, opt.device);
    if (need == 0) return CR_EINVAL;
    if (need > kScratchBytes) return CR_ENOMEM;
    std::lock_guard<std::mutex> lk(g_mu[opt.device]);
    if (hipSetDevice(opt.device) != hipSuccess) return CR_EDEVICE;
    if (!g_scratch[opt.device]) {
        // once per device, with that device current: the array's address on this device
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return CR_EDEVICE;
        }
        g_scratch[opt.device] = p;
    }
    cr_workspace ws;
    ws.base = static_cast<char *>(g_scratch[opt.device]);
    ws.size = kScratchBytes;
    return cr_fit_impl(N, n, x, ybar, delta, tol, &opt, y, xi, lambda, rep, true, &ws, nullptr);
}
