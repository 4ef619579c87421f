// ntd_noalloc.hip -- ntd_dot_noalloc: the FP64 dot product of ntd_dot for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid allocation).  ntd_dot keeps its
// block partial sums and scalars in the handle's workspace; this variant needs
// no handle and keeps them in a fixed static device array instead.
#include <mutex>

#include "ntd.h"
#include "ntd_internal.h"

namespace {

// Partial sums of at most kMaxBlocks blocks, then one Scalars record.
constexpr size_t kScratchDoubles = ntd::kMaxBlocks + sizeof(ntd::Scalars) / sizeof(double);
static_assert(sizeof(ntd::Scalars) % sizeof(double) == 0, "Scalars must pack into doubles");

// One copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel: it uses the device address kept in g_scratch below.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept.
int scratch_on_current_device(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return NTD_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return NTD_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NTD_EHIP;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return NTD_OK;
}

}  // namespace

extern "C" int ntd_dot_noalloc(const double *x, const double *y, long long n, double *result,
                               void *stream) {
    if (!x || !y || !result || n < 0 || n > NTD_DOT_NOALLOC_MAX_N) return NTD_EINVAL;
    double *base = nullptr;
    int st = scratch_on_current_device(&base);
    if (st != NTD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *partials = base;
    ntd::Scalars *sc = reinterpret_cast<ntd::Scalars *>(base + ntd::kMaxBlocks);
    int np = 0;
    // The kernels of ntd_dot: every block writes its partial (grid-stride,
    // at most kMaxBlocks blocks), one block sums them in a fixed order.
    if (ntd::launch_dot(x, y, n, partials, &np, s) != hipSuccess) return NTD_EHIP;
    if (np > ntd::kMaxBlocks) return NTD_EINVAL;
    if (ntd::launch_finalize(partials, np, sc, ntd::kOpResult, s) != hipSuccess) return NTD_EHIP;
    if (hipMemcpyAsync(result, &sc->result, sizeof(double), hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
        return NTD_EHIP;
    return NTD_OK;
}
