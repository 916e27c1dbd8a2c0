// gdgs_poisson_solve_static: the Poisson solve of gdgs_poisson_solve with its
// scratch (multigrid hierarchy, norm partials, flags, counters) in a fixed
// device array of this library instead of a caller workspace, for callers
// that cannot allocate device memory at all.
//
// The array below is a device-side symbol: in host code its name is only a
// stand-in, so host code never passes `scratch` itself to a kernel or a copy.
// The device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in g_scratch_ptr;
// the solve carves its workspace out of that address.
#include <mutex>

#include "internal.hpp"

namespace gdgs {
namespace {

static_assert(GDGS_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size must be 256-byte granular");

// Each GPU the library runs on holds one copy until the process ends.
__device__ __align__(256) unsigned char scratch[GDGS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
gdgs_status scratch_of_current_device(void** out) {
    int dev = 0;
    GDGS_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal %d beyond the %d devices this entry point supports", dev,
                  kMaxDevices);
        return GDGS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the static scratch array failed on device %d: %s",
                      dev, hipGetErrorString(e));
            return GDGS_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GDGS_OK;
}

}  // namespace
}  // namespace gdgs

using namespace gdgs;

extern "C" gdgs_status gdgs_poisson_solve_static(const float* grad, const float* boundary,
                                                 int32_t W, int32_t H, const gdgs_mg_params* mg,
                                                 float* u, gdgs_stats* stats_dev, void* stream) {
    GDGS_TRACE("gdgs_poisson_solve_static");
    clear_error();
    auto aligned4 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; };
    if (grad == nullptr || !aligned4(grad) || u == nullptr || !aligned4(u) ||
        (boundary && !aligned4(boundary))) {
        set_error("grad and u must be non-null and 4-byte aligned (boundary too if given)");
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    if (stats_dev && (reinterpret_cast<uintptr_t>(stats_dev) & 7u) != 0) {
        set_error("stats_dev not 8-byte aligned");
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    if (W < 3 || H < 3) {
        set_error("image size %dx%d: both sides must be >= 3", W, H);
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    MgPlan plan;
    const gdgs_status ps = mg_plan(W, H, mg, &plan);
    if (ps != GDGS_OK) return ps;
    if (plan.neumann && boundary) {
        set_error("the Neumann problem takes no boundary data");
        return GDGS_ERR_INVALID_ARGUMENT;
    }
    const size_t need = poisson_ws_bytes(plan, W, H);
    if (need > (size_t)GDGS_STATIC_SCRATCH_BYTES) {
        set_error("a %dx%d solve needs %zu bytes of scratch, more than the %zu bytes of the "
                  "static array (use gdgs_poisson_solve with a workspace)",
                  W, H, need, (size_t)GDGS_STATIC_SCRATCH_BYTES);
        return GDGS_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    const gdgs_status ss = scratch_of_current_device(&ws);
    if (ss != GDGS_OK) return ss;
    // every channel in each launch on the caller's stream, launched directly:
    // no helper streams, events or graphs are created on this path
    return launch_poisson(grad, nullptr, boundary, W, H, plan, u, stats_dev, ws,
                          reinterpret_cast<hipStream_t>(stream), nullptr, false);
}
