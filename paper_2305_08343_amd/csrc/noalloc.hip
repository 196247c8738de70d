// Device scratch for sc_trace_noalloc: one file-scope array per GPU, sized
// once, so that a trace can run without any allocation (for callers that may
// not allocate device memory: code under HIP graph capture, tight serving
// loops).
//
// Layout of the array: [0, 256) the ray-queue counters of one launch
// (kQueueParts words, cleared by the launch's own reset kernel), then the
// Morton-sort workspace for up to kNoAllocMaxSortRays rays. Every call on a
// GPU uses that GPU's copy and leaves its contents behind; calls that overlap
// on one GPU race for it.
//
// The array's name is a host-side stand-in in host code. Its device address
// is taken once per device, with that device current, by hipGetSymbolAddress
// (scratch_init, from sc_create), and only that address is used afterwards:
// as a kernel argument and as the base of the counters and the workspace.
#include <mutex>

#include "internal.h"

namespace sc {
namespace {

constexpr size_t kCounterBytes = 256;
constexpr int kMaxDevices = 64;

// the workspace size for kNoAllocMaxSortRays rays, as the sort computes it (checked below)
constexpr size_t kScratchBytes = kCounterBytes + 16 * (size_t)kNoAllocMaxSortRays + 4 * (1024 * 256) + 4 * 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};
hipError_t g_err[kMaxDevices] = {hipSuccess};
bool g_done[kMaxDevices] = {false};

}  // namespace

hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = (e == hipSuccess) ? p : nullptr;
        g_done[device] = true;
    }
    return g_err[device];
}

hipError_t scratch_get(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_done[device]) return hipErrorNotInitialized;
    if (g_err[device] != hipSuccess) return g_err[device];
    *ptr = g_ptr[device];
    *bytes = kScratchBytes;
    return hipSuccess;
}

size_t scratch_counter_bytes() { return kCounterBytes; }

bool scratch_fits_sort(uint32_t n) {
    return n <= kNoAllocMaxSortRays && kCounterBytes + ray_order_workspace_bytes(n) <= kScratchBytes;
}

}  // namespace sc
