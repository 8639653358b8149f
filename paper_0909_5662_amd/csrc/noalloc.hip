// rot_batch_noalloc: the dense rotation (rot_batch_ex) for callers that
// cannot allocate device memory.  Its workspace is a file-scope device array
// of kScratchBytes; each GPU holds its own copy from the time the library's
// code is loaded on it until the process ends.  The array's device address
// is queried once per device (hipGetSymbolAddress) and cached; host code
// passes only that address on, never the array's name.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "rot_internal.h"

namespace rot {
namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (queried on the first
// call for that device with the device current).
rot_status scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char msg[160];
        snprintf(msg, sizeof msg, "rot_batch_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return set_error(ROT_ERR_HIP, msg);
    }
    if (dev < 0 || dev >= kMaxDevices) return set_error(ROT_ERR_UNSUPPORTED, "rot_batch_noalloc: device index above 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char msg[160];
            snprintf(msg, sizeof msg, "rot_batch_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return set_error(ROT_ERR_HIP, msg);
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ROT_OK;
}

}  // namespace
}  // namespace rot

extern "C" {

size_t rot_noalloc_scratch_bytes(void) { return rot::kScratchBytes; }

rot_status rot_batch_noalloc(const rot_problem* groups, int32_t n_groups, rot_precision prec, uint32_t flags,
                             void* stream) {
    if (flags & ~ROT_ASSUME_SYMMETRIC_O) return rot::set_error(ROT_ERR_INVALID_ARG, "rot_batch_noalloc: unknown flags");
    const size_t need = rot_workspace_size(groups, n_groups, prec, 1, 0);
    // invalid arguments or nothing to rotate: rot_batch_ex reports or returns
    // without touching a workspace
    if (need == 0) return rot_batch_ex(groups, n_groups, prec, flags, nullptr, 0, stream);
    if (need > rot::kScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "rot_batch_noalloc: one operator needs %zu bytes of workspace, above the fixed %zu-byte scratch; "
                 "use rot_batch_ex with a caller workspace",
                 need, rot::kScratchBytes);
        return rot::set_error(ROT_ERR_WORKSPACE, msg);
    }
    void* ws = nullptr;
    const rot_status st = rot::scratch_for_current_device(&ws);
    if (st != ROT_OK) return st;
    return rot_batch_ex(groups, n_groups, prec, flags, ws, rot::kScratchBytes, stream);
}

}  // extern "C"
