// noalloc.hip -- sgm_aggregate_select_noalloc: the streamlined aggregation
// and selection with its workspace in a fixed device array of this library
// instead of a caller buffer, for callers that cannot allocate device memory.
//
// `scratch` below has one copy per GPU, placed when the GPU first loads this
// code object and held until the process ends.  In host code its name is not
// a device address: the entry point looks the address up once per device with
// hipGetSymbolAddress (that device current) and passes only that pointer on.
// Every call on one GPU shares the array, so calls that overlap on one GPU
// (different streams, or host threads) race; calls in one stream do not.  The
// kernels overwrite or clear everything they read from it (the path kernel
// clears the D^R keys), so no state carries from one call to the next.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sgm.h"

namespace sgm {
int32_t record_hip_error(hipError_t e);   // sgm_capi.cpp
}

namespace {

constexpr size_t kScratchBytes = SGM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_lock;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per GPU

// The address of this GPU's copy of `scratch` (the current device's).
hipError_t scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

}  // namespace

extern "C" int32_t sgm_aggregate_select_noalloc(const uint8_t* cost, int32_t width, int32_t height,
                                                int32_t ndisp, int32_t npaths, int32_t p1, int32_t p2,
                                                int32_t lr_tolerance, int32_t median3x3,
                                                uint16_t* disp_out, uint16_t* disp_right_out,
                                                void* stream) {
    // every check that needs no GPU comes first, so that a rejected call
    // touches no device state
    const size_t need = sgm_aggregate_select_work_bytes(width, height, ndisp, npaths, p2);
    if (need == 0 || !cost || !disp_out || p1 < 0 || p1 > p2) return SGM_ERR_ARG;
    if (median3x3 != 0 && median3x3 != 1) return SGM_ERR_ARG;
    if (need > kScratchBytes) return SGM_ERR_TOO_LARGE;
    if (!aligned(cost, 16) || !aligned(disp_out, 4) ||
        (disp_right_out && !aligned(disp_right_out, 4)))
        return SGM_ERR_ALIGN;
    void* work = nullptr;
    const hipError_t e = scratch_address(&work);
    if (e != hipSuccess) return sgm::record_hip_error(e);
    return sgm_aggregate_select(cost, width, height, ndisp, npaths, p1, p2, lr_tolerance, median3x3,
                                disp_out, disp_right_out, work, kScratchBytes, stream);
}
