// The entry point for callers that cannot allocate device memory: one whole solve whose device state lives in a
// fixed-size array of device memory that the library defines at file scope.  Each GPU holds its own copy of the
// array from module load until the process ends; its address on the current device is looked up once per device.
#include "../../include/dope.h"
#include "dope_internal.h"

#include <mutex>

namespace dope {
dope_status solve_in_buffer(const dope_params *p, void *ws, size_t bytes, const int32_t *u, const int32_t *w,
                            int32_t lambda_q8, uint8_t *labels, dope_info *out);
}

// The device state of dope_solve_noalloc (layout of dope_workspace_bytes).  In host code this name is only a
// handle for the symbol lookup below, never a device address.
static __device__ __align__(256) unsigned char scratch[DOPE_NOALLOC_MAX_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;     // address of this device's copy of scratch
    std::mutex use;          // one solve at a time per device: every call shares the array
};

DeviceScratch g_dev[MAX_DEVICES];

}  // namespace

extern "C" dope_status dope_solve_noalloc(const dope_params *p, const int32_t *u, const int32_t *w,
                                          int32_t lambda_q8, uint8_t *labels, dope_info *out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return DOPE_EDEVICE;
    }
    DeviceScratch &d = g_dev[dev];
    std::call_once(d.once, [&d] {
        void *ptr = nullptr;
        d.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (d.err == hipSuccess) d.ptr = ptr;
        else (void)hipGetLastError();
    });
    if (d.err != hipSuccess || !d.ptr) return DOPE_EDEVICE;
    std::lock_guard<std::mutex> lock(d.use);
    return dope::solve_in_buffer(p, d.ptr, DOPE_NOALLOC_MAX_BYTES, u, w, lambda_q8, labels, out);
}
