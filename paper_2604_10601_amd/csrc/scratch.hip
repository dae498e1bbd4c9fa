// A fixed device-memory arena for the allocation-free count call
// (gm_count_noalloc): the control block, plan, result block and work stream
// of one query, and the stealing mailboxes and parked task groups of the
// wavefronts of its launch.  It is a file-scope device array, so every GPU the
// library runs on holds its own copy, at its own address, from the moment the
// code object is loaded until the process ends; no call allocates it.
//
// The array's name denotes a host-side stand-in in host code, not a device
// address.  Its device address is looked up once per device, with that device
// current (scratch_area, called from gm_create), and only that address is
// ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gm_internal.h"

namespace gm {

namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t *__restrict__ p, unsigned long long words) {
    for (unsigned long long i = static_cast<unsigned long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<unsigned long long>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

}  // namespace

hipError_t scratch_area(int device, void **out) {
    if (!out) return hipErrorInvalidValue;
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t h = hipGetDevice(&cur);
        if (h != hipSuccess) return h;
        if (cur != device) return hipErrorInvalidDevice;  // the caller makes the device current
        void *p = nullptr;
        h = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (h != hipSuccess) return h;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_zero_words(void *p, unsigned long long words, hipStream_t s) {
    if (words == 0) return hipSuccess;
    unsigned long long blocks = (words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_words_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

}  // namespace gm
