// Device scratch of the allocation-free solve (ccg_solve_noalloc): a file-scope
// device array that holds the whole workspace of one FP64 solve, so that the entry
// point needs no device allocation.  Each GPU holds its own copy of the array (at
// its own address) from the first use of the library on it until the process ends.
//
// In host code the array's name is only a stand-in for the symbol: its device
// address is taken once per device, with that device current, by
// hipGetSymbolAddress (scratch_setup, called from ccg_create), and every host use
// of the memory (kernel arguments, the clearing launch) goes through that address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ccg_device.h"

namespace ccg {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

size_t scratch_bytes() { return kScratchBytes; }

// Device address of `scratch` on `device`, which must be the current device.
// Looked up on the first call per device and kept.
hipError_t scratch_setup(int device, void** ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

// Zero `count` 8-byte words at p (a fill kernel: the allocation-free path clears its
// scratch this way rather than with a memset node).
__global__ void k_zero_words(unsigned long long* p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 8;
    if (words == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((words + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, s, static_cast<unsigned long long*>(p), words);
    return hipGetLastError();
}

}  // namespace ccg
