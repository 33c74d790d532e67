// ----------------------------------------------------------------------------
// noalloc.hip -- the allocation-free one-shot randomized SVD (psvd_rsvd_noalloc).
//
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc).  All device workspace
// of the call comes from `scratch`, a fixed array in this file that every GPU
// the library runs on holds until the process ends; the host side uses fixed
// host buffers.  Host code never passes `scratch` itself to a kernel or a copy
// (in host code it names a host-side stand-in, not device memory): the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and used instead.
// ----------------------------------------------------------------------------
#include <hip/hip_runtime.h>

#include <mutex>

#include "psvd_internal.h"

namespace {

constexpr size_t kScratchBytes = PSVD_NOALLOC_SCRATCH_BYTES;
constexpr size_t kOmegaEntries = PSVD_NOALLOC_OMEGA_ENTRIES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Host side: the test matrix staging buffer and the status word; one lock
// serialises the calls of this process, so no two calls share the arrays at once.
double g_omega_host[kOmegaEntries];
int32_t g_status_host[16];
std::mutex g_mu;
void* g_scratch_dev[kMaxDevices];   // device address of each GPU's copy of scratch

}  // namespace

extern "C" int psvd_rsvd_noalloc(const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K,
                                 int32_t oversampling, int32_t power_iters, uint64_t seed, int32_t precision, void* U,
                                 int64_t ldu, void* V, int64_t ldv, int32_t out_dtype, double* s, int32_t* rank,
                                 void* stream) {
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return psvd::set_call_error(PSVD_E_DEVICE, "no usable current device");
    if (g_scratch_dev[dev] == nullptr) {
        // first call on this device (the device is current): its copy's address
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return psvd::set_call_error(PSVD_E_DEVICE, "hipGetSymbolAddress of the scratch array failed");
        g_scratch_dev[dev] = ptr;
    }
    psvd::FixedBuffers fb;
    fb.dev = g_scratch_dev[dev];
    fb.dev_bytes = kScratchBytes;
    fb.omega_host = g_omega_host;
    fb.omega_host_entries = kOmegaEntries;
    fb.status_host = g_status_host;
    return psvd::rsvd_fixed(fb, A, M, N, lda, a_dtype, K, oversampling, power_iters, seed, precision, U, ldu, V, ldv,
                            out_dtype, s, rank, stream);
}
