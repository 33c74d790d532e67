// psvd_internal.h -- shared device/host definitions of the gfx950 library.
#pragma once

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/psvd.h"

namespace psvd {

// Dynamic-LDS limit of a kernel, raised with hipFuncSetAttribute only when a
// launch needs more than was set before on this device (the attribute call is
// a host API round trip; steady-state launches skip it).
inline hipError_t ensure_lds_attr(const void* fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = done[{dev, fn}];
    if (lds <= cur) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) cur = lds;
    return e;
}


typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef short s4_t __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ----------------------------------------------------------------------------
// Matrix-core (MFMA) tiles, 16 x 16 output per wave.
//   A operand (16 x K): lane l supplies row (l % 16), k = (l / 16) * KPL + v.
//   B operand (K x 16): lane l supplies column (l % 16), same k.
//   Result: lane l holds column (l % 16) and, for v = 0..3, row
//     row_of(l, v) = 4 * (l / 16) + v          (f32 accumulators)
//     row_of(l, v) = (l / 16) + 4 * v          (f64 accumulators)
// (lane layouts checked on gfx950 hardware).
// ----------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Global-memory views of generic pointers.  A pointer rebuilt from integers
// (a column base selected among the blocks of a panel) or passed through a
// generic parameter loses its address space, and loads through it become
// FLAT loads, which also count against the LDS wait counter: every wait for
// an LDS read would then wait for all prefetched tile loads too.  Accesses
// through these views are plain global loads and stores.
// Work-group barrier for LDS hand-offs only: waits for this wave's LDS
// operations (lgkmcnt(0); the vector-memory and export counters are left at
// their maximum), then s_barrier.  __syncthreads() also waits for every
// outstanding global load, which would end the prefetch of the next tile at
// each barrier; the tall-panel kernels exchange data between waves only
// through LDS, so this barrier is enough for them.  The signal fences keep
// the compiler from moving memory operations across it.
__device__ __forceinline__ void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);   // gfx9 encoding: vmcnt 63, expcnt 7, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

#define PSVD_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ f4_t gld4(const float* p) { return *(const PSVD_GLOBAL f4_t*)p; }
__device__ __forceinline__ float gld(const float* p) { return *(const PSVD_GLOBAL float*)p; }
__device__ __forceinline__ double gldd(const double* p) { return *(const PSVD_GLOBAL double*)p; }
__device__ __forceinline__ void gst4(float* p, f4_t v) { *(PSVD_GLOBAL f4_t*)p = v; }
__device__ __forceinline__ void gst(float* p, float v) { *(PSVD_GLOBAL float*)p = v; }
__device__ __forceinline__ void gstd(double* p, double v) { *(PSVD_GLOBAL double*)p = v; }

// Two FP32 values -> two BF16 (round to nearest even) packed low-first, by
// the gfx950 packed conversion instruction.
typedef __bf16 bf2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2_t{lo, hi}, bf2_t));
}

template <class CT>
struct Mfma;

template <>
struct Mfma<double> {
    using elem = double;
    using acc = d4_t;
    using frag = double;
    static constexpr int KPL = 1;
    static constexpr int KSTEP = 4;
    __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row_of(int lane, int v) { return (lane >> 4) + 4 * v; }
    __device__ static __forceinline__ elem from_double(double x) { return x; }
    __device__ static __forceinline__ elem from_float(float x) { return (double)x; }
    __device__ static __forceinline__ elem from_acc(double x) { return x; }
};

template <>
struct Mfma<float> {
    using elem = float;
    using acc = f4_t;
    using frag = float;
    static constexpr int KPL = 1;
    static constexpr int KSTEP = 4;
    __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static __forceinline__ elem from_double(double x) { return (float)x; }
    __device__ static __forceinline__ elem from_float(float x) { return x; }
    __device__ static __forceinline__ elem from_acc(float x) { return x; }
};

template <>
struct Mfma<bf16_t> {
    using elem = uint16_t;
    using acc = f4_t;
    using frag = s4_t;
    static constexpr int KPL = 4;
    static constexpr int KSTEP = 16;
    __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
    __device__ static __forceinline__ elem from_double(double x) { return f32_to_bf16_rne((float)x); }
    __device__ static __forceinline__ elem from_float(float x) { return f32_to_bf16_rne(x); }
    __device__ static __forceinline__ elem from_acc(float x) { return f32_to_bf16_rne(x); }
};

// ----------------------------------------------------------------------------
// Panels: up to three column blocks that share rows, e.g. [U | A] of the
// streaming update, [C | U_bar] of the adjoint, or one partition A_i.
// ----------------------------------------------------------------------------
constexpr int kMaxBlocks = 3;

struct PanelBlock {
    const void* ptr;  // column-major
    int64_t ld;
    int32_t dtype;    // PSVD_F32 / PSVD_F64
    int32_t ncols;
};

struct PanelSeg {
    PanelBlock blk[kMaxBlocks];
    int32_t nblk;
    int32_t ncols;    // sum of blk[].ncols
    int64_t rows;
    void* out;        // output rows of this segment (lift), column-major
    int64_t ldo;
    int32_t out_dtype;
    int32_t pad;
};

struct WorkItem {
    int32_t seg;
    int32_t pad;
    int64_t row0;
    int64_t row1;
};

template <class T>
__device__ __forceinline__ double load_elem(const void* p, int64_t idx, int32_t dtype) {
    return dtype == PSVD_F64 ? ((const double*)p)[idx] : (double)((const float*)p)[idx];
}

// Column c of the panel segment, row i (0 outside the segment's rows).
__device__ __forceinline__ const PanelBlock* block_of(const PanelSeg& s, int c, int* local) {
    int cc = c;
    for (int b = 0; b < s.nblk; ++b) {
        if (cc < s.blk[b].ncols) {
            *local = cc;
            return &s.blk[b];
        }
        cc -= s.blk[b].ncols;
    }
    *local = -1;
    return nullptr;
}

// Status word shared by the kernels of one update.
enum DevStatus : int32_t {
    DEV_OK = 0,
    DEV_FALLBACK = 1,     // Cholesky breakdown handled by the eigen route
    DEV_NONFINITE = 2,
    DEV_NOCONV = 4,
    DEV_BREAKDOWN = 8,
    DEV_SMALL_LAMBDA = 16
};

// Fixed buffers of the allocation-free one-shot randomized SVD: a device
// region (dev_bytes at dev, 256-byte aligned) and host buffers for the test
// matrix and the status word.
struct FixedBuffers {
    void* dev;
    size_t dev_bytes;
    double* omega_host;
    size_t omega_host_entries;
    int32_t* status_host;   // 16 entries
};

// psvd_rsvd on FixedBuffers (psvd_host.hip); the error text goes where
// psvd_last_error(NULL) reads it.
int rsvd_fixed(const FixedBuffers& fb, const void* A, int64_t M, int64_t N, int64_t lda, int32_t a_dtype, int32_t K,
               int32_t oversampling, int32_t power_iters, uint64_t seed, int32_t precision, void* U, int64_t ldu,
               void* V, int64_t ldv, int32_t out_dtype, double* s, int32_t* rank, void* stream);
// Record the text of a failed call without a handle (psvd_last_error(NULL)).
int set_call_error(int code, const char* msg);
// The Gaussian test matrix (n x l, column-major) of call `batch` keyed by seed
// (Philox4x32-10 + Box-Muller), FP64 values (rounding 0), FP32 (1) or BF16 (2).
void host_omega(uint64_t seed, int64_t batch, int64_t n, int64_t l, int rounding, double* out);
// Algorithm 2 (apmos.hip) with the exact SVD of W (ell = 0) or its low-rank SVD
// with the ell-column test matrix of (seed, batch).
int apmos_internal(int32_t P, const void* const* A_parts, const int64_t* M_parts, const int64_t* ld_parts, int64_t N,
                   int32_t dtype, int32_t r, int32_t K, int32_t ell, uint64_t seed, int64_t batch,
                   void* const* U_parts, const int64_t* ldu_parts, double* Lambda, double* X, void* stream);

}  // namespace psvd

