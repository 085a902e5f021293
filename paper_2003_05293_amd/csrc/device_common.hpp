// Device helpers shared by the kernel files: address-space views, the
// descriptor search of batched launches and the cross-block hand-off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {
namespace {

__host__ __device__ inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Address-space views of pointers read from the job tables.  Without them
// the compiler sees generic pointers and issues flat loads.  Spot records
// are read-only while a pass reads them (its weight update runs after every
// block of the pass has finished reading), so they are read through the
// constant address space: uniform indices then become scalar loads.
#define HG_CONST __attribute__((address_space(4)))
#define HG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const HG_CONST T* as_const(const T* p) {
  return (const HG_CONST T*)p;
}
template <typename T>
__device__ __forceinline__ const HG_GLOBAL T* as_global(const T* p) {
  return (const HG_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ HG_GLOBAL T* as_global_mut(T* p) {
  return (HG_GLOBAL T*)p;
}

// Index of the descriptor whose block range holds `block` (descriptors are
// sorted by block_begin, the first starts at 0).  Uniform across the block.
template <typename D>
__device__ __forceinline__ int find_desc(const D* __restrict__ d, int n, int block) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].block_begin <= block) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Cross-block hand-off of the pass sums.  The L2 caches of the XCDs are not
// coherent with each other, and an agent-scope fence would write back and
// invalidate the whole L2 of every block's XCD (measured: 4x slower pass).
// Instead the partial sums are written and read with device-scope accesses
// (coherent across XCDs, not left dirty in any L2), each writer waits until
// its own writes have completed before the block's counter increment, and
// the counters are device-scope read-modify-writes.  The block that sees the
// last increment of a group therefore reads every partial of that group.
__device__ __forceinline__ void store_dev(float2* p, float2 v) {
  uint64_t bits;
  __builtin_memcpy(&bits, &v, sizeof(bits));
  __hip_atomic_store(as_global_mut(reinterpret_cast<uint64_t*>(p)), bits, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float2 load_dev(const float2* p) {
  const uint64_t bits = __hip_atomic_load(as_global(reinterpret_cast<const uint64_t*>(p)),
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 v;
  __builtin_memcpy(&v, &bits, sizeof(v));
  return v;
}
__device__ __forceinline__ void store_dev(double2* p, double2 v) {
  HG_GLOBAL double* d = as_global_mut(reinterpret_cast<double*>(p));
  __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 load_dev(const double2* p) {
  const HG_GLOBAL double* d = as_global(reinterpret_cast<const double*>(p));
  return make_double2(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Returns true in the block that made the last of `expected` increments.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned expected, int* flag) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's device-scope writes are complete
  __syncthreads();
  if (threadIdx.x == 0) *flag = atomicAdd(counter, 1u) == expected - 1u;
  __syncthreads();
  return *flag != 0;
}

// Column sums of a row-major [rows][N] float2 array that other blocks wrote
// with device-scope stores: buffer loads with device-scope coherence and a
// 32-bit offset per load, so that
// many loads are in flight per thread at the cost of their data registers
// only.  The resource ends at row_end: the hardware range check returns zero
// for loads past it (the offsets are per-lane offsets, which it checks).
struct ColumnSrc {
  __amdgpu_buffer_rsrc_t rsrc;
  int N, row_end;
};
template <typename T>
__device__ __forceinline__ ColumnSrc column_src(const T* base, int row_end, int N) {
  ColumnSrc c;
  c.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                             (int)((int64_t)row_end * N * sizeof(T)),
                                             0x00020000);
  c.N = N;
  c.row_end = row_end;
  return c;
}
constexpr int kDeviceScope = 1 << 4;  // buffer cache policy: device-scope coherent (sc1)

// Gray level of phase phi (radians) from the SLM's table of L levels, which
// covers one phase period: bin k = floor(L frac(phi / 2 pi)), decided in
// FP32 with individually rounded operations (never fused), clamped to L - 1
// where the fraction rounds up to a whole turn.
__device__ __forceinline__ uint32_t gray_level(float phi, const uint16_t* lut, int L) {
#pragma clang fp contract(off)
  float t = phi * 0.15915494309189535f;
  t = t - floorf(t);
  const int k = (int)(t * (float)L);
  return as_global(lut)[max(0, min(k, L - 1))];  // (a NaN phase lands in bin 0)
}
// Stores a gray level as the image's element type (8 or 16 bits).
__device__ __forceinline__ void store_gray(void* img, int64_t p, int bits, uint32_t g) {
  if (bits == 8) as_global_mut(static_cast<uint8_t*>(img))[p] = (uint8_t)g;
  else as_global_mut(static_cast<uint16_t*>(img))[p] = (uint16_t)g;
}

// Pupil weight of a pixel (paper section 4) with Q = Lx^2 + Ly^2 in doubled
// offsets (Qi exact, Q in FP32): 0 outside the aperture (ap_q >= 0 and
// Qi > ap_q), else the illumination amplitude A = exp(-Q ill_a) (1 when
// ill_a = 0).
__device__ __forceinline__ float pupil_weight(int32_t Qi, float Q, int32_t ap_q, float ill_a) {
  if (ap_q >= 0 && Qi > ap_q) return 0.f;
  return ill_a > 0.f ? expf(-Q * ill_a) : 1.f;
}

}  // namespace
}  // namespace hg
