// Hand-off of the FP32 passes: the per-block context, the exact fixed-point
// sums of the forward projection (eq. 3) and the weight update of eqs.
// (4)-(6), shared by the per-pixel and the separable kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace hg {
namespace {

// Everything one (virtual) block of a pass needs, uniform across the block.
struct PassCtx {
  SpotRec* sp;
  float2* coef;
  int N, W, H;
  PixelSet ps;
  const float* phi;
  PassPlan plan;
  int lb;  // this block within the pass
  float2* partial;
  double2* gpart;
  unsigned long long* acc;
  unsigned* counters;
  double inv_count;
  double2* V;
  int32_t* status;
  int update, from_phi;
  // pupil: forward terms weighted by the illumination (ill_a > 0), and
  // pixels outside the aperture dropped (ap_q >= 0: the whole-grid set)
  int32_t ap_q = -1;
  float ill_a = 0.f;
  // chained launches: the pass's spot state in LDS, and the generation word
  // to publish after the update
  int chain = 0;
  const SpotRec* recs = nullptr;
  unsigned* gen = nullptr;
  unsigned gen_next = 0;
};

// Device-scope copies of a spot record (read by the other blocks of a
// chained launch after the generation word says it is complete).
__device__ __forceinline__ void store_rec_dev(SpotRec* p, const SpotRec& r) {
  uint64_t w[4];
  __builtin_memcpy(w, &r, sizeof(w));
  HG_GLOBAL uint64_t* q = as_global_mut(reinterpret_cast<uint64_t*>(p));
#pragma unroll
  for (int i = 0; i < 4; ++i) __hip_atomic_store(q + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void load_recs_dev(const SpotRec* sp, int N, SpotRec* recs_lds) {
  const HG_GLOBAL uint64_t* q = as_global(reinterpret_cast<const uint64_t*>(sp));
  uint64_t* d = reinterpret_cast<uint64_t*>(recs_lds);
  for (int k = threadIdx.x; k < 4 * N; k += kBlock)
    d[k] = __hip_atomic_load(q + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exact sums.  Each tile's per-spot partial is rounded once to a 64-bit
// fixed-point integer (scale 2^shift, |sum over the pass| <= pixels, so no
// sum overflows) and added with device-scope integer atomics: integer
// addition is associative, so the sums do not depend on the order in which
// tiles, groups or blocks arrive.  Rows: 0 = pass total, 1 + g = group g.
__device__ __forceinline__ void acc_add(unsigned long long* acc, int N, int shift, int row, int n,
                                        float2 v) {
  const double scale = ldexp(1.0, shift);
  unsigned long long* p = acc + ((int64_t)row * N + n) * kAccSpotWords;
  atomicAdd(p, (unsigned long long)llrint((double)v.x * scale));
  atomicAdd(p + 1, (unsigned long long)llrint((double)v.y * scale));
}
__device__ __forceinline__ unsigned long long take_dev(unsigned long long* p) {
  HG_GLOBAL unsigned long long* q = as_global_mut(p);
  const unsigned long long v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Group g of tiles is complete: move its sums into the pass total (and clear
// them for the next pass), then count the group.  Returns true in the block
// that completes the last group.
__device__ bool tail_group(const PassCtx& a, int g, int* flag) {
  for (int k = threadIdx.x; k < 2 * a.N; k += kBlock) {
    const int64_t e = (int64_t)(k >> 1) * kAccSpotWords + (k & 1);  // spot k / 2, part k % 2
    const unsigned long long v = take_dev(a.acc + (int64_t)(1 + g) * a.N * kAccSpotWords + e);
    atomicAdd(a.acc + e, v);
  }
  return arrive_last(&a.counters[a.plan.ngroups * kCounterStride], (unsigned)a.plan.ngroups, flag);
}

// Every group is complete: V_n = total / 2^shift / |Omega| (the total row is
// cleared for the next pass, and so are the counters); with a.update,
// eqs. (4)-(6): w_n <- w_n mean/|V_n|, theta_n <- arg V_n, A_n = a_n^0 w_n.
__device__ void tail_final(const PassCtx& a, double* wsum) {
  const int N = a.N;
  const double inv = ldexp(1.0, -a.plan.shift) * a.inv_count;
  double magsum = 0.0;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const long long re = (long long)take_dev(a.acc + (int64_t)n * kAccSpotWords);
    const long long im = (long long)take_dev(a.acc + (int64_t)n * kAccSpotWords + 1);
    const double2 t = make_double2((double)re * inv, (double)im * inv);
    a.V[n] = t;
    magsum += sqrt(t.x * t.x + t.y * t.y);
  }
  // the counters are ready for the next pass (kernel end orders these
  // writes; in a chained launch, the generation word)
  for (int k = threadIdx.x; k <= a.plan.ngroups; k += kBlock) {
    if (a.chain)
      __hip_atomic_store(a.counters + k * kCounterStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      a.counters[k * kCounterStride] = 0u;
  }
  if (!a.update) return;
  // sum of |V_n| in a fixed order: per thread, within each wave, then the waves
  for (int off = 32; off > 0; off >>= 1) magsum += __shfl_xor(magsum, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = magsum;
  __syncthreads();
  double total = wsum[0];
  for (int w = 1; w < kWaves; ++w) total += wsum[w];
  const double mean = total / (double)N;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const double2 v = a.V[n];  // written above by this same thread
    const double mag = sqrt(v.x * v.x + v.y * v.y);
    SpotRec r = a.chain ? a.recs[n] : a.sp[n];
    const double w = (double)r.w * (mean / mag);
    if (!(mag > 0.0) || !isfinite(w)) {
      a.status[0] = 4;  // HG_ENUMERIC
      continue;
    }
    r.w = (float)w;
    r.A = (float)(w * (double)r.a0);
    // theta is kept in FP32 turns: the FP32 arctangent of the FP64 sum
    // (rounded to FP32) is within a few FP32 ulps of the rounded FP64 one
    r.th = atan2f((float)v.y, (float)v.x) * 0.15915494309189535f;
    if (a.chain) store_rec_dev(a.sp + n, r);
    else a.sp[n] = r;
    // C_n = A_n e^{i theta_n} = A_n V_n / |V_n|
    const double Am = w * (double)r.a0 / mag;
    a.coef[n] = make_float2((float)(Am * v.x), (float)(Am * v.y));
  }
}

// Chained launch: the update of this pass is complete (this block's state
// stores first), so the next pass may start.
__device__ void publish_gen(const PassCtx& a) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if ((int)threadIdx.x < kGenCopies)
    __hip_atomic_store(a.gen + threadIdx.x * kCounterStride, a.gen_next, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Counts `count` tiles listed in done[] into their groups (the block's own
// additions to the group sums are complete first); the groups this block
// completes are appended to owned[].
constexpr int kDoneList = 256;  // = kBlock: one counting thread per tile
constexpr int kMaxGroups = 128;
__device__ void count_tiles(const PassCtx& a, const int* done, int count, int* owned,
                            int* nowned) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's atomic additions are complete
  __syncthreads();
  if ((int)threadIdx.x < count) {
    const int g = done[threadIdx.x] / a.plan.group_size;
    const int size = min(a.plan.group_size, a.plan.tiles - g * a.plan.group_size);
    if (atomicAdd(&a.counters[g * kCounterStride], 1u) == (unsigned)size - 1u) owned[atomicAdd(nowned, 1)] = g;
  }
  __syncthreads();
}

}  // namespace
}  // namespace hg
