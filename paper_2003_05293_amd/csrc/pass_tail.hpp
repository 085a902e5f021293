// Hand-off of the FP32 passes: the per-block context, the exact fixed-point
// sums of the forward projection (eq. 3) and the weight update of eqs.
// (4)-(6), shared by the per-pixel and the separable kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_common.hpp"
#include "device_math.hpp"
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
  // deferred updates (PassDesc): the total row of this pass's sums, whether
  // the pass stops after the group sums, and the previous pass's total row,
  // which the update clears (-1: none)
  int tot_row = 0;
  int defer = 0;
  int pend_row = -1;
  // chained launches and pending passes: the pass's spot state in LDS;
  // chained launches: the generation word to publish after the update
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
// tiles, groups or blocks arrive.  Rows: the sets of pass totals (rows
// 0..kAccGroupRow0-1, kAccReplicas per set), then row kAccGroupRow0 + g =
// group g.
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
    const unsigned long long v = take_dev(a.acc + (int64_t)(kAccGroupRow0 + g) * a.N * kAccSpotWords + e);
    atomicAdd(a.acc + (int64_t)a.tot_row * kAccReplicas * a.N * kAccSpotWords + e, v);
  }
  return arrive_last(&a.counters[a.plan.ngroups * kCounterStride], (unsigned)a.plan.ngroups, flag);
}

// The weight update of eqs. (4)-(6) in FP32: the one place that does this
// arithmetic, so that a deferred update gives the bits of an immediate one.
// A spot field enters as the FP64 mean of the exact sums rounded to FP32.
__device__ __forceinline__ float2 field32(double2 t) { return make_float2((float)t.x, (float)t.y); }
__device__ __forceinline__ float mag32(float2 v) { return sqrtf(fmaf(v.x, v.x, v.y * v.y)); }
// mean_n |V_n| (eq. 4), the same in every thread of the block: thread t
// adds |V_n| for n = t, t + kBlock, ... in that order, starting from 0 (s
// is that thread sum); the thread sums are added in a fixed tree within
// each wave, then the wave sums in wave order.  Every thread must call it
// (it holds a block barrier).
__device__ __forceinline__ float block_mean_of(float s, int N) {
  __shared__ float wsum[kWaves];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  float total = wsum[0];
  for (int w = 1; w < kWaves; ++w) total += wsum[w];
  return total / (float)N;
}
// false (record unchanged) where the weight would come out zero or not finite
__device__ __forceinline__ bool update_rec(SpotRec& r, float2 v, float mag, float mean) {
  const float w = r.w * (mean / mag);
  if (!(mag > 0.f) || !isfinite(w)) return false;
  r.w = w;
  r.A = w * r.a0;
  r.th = atan2f(v.y, v.x) * 0.15915494309189535f;
  return true;
}

// Every group is complete: V_n = total / 2^shift / |Omega| (the total row is
// cleared for the next pass, and so are the counters); with a.update,
// eqs. (4)-(6): w_n <- w_n mean/|V_n|, theta_n <- arg V_n, A_n = a_n^0 w_n.
// vs: LDS room for N float2 (the spot fields in FP32, kept for the update:
// values other threads stored to memory are not read back, since a block
// of a chained launch may hold stale copies of them in its L1 cache).
// In a chained launch the passes' updates run in blocks on any XCD, and the
// XCDs' L2 caches write back independently: a plain store of C_n or V_n
// could leave an older pass's value dirty in one L2 and written back after
// the newer one, so there every state word goes out with device-scope
// stores (not left dirty in any L2).
__device__ void tail_final(const PassCtx& a, float2* vs) {
  const int N = a.N;
  const double inv = ldexp(1.0, -a.plan.shift) * a.inv_count;
  unsigned long long* tot = a.acc + (int64_t)a.tot_row * kAccReplicas * N * kAccSpotWords;
  float msum = 0.f;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const long long re = (long long)take_dev(tot + (int64_t)n * kAccSpotWords);
    const long long im = (long long)take_dev(tot + (int64_t)n * kAccSpotWords + 1);
    const double2 t = make_double2((double)re * inv, (double)im * inv);
    if (a.chain) store_dev(a.V + n, t);
    else a.V[n] = t;
    const float2 v = field32(t);
    vs[n] = v;
    msum += mag32(v);
  }
  // the previous pass's total set, which every block of this pass has read
  // before counting its tiles, is cleared
  if (a.pend_row >= 0) {
    HG_GLOBAL unsigned long long* q =
        as_global_mut(a.acc + (int64_t)a.pend_row * kAccReplicas * N * kAccSpotWords);
    for (int k = threadIdx.x; k < kAccReplicas * N * kAccSpotWords; k += kBlock)
      __hip_atomic_store(q + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  const float mean = block_mean_of(msum, N);
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const float2 v = vs[n];
    const float mag = mag32(v);
    SpotRec r = a.recs ? a.recs[n] : a.sp[n];
    if (!update_rec(r, v, mag, mean)) {
      a.status[0] = 4;  // HG_ENUMERIC
      if (a.recs && !a.chain) a.sp[n] = r;  // the state this pass used
      continue;
    }
    if (a.chain) store_rec_dev(a.sp + n, r);
    else a.sp[n] = r;
    // C_n = A_n e^{i theta_n} = A_n V_n / |V_n|
    const float Am = r.A / mag;
    if (a.chain) store_dev(a.coef + n, make_float2(Am * v.x, Am * v.y));
    else a.coef[n] = make_float2(Am * v.x, Am * v.y);
  }
}

// Pending pass: every block adds the rows of the previous pass's total set
// (integer sums: the total that a hand-off would have formed), applies that
// pass's update to the state before it (d.st_in) and keeps the result in
// recs (LDS), with the arithmetic and the mean of tail_final (one spot per
// thread); with cl, also C_n = A_n e^{i theta_n} in FP32 (LDS), formed as
// tail_final forms it.  Block 0 (lead) also clears
// the total set two passes back, stores the state for the next pass when
// this pass defers in turn (the final state, in the final hologram), the
// previous V when traced, and the status.  N <= kPendMaxSpots <= kBlock.
// D: PassDesc or SepDesc.
template <typename D>
__device__ void apply_pending(const JobDev& jb, const D& d, bool lead, SpotRec* recs,
                              float2* cl = nullptr) {
  const int N = jb.N;
  const int n = threadIdx.x;
  if (lead && d.clear_row >= 0) {
    HG_GLOBAL unsigned long long* q =
        as_global_mut(jb.acc + (int64_t)d.clear_row * kAccReplicas * N * kAccSpotWords);
    for (int k = threadIdx.x; k < kAccReplicas * N * kAccSpotWords; k += kBlock)
      __hip_atomic_store(q + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  double2 t = make_double2(0.0, 0.0);
  // the record as eight words (a struct copy through a generic pointer
  // would go through the stack)
  constexpr int kWords = (int)(sizeof(SpotRec) / sizeof(float));
  float f[kWords];
#pragma unroll
  for (int k = 0; k < kWords; ++k) f[k] = 0.f;
  if (n < N) {
    const HG_GLOBAL unsigned long long* tot =
        as_global(jb.acc + ((int64_t)d.prev_row * kAccReplicas * N + n) * kAccSpotWords);
    unsigned long long sre = 0ull, sim = 0ull;  // modulo 2^64: the exact total fits
#pragma unroll
    for (int r = 0; r < kAccReplicas; ++r) {
      const HG_GLOBAL unsigned long long* t = tot + (int64_t)r * N * kAccSpotWords;
      sre += __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sim += __hip_atomic_load(t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const long long re = (long long)sre, im = (long long)sim;
    t = make_double2((double)re * d.prev_inv, (double)im * d.prev_inv);
    const HG_GLOBAL float* src = as_global(reinterpret_cast<const float*>(d.st_in + n));
#pragma unroll
    for (int k = 0; k < kWords; ++k) f[k] = src[k];
  }
  const float mean = block_mean_of(n < N ? mag32(field32(t)) : 0.f, N);
  if (n < N) {
    if (lead && d.prev_V) {
      HG_GLOBAL double* v = as_global_mut(reinterpret_cast<double*>(d.prev_V + n));
      v[0] = t.x;
      v[1] = t.y;
    }
    SpotRec r;
    __builtin_memcpy(&r, f, sizeof(r));
    const float2 v = field32(t);
    const float mag = mag32(v);
    const bool ok = update_rec(r, v, mag, mean);
    if (!ok && lead) jb.status[0] = 4;  // HG_ENUMERIC
    if (cl) {  // C_n = A_n e^{i theta_n}
      float2 C;
      if (ok) {
        const float Am = r.A / mag;  // as tail_final forms it
        C = make_float2(Am * v.x, Am * v.y);
      } else {
        float sn, cs;
        sincos_turns(r.th, sn, cs);
        C = make_float2(r.A * cs, r.A * sn);
      }
      cl[n] = C;
    }
    __builtin_memcpy(f, &r, sizeof(r));
    float* dst = reinterpret_cast<float*>(recs + n);
#pragma unroll
    for (int k = 0; k < kWords; ++k) dst[k] = f[k];
    if (lead && d.st_out) {
      HG_GLOBAL float* out = as_global_mut(reinterpret_cast<float*>(d.st_out + n));
#pragma unroll
      for (int k = 0; k < kWords; ++k) out[k] = f[k];
    }
  }
  __syncthreads();
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
