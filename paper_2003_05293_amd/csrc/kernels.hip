// HIP kernels of the RS / WGS / CS-WGS hot path for gfx950 (wave64).
//
// Paper section 2: eq. (1) back-propagation, eq. (2) lens-and-prism phase,
// eq. (3) forward projection, eqs. (4)-(6) weight update, eq. (7) metrics.
// The paper's GPU section recomputes phi_n per pixel rather than storing it;
// the kernels here do the same, in turns, from per-spot coefficients.
//
// All iteration kernels are batched: a launch covers one pass of every job
// listed in its descriptor array, and each block finds its job by a binary
// search over the descriptors' first-block offsets.
#include <math.h>

#include "device_math.hpp"
#include "kernels.hpp"

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

__device__ __forceinline__ int32_t pixel_of(const PixelSet& ps, int32_t q) {
  if (ps.idx) return as_global(ps.idx)[q];
  if (ps.perm) {
    int64_t k = ps.start + q;
    if (k >= ps.M) k -= ps.M;
    return as_global(ps.perm)[k];
  }
  return q;
}

// Doubled integer offsets of pixel p from the grid centre and Q = Lx^2+Ly^2.
struct PixCoord {
  float Lx, Ly, Q;
};

__device__ __forceinline__ PixCoord pixel_coord(int32_t p, int W, int H) {
  const int32_t j = p / W;
  const int32_t i = p - j * W;
  const int32_t lx = 2 * i - (W - 1);
  const int32_t ly = 2 * j - (H - 1);
  PixCoord c;
  c.Lx = (float)lx;
  c.Ly = (float)ly;
  c.Q = (float)(lx * lx + ly * ly);
  return c;
}

// Field of eq. (1) at one pixel over spots [n0, n1): sum A_n e^{i 2 pi (t_n + th_n)}.
// The spot loop index is uniform across the wave, so the records come in
// through scalar loads and feed the vector ALU as scalar operands.
__device__ __forceinline__ float2 backprop_field(const SpotRec* spg, int n0, int n1,
                                                 const PixCoord& c) {
  const HG_CONST SpotRec* sp = as_const(spg);
  float sr = 0.f, si = 0.f;
#pragma unroll 4
  for (int n = n0; n < n1; ++n) {
    const float scx = sp[n].cx, scy = sp[n].cy, scz = sp[n].cz, sth = sp[n].th, sA = sp[n].A;
    const float t = fmaf(scx, c.Lx, fmaf(scy, c.Ly, fmaf(scz, c.Q, sth)));
    float sn, cs;
    sincos_turns(t, sn, cs);
    sr = fmaf(sA, cs, sr);
    si = fmaf(sA, sn, si);
  }
  return make_float2(sr, si);
}

// ---------------------------------------------------------------- setup ---

// Spot coefficients in FP64, rounded once to FP32; theta^0 from Philox;
// w = 1; pass counters cleared.  Spot values that are not finite, or
// amplitudes that are not positive, raise the argument status flag
// (device-resident inputs cannot be checked on the host).  Blocks with
// blockIdx.y > 0 fill the Feistel round tables of compressed jobs.
__global__ __launch_bounds__(256) void k_setup_batch(const JobDev* __restrict__ jobs) {
  const JobDev& jb = jobs[blockIdx.x];
  if (blockIdx.y == 0) {
    const double lf = jb.lambda_mm * jb.focal_mm;
    const double lf2 = lf * jb.focal_mm;
    for (int n = threadIdx.x; n < jb.N; n += blockDim.x) {
      const double x = jb.in.x[n], y = jb.in.y[n], z = jb.in.z[n], amp = jb.in.amp[n];
      if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !(amp > 0.0) || !isfinite(amp))
        jb.status[0] = 1;  // HG_EINVAL
      SpotRec r;
      r.cx = (float)(x * jb.pitch_mm / (2.0 * lf));
      r.cy = (float)(y * jb.pitch_mm / (2.0 * lf));
      r.cz = (float)(z * jb.pitch_mm * jb.pitch_mm / (4.0 * lf2));
      r.th = (float)theta0_turns(jb.seed, (uint64_t)n);
      r.A = (float)amp;
      r.a0 = (float)amp;
      r.w = 1.0f;
      r.pad = 0.0f;
      jb.sp[n] = r;
    }
    for (int k = threadIdx.x; k < jb.counters_len; k += blockDim.x) jb.counters[k] = 0u;
  } else if (jb.compressed) {
    const int total = kFeistelRounds << jb.h;
    const int stride = (gridDim.y - 1) * blockDim.x;
    for (int k = (blockIdx.y - 1) * blockDim.x + threadIdx.x; k < total; k += stride)
      jb.tab[k] = feistel_table_entry(jb.seed, k >> jb.h, (uint32_t)k & ((1u << jb.h) - 1u), jb.h);
  }
}

// pi(k) for every k < M of each compressed job.  With LDS, the Feistel
// tables (h <= 11: 48 KB) are staged in LDS; otherwise read from memory.
constexpr int kPermThreads = 512;
constexpr int kPermLdsHalfBits = 11;
constexpr int kPermPerThread = 4;

template <bool LDS>
__global__ __launch_bounds__(kPermThreads) void k_perm_batch(const JobDev* __restrict__ jobs,
                                                             const JobSlice* __restrict__ slices,
                                                             int nslices) {
  __shared__ uint32_t tab_s[LDS ? (kFeistelRounds << kPermLdsHalfBits) : 1];
  const int si = find_desc(slices, nslices, blockIdx.x);
  const JobDev& jb = jobs[slices[si].job];
  const int lb = blockIdx.x - slices[si].block_begin;
  const int nb = ceil_div(jb.M, (int64_t)kPermThreads * kPermPerThread);
  const uint32_t* tab = jb.tab;
  if (LDS) {
    const int total = kFeistelRounds << jb.h;
    for (int k = threadIdx.x; k < total; k += kPermThreads) tab_s[k] = jb.tab[k];
    __syncthreads();
    tab = tab_s;
  }
  for (int32_t k = lb * kPermThreads + threadIdx.x; k < jb.M; k += nb * kPermThreads)
    jb.perm[k] = (int32_t)permute((uint32_t)k, (uint32_t)jb.M, tab, jb.h);
}

__global__ void k_theta0(uint64_t seed, int count, double* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= count) return;
  out[n] = (2.0 * M_PI) * theta0_turns(seed, (uint64_t)n);
}

__global__ void k_set_state(int N, const double* __restrict__ wth, SpotRec* __restrict__ sp) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double w = wth[n];
  double t = wth[N + n] / (2.0 * M_PI);
  t -= floor(t);
  SpotRec r = sp[n];
  r.w = (float)w;
  r.A = (float)(w * (double)r.a0);
  r.th = (float)t;
  sp[n] = r;
}

__global__ void k_gather(PixelSet ps, int32_t* __restrict__ out) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ps.count) return;
  out[q] = pixel_of(ps, q);
}

// ------------------------------------------------------------ iteration ---

// One pass of one job over a pixel set, in tiles of kTile pixels:
//  phase 1  back-propagation (eq. 1) of the current state, the spot sum
//           split over the block's waves (wave w adds spots
//           [w N/4, (w+1) N/4) for all kTile pixels, lane = pixel, spot
//           records uniform across the wave); the four partial fields are
//           added in wave order and normalised to u = e^{i Phi};
//           or, for a forward test pass, u = e^{i Phi} of a stored hologram;
//  phase 2  forward projection (eq. 3): lanes map to spots (groups of Lg
//           lanes, R = 64/Lg replicas each taking every R-th pixel), waves
//           to (spot chunk, pixel slice) units; each lane keeps its running
//           sum across all tiles of the block;
//  tail     the block's per-spot sums go to partial[block]; the last block
//           of each group of blocks to finish adds its group's partials (in
//           block order, FP64), and the last group to finish adds the group
//           sums (in group order), divides by |Omega| and, when asked,
//           applies the weight update of eqs. (4)-(6) in place.
// Every sum is taken in an order fixed by the job's pass alone, so results
// depend neither on scheduling nor on the other jobs of the batch.

__device__ __forceinline__ void forward_term(float cx, float cy, float cz, const float4& a,
                                             float ui, float& vr, float& vi) {
  const float t = fmaf(cx, a.x, fmaf(cy, a.y, cz * a.z));
  float sn, cs;
  sincos_turns(t, sn, cs);
  // u * conj(e^{i 2 pi t})
  vr = fmaf(a.w, cs, fmaf(ui, sn, vr));
  vi = fmaf(ui, cs, fmaf(-a.w, sn, vi));
}

// Spot-lane layout of phase 2 for N spots.
struct LaneMap {
  int Lg;   // lanes per spot group (8, 16, 32 or 64)
  int R;    // replicas per wave = 64 / Lg
  int nch;  // spot chunks = ceil(N / Lg)
  int S;    // pixel slices per chunk
  int U;    // units = nch * S
};

__host__ __device__ inline LaneMap lane_map(int N) {
  LaneMap m;
  const int n = N < 64 ? N : 64;
  m.Lg = n <= 8 ? 8 : n <= 16 ? 16 : n <= 32 ? 32 : 64;
  m.R = 64 / m.Lg;
  m.nch = (N + m.Lg - 1) / m.Lg;
  m.S = m.nch >= kWaves ? 1 : kWaves / m.nch;
  m.U = m.nch * m.S;
  return m;
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

// Sum over rows k = k0, k0 + step, ... < k1 of src[k * N + n], in that
// order, in FP64.  Loads are issued kBatch at a time so that their latency
// overlaps; out-of-range slots contribute exact zeros.
constexpr int kBatch = 8;
template <typename T>
__device__ __forceinline__ double2 ordered_column_sum(const T* __restrict__ src, int N, int n,
                                                      int k0, int k1, int step) {
  double re = 0.0, im = 0.0;
  for (int k = k0; k < k1; k += step * kBatch) {
    T v[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const int kk = k + b * step;
      v[b] = kk < k1 ? load_dev(src + (int64_t)kk * N + n) : T{};
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      re += (double)v[b].x;
      im += (double)v[b].y;
    }
  }
  return make_double2(re, im);
}

// Returns true in the block that made the last of `expected` increments.
__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned expected, int* flag) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's device-scope writes are complete
  __syncthreads();
  if (threadIdx.x == 0) *flag = atomicAdd(counter, 1u) == expected - 1u;
  __syncthreads();
  return *flag != 0;
}

// Everything one (virtual) block of a pass needs, uniform across the block.
struct PassCtx {
  SpotRec* sp;
  int N, W, H;
  PixelSet ps;
  const float* phi;
  int tiles, group_size, ngroups;
  int lb, nb;  // this block within the pass, blocks of the pass
  float2* partial;
  double2* gpart;
  unsigned* counters;
  double inv_count;
  double2* V;
  int32_t* status;
  int update, from_phi;
};

// Adds this block's partials into the group / global sums (see above).
__device__ void pass_tail(const PassCtx& a) {
  __shared__ int last;
  __shared__ double mred[kBlock];
  __shared__ double2 cred[kBlock];
  const int N = a.N;
  // thread = (spot lane c, slice s): Npad spot lanes, S slices
  int Npad = 1;
  while (Npad < N && Npad < kBlock) Npad <<= 1;
  const int S = kBlock / Npad;
  const int c = threadIdx.x % Npad, s = threadIdx.x / Npad;

  const int g = a.lb / a.group_size;
  const int b0 = g * a.group_size;
  const int b1 = min(b0 + a.group_size, a.nb);
  if (!arrive_last(&a.counters[g], (unsigned)(b1 - b0), &last)) return;
  for (int n0 = 0; n0 < N; n0 += Npad) {
    const int n = n0 + c;
    cred[threadIdx.x] = n < N ? ordered_column_sum(a.partial, N, n, b0 + s, b1, S)
                              : make_double2(0.0, 0.0);
    __syncthreads();
    if (s == 0 && n < N) {
      double2 t = cred[c];
      for (int k = 1; k < S; ++k) {
        t.x += cred[k * Npad + c].x;
        t.y += cred[k * Npad + c].y;
      }
      store_dev(a.gpart + (int64_t)g * N + n, t);
    }
    __syncthreads();
  }
  if (!arrive_last(&a.counters[a.ngroups], (unsigned)a.ngroups, &last)) return;
  // global sums, |V_n| and their total (thread (c, 0) owns spot n = n0 + c)
  double magsum = 0.0;
  for (int n0 = 0; n0 < N; n0 += Npad) {
    const int n = n0 + c;
    cred[threadIdx.x] = n < N ? ordered_column_sum(a.gpart, N, n, s, a.ngroups, S)
                              : make_double2(0.0, 0.0);
    __syncthreads();
    if (s == 0 && n < N) {
      double2 t = cred[c];
      for (int k = 1; k < S; ++k) {
        t.x += cred[k * Npad + c].x;
        t.y += cred[k * Npad + c].y;
      }
      t.x *= a.inv_count;
      t.y *= a.inv_count;
      a.V[n] = t;
      magsum += sqrt(t.x * t.x + t.y * t.y);
    }
    __syncthreads();
  }
  // the counters are ready for the next pass (kernel end orders these writes)
  for (int k = threadIdx.x; k <= a.ngroups; k += kBlock) a.counters[k] = 0u;
  if (!a.update) return;
  mred[threadIdx.x] = magsum;
  __syncthreads();
  for (int stride = kBlock / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) mred[threadIdx.x] += mred[threadIdx.x + stride];
    __syncthreads();
  }
  const double mean = mred[0] / (double)N;
  if (s != 0) return;
  // eqs. (4)-(6): w_n <- w_n mean/|V_n|, theta_n <- arg V_n, A_n = a_n^0 w_n.
  for (int n = c; n < N; n += Npad) {
    const double2 v = a.V[n];  // written above by this same thread
    const double mag = sqrt(v.x * v.x + v.y * v.y);
    SpotRec r = a.sp[n];
    const double w = (double)r.w * (mean / mag);
    if (!(mag > 0.0) || !isfinite(w)) {
      a.status[0] = 4;  // HG_ENUMERIC
      continue;
    }
    r.w = (float)w;
    r.A = (float)(w * (double)r.a0);
    r.th = (float)(atan2(v.y, v.x) / (2.0 * M_PI));
    a.sp[n] = r;
  }
}

template <int MAXU>
__device__ void pass_block(const PassCtx& a, float2 (*sw)[kTile], float4* px, float* pui,
                           float2 (*red)[64]) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N;
  const LaneMap lm = lane_map(N);
  const int g = lane % lm.Lg, r = lane / lm.Lg;
  const SpotRec* __restrict__ sp = a.sp;

  float cx[MAXU], cy[MAXU], cz[MAXU], vr[MAXU], vi[MAXU];
#pragma unroll
  for (int k = 0; k < MAXU; ++k) {
    const int u = wave + k * kWaves;
    const int n = (u / lm.S) * lm.Lg + g;
    cx[k] = cy[k] = cz[k] = 0.f;
    vr[k] = vi[k] = 0.f;
    if (u < lm.U && n < N) {
      const HG_GLOBAL SpotRec* rec = as_global(sp + n);
      cx[k] = rec->cx;
      cy[k] = rec->cy;
      cz[k] = rec->cz;
    }
  }
  const int n_lo = (wave * N) / kWaves, n_hi = ((wave + 1) * N) / kWaves;

  for (int tile = a.lb; tile < a.tiles; tile += a.nb) {
    const int32_t q = tile * kTile + lane;
    const bool valid = q < a.ps.count;
    if (a.from_phi) {
      if (wave == 0) {
        float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
        float ui = 0.f;
        if (valid) {
          const int32_t p = pixel_of(a.ps, q);
          const PixCoord c = pixel_coord(p, a.W, a.H);
          float sn, cs;
          sincos_turns(as_global(a.phi)[p] * 0.15915494309189535f, sn, cs);
          rec = make_float4(c.Lx, c.Ly, c.Q, cs);
          ui = sn;
        }
        px[lane] = rec;
        pui[lane] = ui;
      }
      __syncthreads();
    } else {
      PixCoord c{0.f, 0.f, 0.f};
      if (valid) c = pixel_coord(pixel_of(a.ps, q), a.W, a.H);
      sw[wave][lane] = backprop_field(sp, n_lo, n_hi, c);
      __syncthreads();
      if (wave == 0) {
        float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
        float ui = 0.f;
        if (valid) {
          float2 S = sw[0][lane];
#pragma unroll
          for (int w = 1; w < kWaves; ++w) {
            S.x += sw[w][lane].x;
            S.y += sw[w][lane].y;
          }
          const float m2 = S.x * S.x + S.y * S.y;
          float ur = 1.f;
          if (m2 > 0.f) {
            const float inv = rsqrtf(m2);
            ur = S.x * inv;
            ui = S.y * inv;
          }
          rec = make_float4(c.Lx, c.Ly, c.Q, ur);
        }
        px[lane] = rec;
        pui[lane] = ui;
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MAXU; ++k) {
      const int u = wave + k * kWaves;
      if (u < lm.U) {
        const int sl = u % lm.S;
        const int j0 = (sl * kTile) / lm.S + r, j1 = ((sl + 1) * kTile) / lm.S;
        for (int j = j0; j < j1; j += lm.R)
          forward_term(cx[k], cy[k], cz[k], px[j], pui[j], vr[k], vi[k]);
      }
    }
    __syncthreads();
  }
  // block partials: spot n = c*Lg + g of chunk c sums units (c, s) over
  // slices s and replicas r, in that order.
#pragma unroll
  for (int k = 0; k < MAXU; ++k) {
    const int u = wave + k * kWaves;
    if (u < lm.U) red[u][lane] = make_float2(vr[k], vi[k]);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < lm.nch * lm.Lg; idx += kBlock) {
    const int ch = idx / lm.Lg, gg = idx % lm.Lg;
    const int n = ch * lm.Lg + gg;
    if (n >= N) continue;
    float2 acc = make_float2(0.f, 0.f);
    for (int sl = 0; sl < lm.S; ++sl)
      for (int rr = 0; rr < lm.R; ++rr) {
        const float2 v = red[ch * lm.S + sl][rr * lm.Lg + gg];
        acc.x += v.x;
        acc.y += v.y;
      }
    store_dev(a.partial + (int64_t)a.lb * N + n, acc);
  }
  pass_tail(a);
}

// Batched pass launch: blocks [descs[i].block_begin, descs[i+1].block_begin)
// work on pass i.
template <int MAXU>
__global__ __launch_bounds__(kBlock) void k_pass_batch(const JobDev* __restrict__ jobs,
                                                       const PassDesc* __restrict__ descs,
                                                       int ndesc) {
  __shared__ float2 sw[kWaves][kTile];
  __shared__ float4 px[kTile];
  __shared__ float pui[kTile];
  __shared__ float2 red[kWaves * MAXU][64];
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const PassDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  PassCtx a;
  a.sp = jb.sp;
  a.N = jb.N;
  a.W = jb.W;
  a.H = jb.H;
  a.ps = d.ps;
  a.phi = jb.phi;
  a.tiles = d.plan.tiles;
  a.group_size = d.plan.group_size;
  a.ngroups = d.plan.ngroups;
  a.lb = blockIdx.x - d.block_begin;
  a.nb = d.plan.blocks;
  a.partial = jb.partial;
  a.gpart = jb.gpart;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = d.from_phi;
  pass_block<MAXU>(a, sw, px, pui, red);
}

// Final hologram on a pixel set: Phi = atan2(Im S, Re S), written to out[q].
__global__ __launch_bounds__(kBlock) void k_backprop_batch(const JobDev* __restrict__ jobs,
                                                           const BackDesc* __restrict__ descs,
                                                           int ndesc) {
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const BackDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  const int32_t q = (blockIdx.x - d.block_begin) * kBlock + threadIdx.x;
  if (q >= d.ps.count) return;
  const PixCoord c = pixel_coord(pixel_of(d.ps, q), jb.W, jb.H);
  const float2 S = backprop_field(jb.sp, 0, jb.N, c);
  as_global_mut(d.out)[q] = atan2f(S.y, S.x);
}

// ------------------------------------------------- separable full passes ---

// Separable factors of eq. (2) for the full-grid passes, from FP64 phases:
//   F[n][i] = e^{i 2 pi fx_n(i)},  G[j][n] = e^{i 2 pi fy_n(j)},
//   B[j][n] = A_n e^{i 2 pi (fy_n(j) + th_n)}   (current state A, th).
__global__ __launch_bounds__(256) void k_sep_tables(const JobDev* __restrict__ jobs,
                                                    const JobSlice* __restrict__ slices,
                                                    int nslices) {
  const int si = find_desc(slices, nslices, blockIdx.x);
  const JobDev& jb = jobs[slices[si].job];
  const int lb = blockIdx.x - slices[si].block_begin;
  const int W = jb.W, H = jb.H, N = jb.N;
  const int nb = ceil_div((int64_t)N * (W + H), 256);
  const int64_t nF = (int64_t)N * W, total = nF + (int64_t)H * N;
  const double lf = jb.lambda_mm * jb.focal_mm;
  const double lf2 = lf * jb.focal_mm;
  const double kxy = jb.pitch_mm / (2.0 * lf), kz = jb.pitch_mm * jb.pitch_mm / (4.0 * lf2);
  for (int64_t k = (int64_t)lb * 256 + threadIdx.x; k < total; k += (int64_t)nb * 256) {
    if (k < nF) {
      const int n = (int)(k / W), i = (int)(k % W);
      const double L = (double)(2 * i - (W - 1));
      double t = jb.in.x[n] * kxy * L + jb.in.z[n] * kz * L * L;
      t -= rint(t);
      double s, c;
      sincospi(2.0 * t, &s, &c);
      jb.sepF[k] = make_float2((float)c, (float)s);
    } else {
      const int64_t kk = k - nF;
      const int j = (int)(kk / N), n = (int)(kk % N);
      const double L = (double)(2 * j - (H - 1));
      double t = jb.in.y[n] * kxy * L + jb.in.z[n] * kz * L * L;
      t -= rint(t);
      double s, c;
      sincospi(2.0 * t, &s, &c);
      jb.sepG[kk] = make_float2((float)c, (float)s);
      double tb = t + (double)jb.sp[n].th;
      tb -= rint(tb);
      sincospi(2.0 * tb, &s, &c);
      const double A = (double)jb.sp[n].A;
      jb.sepB[kk] = make_float2((float)(A * c), (float)(A * s));
    }
  }
}

constexpr int kGK = 16;  // K chunk of the separable products

// float2 load through a global-address-space view (two adjacent floats).
__device__ __forceinline__ float2 ldg2(const float2* p) {
  const HG_GLOBAL float* f = as_global(reinterpret_cast<const float*>(p));
  return make_float2(f[0], f[1]);
}

__device__ __forceinline__ void cmac(float2& acc, const float2& a, const float2& b) {
  acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
  acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}

// One 64 x 64 output tile (rows j, columns i) per block.  Thread (tr, tc)
// of the 16 x 16 thread grid owns rows tr + 16 r and columns tc + 16 c
// (r, c < 4), so LDS reads of a column group are conflict-free.
//  phase A  S = B F over the N spots (FP32, K chunks of 16 in LDS);
//  FINAL    Phi = atan2(S) is written and the block ends;
//  else     u = S / |S| goes to LDS; phase B forms, per chunk of 64 spots,
//           T[j][n] = sum_i u(j,i) conj(F_n(i)) over the tile's columns and
//           the block's partial V_n = sum_j conj(G_n(j)) T[j][n] (rows in
//           fixed order), which the pass tail reduces and applies.
template <bool FINAL>
__global__ __launch_bounds__(kBlock) void k_sep_pass(const JobDev* __restrict__ jobs,
                                                     const SepDesc* __restrict__ descs,
                                                     int ndesc) {
  __shared__ float2 As[kSepTile][kGK + 1];
  __shared__ float2 Bs[kGK][kSepTile];
  __shared__ float2 us[FINAL ? 1 : kSepTile][kSepTile + 1];
  __shared__ float2 red[16][kSepTile];
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const SepDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  const int W = jb.W, H = jb.H, N = jb.N;
  const int lb = blockIdx.x - d.block_begin;
  const int j0 = (lb / d.tiles_x) * kSepTile, i0 = (lb % d.tiles_x) * kSepTile;
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  const float2* Bt = jb.sepB;
  const float2* Ft = jb.sepF;

  float2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < N; k0 += kGK) {
    for (int e = threadIdx.x; e < kSepTile * kGK; e += kBlock) {
      const int r = e / kGK, kk = e % kGK, j = j0 + r, n = k0 + kk;
      As[r][kk] = (j < H && n < N) ? ldg2(Bt + (int64_t)j * N + n) : make_float2(0.f, 0.f);
    }
    for (int e = threadIdx.x; e < kGK * kSepTile; e += kBlock) {
      const int kk = e / kSepTile, c = e % kSepTile, n = k0 + kk, i = i0 + c;
      Bs[kk][c] = (n < N && i < W) ? ldg2(Ft + (int64_t)n * W + i) : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kGK; ++kk) {
      float2 a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[tr + 16 * r][kk];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tc + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cmac(acc[r][c], a[r], b[c]);
    }
    __syncthreads();
  }
  if (FINAL) {
    HG_GLOBAL float* out = as_global_mut(d.out);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = j0 + tr + 16 * r, i = i0 + tc + 16 * c;
        if (j < H && i < W) out[(int64_t)j * W + i] = atan2f(acc[r][c].y, acc[r][c].x);
      }
    return;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + tr + 16 * r, i = i0 + tc + 16 * c;
      float2 u = make_float2(0.f, 0.f);
      if (j < H && i < W) {
        const float m2 = acc[r][c].x * acc[r][c].x + acc[r][c].y * acc[r][c].y;
        u = make_float2(1.f, 0.f);
        if (m2 > 0.f) {
          const float inv = rsqrtf(m2);
          u = make_float2(acc[r][c].x * inv, acc[r][c].y * inv);
        }
      }
      us[tr + 16 * r][tc + 16 * c] = u;
    }
  __syncthreads();
  const float2* Gt = jb.sepG;
  for (int n0 = 0; n0 < N; n0 += kSepTile) {
    float2 t[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) t[r][c] = make_float2(0.f, 0.f);
    for (int k0 = 0; k0 < kSepTile; k0 += kGK) {
      for (int e = threadIdx.x; e < kGK * kSepTile; e += kBlock) {
        const int c = e / kGK, kk = e % kGK, n = n0 + c, i = i0 + k0 + kk;
        const float2 v = (n < N && i < W) ? ldg2(Ft + (int64_t)n * W + i) : make_float2(0.f, 0.f);
        Bs[kk][c] = make_float2(v.x, -v.y);
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < kGK; ++kk) {
        float2 a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = us[tr + 16 * r][k0 + kk];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tc + 16 * c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) cmac(t[r][c], a[r], b[c]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int n = n0 + tc + 16 * c;
      float2 v = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + tr + 16 * r;
        if (j < H && n < N) {
          const float2 g = ldg2(Gt + (int64_t)j * N + n);
          cmac(v, make_float2(g.x, -g.y), t[r][c]);
        }
      }
      red[tr][tc + 16 * c] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSepTile) {
      const int n = n0 + threadIdx.x;
      if (n < N) {
        float2 s = red[0][threadIdx.x];
        for (int k = 1; k < 16; ++k) {
          s.x += red[k][threadIdx.x].x;
          s.y += red[k][threadIdx.x].y;
        }
        store_dev(jb.partial + (int64_t)lb * N + n, s);
      }
    }
    __syncthreads();
  }
  PassCtx a;
  a.sp = jb.sp;
  a.N = N;
  a.W = W;
  a.H = H;
  a.ps = PixelSet{nullptr, nullptr, 0, W * H, W * H};
  a.phi = nullptr;
  a.tiles = d.plan.tiles;
  a.group_size = d.plan.group_size;
  a.ngroups = d.plan.ngroups;
  a.lb = lb;
  a.nb = d.plan.blocks;
  a.partial = jb.partial;
  a.gpart = jb.gpart;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = 0;
  pass_tail(a);
}

// -------------------------------------------------------------- metrics ---

// FP64 separable factors of e^{-i phi_n}: eq. (2) splits into a part in x'
// and a part in y', so e^{-i phi_n(i,j)} = Ex[i][n] * Ey[j][n].
__global__ void k_metric_tables(SetupArgs a, SpotPtrs in, double2* __restrict__ Ex,
                                double2* __restrict__ Ey) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = a.N;
  const int64_t nx = (int64_t)a.W * N, ny = (int64_t)a.H * N;
  if (k >= nx + ny) return;
  const bool is_x = k < nx;
  const int64_t kk = is_x ? k : k - nx;
  const int pix = (int)(kk / N);
  const int n = (int)(kk % N);
  const int len = is_x ? a.W : a.H;
  const double off = ((double)pix - 0.5 * (double)(len - 1)) * a.pitch_mm;
  const double lat = is_x ? in.x[n] : in.y[n];
  const double z = in.z[n];
  const double lf = a.lambda_mm * a.focal_mm;
  const double lf2 = lf * a.focal_mm;
  double t = lat * off / lf + z * off * off / lf2;  // turns
  t -= rint(t);
  double s, c;
  sincospi(2.0 * t, &s, &c);
  (is_x ? Ex : Ey)[kk] = make_double2(c, -s);
}

constexpr int kMetricRows = 4;
constexpr int kMetricThreads = 128;
constexpr int kMetricCols = 512;

// V*_n partial over kMetricRows rows: sum_j Ey[j][n] * sum_i e^{i Phi(i,j)} Ex[i][n].
__global__ __launch_bounds__(kMetricThreads) void k_metric_rows(
    const double2* __restrict__ Ex, const double2* __restrict__ Ey, int N, int W, int H,
    const float* __restrict__ phi, double2* __restrict__ partial) {
  __shared__ double2 u[kMetricCols];
  const int j0 = blockIdx.x * kMetricRows;
  for (int n0 = 0; n0 < N; n0 += kMetricThreads) {
    const int n = n0 + threadIdx.x;
    double are = 0.0, aim = 0.0;
    for (int r = 0; r < kMetricRows; ++r) {
      const int j = j0 + r;
      if (j >= H) break;
      double rre = 0.0, rim = 0.0;
      for (int i0 = 0; i0 < W; i0 += kMetricCols) {
        const int cols = min(kMetricCols, W - i0);
        __syncthreads();
        for (int k = threadIdx.x; k < cols; k += kMetricThreads) {
          double s, c;
          sincos((double)phi[(int64_t)j * W + i0 + k], &s, &c);
          u[k] = make_double2(c, s);
        }
        __syncthreads();
        if (n < N) {
          for (int k = 0; k < cols; ++k) {
            const double2 e = Ex[(int64_t)(i0 + k) * N + n];
            const double2 v = u[k];
            rre = fma(v.x, e.x, fma(-v.y, e.y, rre));
            rim = fma(v.x, e.y, fma(v.y, e.x, rim));
          }
        }
      }
      if (n < N) {
        const double2 e = Ey[(int64_t)j * N + n];
        are = fma(rre, e.x, fma(-rim, e.y, are));
        aim = fma(rre, e.y, fma(rim, e.x, aim));
      }
    }
    if (n < N) partial[(int64_t)blockIdx.x * N + n] = make_double2(are, aim);
  }
}

__global__ void k_metric_reduce(const double2* __restrict__ partial, int nblk, int N,
                                double inv_count, double2* __restrict__ V) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double re = 0.0, im = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2 v = partial[(int64_t)b * N + n];
    re += v.x;
    im += v.y;
  }
  V[n] = make_double2(re * inv_count, im * inv_count);
}


}  // namespace

// ------------------------------------------------------------ launchers ---

PassPlan plan_pass(int32_t count, int32_t block_cap) {
  PassPlan p;
  p.tiles = ceil_div(count, kTile);
  if (p.tiles < 1) p.tiles = 1;
  p.blocks = p.tiles < block_cap ? p.tiles : block_cap;
  if (p.blocks < 1) p.blocks = 1;
  int gs = 1;
  while (gs * gs < p.blocks) ++gs;
  p.group_size = gs;
  p.ngroups = ceil_div(p.blocks, gs);
  return p;
}

int setup_table_blocks(int max_h) {
  if (max_h <= 0) return 0;
  const int total = kFeistelRounds << max_h;
  int b = ceil_div(total, 256 * 4);
  return b > 64 ? 64 : b;
}

void launch_setup_batch(const JobDev* jobs, int njobs, int max_h, hipStream_t s) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_setup_batch, dim3(njobs, 1 + setup_table_blocks(max_h)), dim3(256), 0, s,
                     jobs);
}

int perm_blocks(int32_t M) { return ceil_div(M, (int64_t)kPermThreads * kPermPerThread); }

void launch_perm_batch(const JobDev* jobs, const JobSlice* slices, int nslices, int total_blocks,
                       bool lds, hipStream_t s) {
  if (nslices <= 0 || total_blocks <= 0) return;
  if (lds)
    hipLaunchKernelGGL(k_perm_batch<true>, dim3(total_blocks), dim3(kPermThreads), 0, s, jobs,
                       slices, nslices);
  else
    hipLaunchKernelGGL(k_perm_batch<false>, dim3(total_blocks), dim3(kPermThreads), 0, s, jobs,
                       slices, nslices);
}

void launch_theta0(uint64_t seed, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_theta0, dim3(ceil_div(count, 256)), dim3(256), 0, s, seed, count, out);
}

void launch_set_state(int N, const double* wth, SpotRec* sp, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, wth, sp);
}

void launch_gather(const PixelSet& ps, int32_t* out, hipStream_t s) {
  if (ps.count <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(ceil_div(ps.count, 256)), dim3(256), 0, s, ps, out);
}

int pass_units_per_wave(int N) {
  const LaneMap lm = lane_map(N);
  return ceil_div(lm.U, kWaves);
}

void launch_pass_batch(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                       int max_units, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  const dim3 grid(total_blocks), block(kBlock);
  if (max_units <= 1) hipLaunchKernelGGL(k_pass_batch<1>, grid, block, 0, s, jobs, descs, ndesc);
  else if (max_units <= 4) hipLaunchKernelGGL(k_pass_batch<4>, grid, block, 0, s, jobs, descs, ndesc);
  else hipLaunchKernelGGL(k_pass_batch<16>, grid, block, 0, s, jobs, descs, ndesc);
}

int backprop_blocks(int32_t count) { return ceil_div(count, kBlock); }

int sep_table_blocks(int W, int H, int N) { return ceil_div((int64_t)N * (W + H), 256); }

void launch_sep_tables(const JobDev* jobs, const JobSlice* slices, int nslices, int total_blocks,
                       hipStream_t s) {
  if (nslices <= 0 || total_blocks <= 0) return;
  hipLaunchKernelGGL(k_sep_tables, dim3(total_blocks), dim3(256), 0, s, jobs, slices, nslices);
}

PassPlan plan_sep(int W, int H) {
  PassPlan p;
  p.tiles = ceil_div(W, kSepTile) * ceil_div(H, kSepTile);
  p.blocks = p.tiles;
  int gs = 1;
  while (gs * gs < p.blocks) ++gs;
  p.group_size = gs;
  p.ngroups = ceil_div(p.blocks, gs);
  return p;
}

void launch_sep_pass(const JobDev* jobs, const SepDesc* descs, int ndesc, int total_blocks,
                     bool final, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  if (final)
    hipLaunchKernelGGL(k_sep_pass<true>, dim3(total_blocks), dim3(kBlock), 0, s, jobs, descs, ndesc);
  else
    hipLaunchKernelGGL(k_sep_pass<false>, dim3(total_blocks), dim3(kBlock), 0, s, jobs, descs,
                       ndesc);
}

void launch_backprop_batch(const JobDev* jobs, const BackDesc* descs, int ndesc,
                           int total_blocks, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  hipLaunchKernelGGL(k_backprop_batch, dim3(total_blocks), dim3(kBlock), 0, s, jobs, descs,
                     ndesc);
}

void launch_metric_tables(const SetupArgs& a, const SpotPtrs& in, double2* Ex, double2* Ey,
                          hipStream_t s) {
  const int64_t total = (int64_t)(a.W + a.H) * a.N;
  hipLaunchKernelGGL(k_metric_tables, dim3(ceil_div(total, 256)), dim3(256), 0, s, a, in, Ex,
                     Ey);
}

int metric_blocks(int H) { return ceil_div(H, kMetricRows); }

void launch_metric_rows(const double2* Ex, const double2* Ey, int N, int W, int H,
                        const float* phi, double2* partial, hipStream_t s) {
  hipLaunchKernelGGL(k_metric_rows, dim3(metric_blocks(H)), dim3(kMetricThreads), 0, s, Ex, Ey,
                     N, W, H, phi, partial);
}

void launch_metric_reduce(const double2* partial, int nblk, int N, double inv_count,
                          double2* V_out, hipStream_t s) {
  hipLaunchKernelGGL(k_metric_reduce, dim3(ceil_div(N, 128)), dim3(128), 0, s, partial, nblk, N,
                     inv_count, V_out);
}

}  // namespace hg
