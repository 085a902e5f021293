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

#include "device_common.hpp"
#include "device_math.hpp"
#include "kernels.hpp"

namespace hg {

namespace {

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
      double sn, cn;
      sincospi(2.0 * theta0_turns(jb.seed, (uint64_t)n), &sn, &cn);
      jb.coef[n] = make_float2((float)(amp * cn), (float)(amp * sn));
    }
    for (int k = threadIdx.x; k < jb.counters_len; k += blockDim.x) jb.counters[k] = 0u;
  } else if (jb.compressed) {
    const int total = kFeistelRounds << jb.h;
    const int stride = (gridDim.y - 1) * blockDim.x;
    for (int k = (blockIdx.y - 1) * blockDim.x + threadIdx.x; k < total; k += stride)
      jb.tab[k] = feistel_table_entry(jb.seed, k >> jb.h, (uint32_t)k & ((1u << jb.h) - 1u), jb.h);
  }
}

// pi(k) for every k < M of each compressed job (and, for mixed-precision
// jobs, the inverse: the rank of every pixel in the order).  With LDS, the Feistel
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
  for (int32_t k = lb * kPermThreads + threadIdx.x; k < jb.M; k += nb * kPermThreads) {
    const uint32_t p = permute((uint32_t)k, (uint32_t)jb.M, tab, jb.h);
    jb.perm[k] = (int32_t)p;
    if (jb.rank) jb.rank[p] = (uint32_t)k;  // pixel p is the k-th of the random order
  }
}

__global__ void k_theta0(uint64_t seed, int count, double* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= count) return;
  out[n] = (2.0 * M_PI) * theta0_turns(seed, (uint64_t)n);
}

__global__ void k_set_state(int N, const double* __restrict__ wth, SpotRec* __restrict__ sp,
                            float2* __restrict__ coef) {
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
  double sn, cn;
  sincospi(2.0 * t, &sn, &cn);
  const double A = w * (double)r.a0;
  coef[n] = make_float2((float)(A * cn), (float)(A * sn));
}

__global__ void k_gather(PixelSet ps, int32_t* __restrict__ out) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ps.count) return;
  out[q] = pixel_of(ps, q);
}

// ------------------------------------------------------------ iteration ---

// One pass of one job over a pixel set, in tiles of kTile pixels.  The
// pass's blocks take tiles dynamically: block b starts with tile b, then
// takes tiles nb, nb + 1, ... in the order the blocks ask for them (one
// counter per pass), so a block on a busy compute unit takes fewer tiles.
// For each tile:
//  phase 1  back-propagation (eq. 1) of the current state, the spot sum
//           split over the block's waves (wave w adds spots
//           [w N/4, (w+1) N/4) for all kTile pixels, lane = pixel, spot
//           records uniform across the wave); the four partial fields are
//           added in wave order and normalised to u = e^{i Phi};
//           or, for a forward test pass, u = e^{i Phi} of a stored hologram;
//  phase 2  forward projection (eq. 3): lanes map to spots (groups of Lg
//           lanes, R = 64/Lg replicas each taking every R-th pixel), waves
//           to (spot chunk, pixel slice) units;
//  partial  the tile's per-spot sums go to partial[tile] (FP32);
//  tail     the block that completes a group of tiles adds the group's
//           partials (tile order, FP64); the block that completes the last
//           group adds the group sums (group order), divides by |Omega|
//           and, when asked, applies the weight update of eqs. (4)-(6).
// A tile's sums do not depend on which block computed it, and every sum is
// taken in an order fixed by the pass alone, so results depend neither on
// scheduling nor on the other jobs of the batch.

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

// Sum over rows k0 + s, k0 + s + S, ... < min(k1, row_end) of column n, in
// that order, in FP64; kBatch loads are issued before any is used.  s is
// the thread's slice; k0 and S are uniform across the block.  Rows past
// row_end fall outside the buffer resource and load as zero.
constexpr int kBatch = 10;
__device__ __forceinline__ double2 column_sum(const ColumnSrc& src, int n, int s, int k0, int k1,
                                              int S) {
  double re = 0.0, im = 0.0;
  const int step = S * src.N * (int)sizeof(float2);
  int off = ((k0 + s) * src.N + n) * (int)sizeof(float2);
  for (int k = k0; k < k1; k += S * kBatch, off += kBatch * step) {
    float2 v[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const auto bits =
          __builtin_amdgcn_raw_buffer_load_b64(src.rsrc, off + b * step, 0, kDeviceScope);
      __builtin_memcpy(&v[b], &bits, sizeof(float2));
    }
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      re += (double)v[b].x;
      im += (double)v[b].y;
    }
  }
  return make_double2(re, im);
}

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
  unsigned* counters;
  double inv_count;
  double2* V;
  int32_t* status;
  int update, from_phi;
};

// Thread layout of the reductions: Npad spot lanes x S slices.
struct RedLayout {
  int Npad, S, c, s;
};
__device__ __forceinline__ RedLayout red_layout(int N) {
  RedLayout r;
  r.Npad = 1;
  while (r.Npad < N && r.Npad < kBlock) r.Npad <<= 1;
  r.S = kBlock / r.Npad;
  r.c = threadIdx.x % r.Npad;
  r.s = threadIdx.x / r.Npad;
  return r;
}

// Group g of tiles is complete: add its tiles' partials (tile order, FP64),
// store the group sums (FP32) and count the group.  Returns true in the
// block that completes the last group.
__device__ bool tail_group(const PassCtx& a, int g, double2* cred, int* flag) {
  const int N = a.N;
  const RedLayout L = red_layout(N);
  const int t0 = g * a.plan.group_size;
  const int t1 = min(t0 + a.plan.group_size, a.plan.tiles);
  const ColumnSrc src = column_src(a.partial, t1, N);
  float2* gsum = reinterpret_cast<float2*>(a.gpart);
  for (int n0 = 0; n0 < N; n0 += L.Npad) {
    const int n = n0 + L.c;
    cred[threadIdx.x] = n < N ? column_sum(src, n, L.s, t0, t1, L.S) : make_double2(0.0, 0.0);
    __syncthreads();
    if (L.s == 0 && n < N) {
      double2 t = cred[L.c];
      for (int k = 1; k < L.S; ++k) {
        t.x += cred[k * L.Npad + L.c].x;
        t.y += cred[k * L.Npad + L.c].y;
      }
      store_dev(gsum + (int64_t)g * N + n, make_float2((float)t.x, (float)t.y));
    }
    __syncthreads();
  }
  return arrive_last(&a.counters[a.plan.ngroups * kCounterStride], (unsigned)a.plan.ngroups, flag);
}

// Every group is complete: V_n = (group sums, group order) / |Omega|; the
// counters are cleared for the next pass; with a.update, eqs. (4)-(6):
// w_n <- w_n mean/|V_n|, theta_n <- arg V_n, A_n = a_n^0 w_n.
__device__ void tail_final(const PassCtx& a, double2* cred, double* wsum) {
  const int N = a.N;
  const RedLayout L = red_layout(N);
  // the spot records of the update travel with the group sums
  SpotRec pre{};
  if (a.update && L.s == 0 && L.c < N) pre = a.sp[L.c];
  const ColumnSrc src = column_src(reinterpret_cast<const float2*>(a.gpart), a.plan.ngroups, N);
  double magsum = 0.0;
  for (int n0 = 0; n0 < N; n0 += L.Npad) {
    const int n = n0 + L.c;
    cred[threadIdx.x] = n < N ? column_sum(src, n, L.s, 0, a.plan.ngroups, L.S)
                              : make_double2(0.0, 0.0);
    __syncthreads();
    if (L.s == 0 && n < N) {
      double2 t = cred[L.c];
      for (int k = 1; k < L.S; ++k) {
        t.x += cred[k * L.Npad + L.c].x;
        t.y += cred[k * L.Npad + L.c].y;
      }
      t.x *= a.inv_count;
      t.y *= a.inv_count;
      a.V[n] = t;
      magsum += sqrt(t.x * t.x + t.y * t.y);
    }
    __syncthreads();
  }
  // the counters are ready for the next pass (kernel end orders these writes)
  for (int k = threadIdx.x; k <= a.plan.ngroups; k += kBlock) a.counters[k * kCounterStride] = 0u;
  if (!a.update) return;
  // sum of |V_n| in a fixed order: within each wave, then the waves in order
  for (int off = 32; off > 0; off >>= 1) magsum += __shfl_xor(magsum, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = magsum;
  __syncthreads();
  double total = wsum[0];
  for (int w = 1; w < kWaves; ++w) total += wsum[w];
  const double mean = total / (double)N;
  if (L.s != 0) return;
  for (int n = L.c; n < N; n += L.Npad) {
    const double2 v = a.V[n];  // written above by this same thread
    const double mag = sqrt(v.x * v.x + v.y * v.y);
    SpotRec r = n == L.c ? pre : a.sp[n];
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
    a.sp[n] = r;
    // C_n = A_n e^{i theta_n} = A_n V_n / |V_n|
    const double Am = w * (double)r.a0 / mag;
    a.coef[n] = make_float2((float)(Am * v.x), (float)(Am * v.y));
  }
}

// Counts the partials of `count` tiles listed in done[] into their groups
// (the block's own partial stores are complete first); the groups this
// block completes are appended to owned[].
constexpr int kDoneList = 256;  // = kBlock: one counting thread per tile
constexpr int kMaxGroups = 128;
__device__ void count_tiles(const PassCtx& a, const int* done, int count, int* owned,
                            int* nowned) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's partial stores are complete
  __syncthreads();
  if ((int)threadIdx.x < count) {
    const int g = done[threadIdx.x] / a.plan.group_size;
    const int size = min(a.plan.group_size, a.plan.tiles - g * a.plan.group_size);
    if (atomicAdd(&a.counters[g * kCounterStride], 1u) == (unsigned)size - 1u) owned[atomicAdd(nowned, 1)] = g;
  }
  __syncthreads();
}

template <int MAXU>
__device__ void pass_block(const PassCtx& a, unsigned* grab) {
  __shared__ float2 sw[kWaves][kTile];
  __shared__ float4 px[kTile];
  __shared__ float pui[kTile];
  __shared__ float2 red[kWaves * MAXU][64];
  __shared__ int done[kDoneList];
  __shared__ int owned[kMaxGroups];
  __shared__ int ndone, nowned, next_tile, flag;
  __shared__ double2 cred[kBlock];
  __shared__ double wsum[kWaves];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N;
  const LaneMap lm = lane_map(N);
  const int g = lane % lm.Lg, r = lane / lm.Lg;
  const SpotRec* __restrict__ sp = a.sp;
  if (threadIdx.x == 0) ndone = nowned = 0;

  float cx[MAXU], cy[MAXU], cz[MAXU];
#pragma unroll
  for (int k = 0; k < MAXU; ++k) {
    const int u = wave + k * kWaves;
    const int n = (u / lm.S) * lm.Lg + g;
    cx[k] = cy[k] = cz[k] = 0.f;
    if (u < lm.U && n < N) {
      const HG_GLOBAL SpotRec* rec = as_global(sp + n);
      cx[k] = rec->cx;
      cy[k] = rec->cy;
      cz[k] = rec->cz;
    }
  }
  const int n_lo = (wave * N) / kWaves, n_hi = ((wave + 1) * N) / kWaves;

  // with fewer blocks than tiles, blocks ask for their next tile while they
  // work on the current one (after its back-propagation, whose memory reads
  // would otherwise wait for the counter's answer)
  const bool dynamic = a.plan.blocks < a.plan.tiles;
  int tile = a.lb;
  while (tile < a.plan.tiles) {
    unsigned ticket = 0u;
    float vr[MAXU], vi[MAXU];
#pragma unroll
    for (int k = 0; k < MAXU; ++k) vr[k] = vi[k] = 0.f;
    for (int st = 0; st < a.plan.sub; ++st) {
      const int32_t q = (tile * a.plan.sub + st) * kTile + lane;
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
        const int32_t p = valid ? pixel_of(a.ps, q) : 0;
        if (dynamic && st == a.plan.sub - 1 && threadIdx.x == 0)
          ticket = atomicAdd(grab, p >= 0 ? 1u : 1u);
        PixCoord c{0.f, 0.f, 0.f};
        if (valid) c = pixel_coord(p, a.W, a.H);
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
      if (a.from_phi && dynamic && st == a.plan.sub - 1 && threadIdx.x == 0)
        ticket = atomicAdd(grab, 1u);
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
    // tile partials: spot n = c*Lg + g of chunk c sums units (c, s) over
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
      store_dev(a.partial + (int64_t)tile * N + n, acc);
    }
    if (threadIdx.x == 0) {
      done[ndone++] = tile;
      next_tile = dynamic ? a.plan.blocks + (int)ticket : a.plan.tiles;
    }
    __syncthreads();
    tile = next_tile;
    if (ndone == kDoneList) {
      count_tiles(a, done, ndone, owned, &nowned);
      if (threadIdx.x == 0) ndone = 0;
      __syncthreads();
    }
  }
  count_tiles(a, done, ndone, owned, &nowned);
  for (int i = 0; i < nowned; ++i)
    if (tail_group(a, owned[i], cred, &flag)) tail_final(a, cred, wsum);
}

}  // namespace

__host__ __device__ int pass_e_width(int N) {
  const int per_wave = (N + kWaves - 1) / kWaves;
  return per_wave <= 8 ? 8 : per_wave <= 16 ? 16 : per_wave <= 25 ? 25 : 0;
}

namespace {

// Sum of x over the 64 lanes of the wave, left in lane 63: an inclusive
// scan within each row of 16 lanes (row shifts 1, 2, 4, 8), then the row
// totals carried across rows (row broadcasts of lanes 15 and 31).  Fixed
// order, so the result does not depend on scheduling.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_shift(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                               ROWMASK, 0xf, ROWMASK == 0xf));
}
__device__ __forceinline__ float wave_sum_lane63(float x) {
  x += dpp_shift<0x111, 0xf>(x);  // row_shr:1
  x += dpp_shift<0x112, 0xf>(x);  // row_shr:2
  x += dpp_shift<0x114, 0xf>(x);  // row_shr:4
  x += dpp_shift<0x118, 0xf>(x);  // row_shr:8
  x += dpp_shift<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_shift<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// The pass with one complex exponential per (pixel, spot) pair, for
// N <= 4 MAXE (MAXE <= 25: the exponentials stay in registers at six waves
// per SIMD).  Lane = pixel, wave w = spots [w N/4, (w+1) N/4):
//  phase 1  E_n(p) = e^{i 2 pi (cx Lx + cy Ly + cz Q)} (eq. 2 without theta)
//           kept in registers, and the wave's share of eq. (1),
//           sum_n C_n E_n(p) with C_n = A_n e^{i theta_n};
//  u        every wave adds the four shares in wave order and normalises
//           (all waves obtain the same u for their lane's pixel);
//  phase 2  the forward terms u conj(E_n(p)) of eq. (3), added over the
//           wave's 64 pixels with a fixed lane reduction.
// Partials, tiles, tile order and the tail are those of pass_block.
template <int MAXE>
__device__ void pass_block_e(const PassCtx& a, unsigned* grab) {
  __shared__ float2 sw[kWaves][kTile];
  __shared__ float2 rede[kWaves][MAXE];
  __shared__ int done[kDoneList];
  __shared__ int owned[kMaxGroups];
  __shared__ int ndone, nowned, next_tile, flag;
  __shared__ double2 cred[kBlock];
  __shared__ double wsum[kWaves];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N;
  const int n_lo = (wave * N) / kWaves, n_hi = ((wave + 1) * N) / kWaves;
  const int cnt = n_hi - n_lo;
  const HG_CONST SpotRec* sp = as_const(a.sp) + n_lo;
  const HG_CONST float2* cf = as_const(a.coef) + n_lo;
  if (threadIdx.x == 0) ndone = nowned = 0;
  const bool dynamic = a.plan.blocks < a.plan.tiles;
  int tile = a.lb;
  while (tile < a.plan.tiles) {
    unsigned ticket = 0u;
    for (int st = 0; st < a.plan.sub; ++st) {
      const int32_t q = (tile * a.plan.sub + st) * kTile + lane;
      const bool valid = q < a.ps.count;
      const int32_t p = valid ? pixel_of(a.ps, q) : 0;
      // the next tile is asked for once the pixel index has arrived (the
      // counter's answer is first needed after phase 1)
      if (dynamic && st == a.plan.sub - 1 && threadIdx.x == 0) ticket = atomicAdd(grab, p >= 0 ? 1u : 1u);
      PixCoord c{0.f, 0.f, 0.f};
      if (valid) c = pixel_coord(p, a.W, a.H);
      float er[MAXE], ei[MAXE];
      float Sr = 0.f, Si = 0.f;
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        er[k] = ei[k] = 0.f;
        if (k < cnt) {
          const float t = fmaf(sp[k].cx, c.Lx, fmaf(sp[k].cy, c.Ly, sp[k].cz * c.Q));
          sincos_turns(t, ei[k], er[k]);
          const float Cr = cf[k].x, Ci = cf[k].y;
          Sr = fmaf(Cr, er[k], fmaf(-Ci, ei[k], Sr));
          Si = fmaf(Cr, ei[k], fmaf(Ci, er[k], Si));
        }
      }
      sw[wave][lane] = make_float2(Sr, Si);
      __syncthreads();
      float2 S = sw[0][lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        S.x += sw[w][lane].x;
        S.y += sw[w][lane].y;
      }
      float ur = 0.f, ui = 0.f;
      if (valid) {
        const float m2 = S.x * S.x + S.y * S.y;
        ur = 1.f;
        if (m2 > 0.f) {
          const float inv = rsqrtf(m2);
          ur = S.x * inv;
          ui = S.y * inv;
        }
      }
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        if (k < cnt) {
          // u conj(E_n)
          const float pr = wave_sum_lane63(fmaf(ur, er[k], ui * ei[k]));
          const float pi = wave_sum_lane63(fmaf(ui, er[k], -ur * ei[k]));
          if (lane == 63) {
            if (st == 0) {
              rede[wave][k] = make_float2(pr, pi);
            } else {
              rede[wave][k].x += pr;
              rede[wave][k].y += pi;
            }
          }
        }
      }
      __syncthreads();  // sw is rewritten by the next sub-tile
    }
    // the tile's partials: spot n_lo + lane of each wave
    if (lane < cnt) store_dev(a.partial + (int64_t)tile * N + n_lo + lane, rede[wave][lane]);
    if (threadIdx.x == 0) {
      done[ndone++] = tile;
      next_tile = dynamic ? a.plan.blocks + (int)ticket : a.plan.tiles;
    }
    __syncthreads();
    tile = next_tile;
    if (ndone == kDoneList) {
      count_tiles(a, done, ndone, owned, &nowned);
      if (threadIdx.x == 0) ndone = 0;
      __syncthreads();
    }
  }
  count_tiles(a, done, ndone, owned, &nowned);
  for (int i = 0; i < nowned; ++i)
    if (tail_group(a, owned[i], cred, &flag)) tail_final(a, cred, wsum);
}

// Batched pass launch: blocks [descs[i].block_begin, descs[i+1].block_begin)
// work on pass i.
// Occupancy target: six waves per SIMD (all blocks of a 1152^2 compressed
// pass resident) except for the widest register forms.
template <int MAXU, int MAXE>
__global__ __launch_bounds__(kBlock, MAXU > 4 ? 4 : 6) void k_pass_batch(const JobDev* __restrict__ jobs,
                                                       const PassDesc* __restrict__ descs,
                                                       int ndesc) {
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const PassDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  PassCtx a;
  a.sp = jb.sp;
  a.coef = jb.coef;
  a.N = jb.N;
  a.W = jb.W;
  a.H = jb.H;
  a.ps = d.ps;
  a.phi = jb.phi;
  a.plan = d.plan;
  a.lb = blockIdx.x - d.block_begin;
  a.partial = jb.partial;
  a.gpart = jb.gpart;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = d.from_phi;
  // the form depends on the job alone (its N, and whether it back-propagates),
  // so a hologram gives the same bits alone and in any batch
  if constexpr (MAXE > 0) {
    if (!d.from_phi && pass_e_width(jb.N) != 0) {
      pass_block_e<MAXE>(a, jb.grab + d.grab_slot);
      return;
    }
  }
  pass_block<MAXU>(a, jb.grab + d.grab_slot);
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
  a.coef = jb.coef;
  a.N = N;
  a.W = W;
  a.H = H;
  a.ps = PixelSet{nullptr, nullptr, 0, W * H, W * H};
  a.phi = nullptr;
  a.plan = d.plan;
  a.lb = lb;
  a.partial = jb.partial;
  a.gpart = jb.gpart;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = 0;
  // one tile per block: count it, then the group and final sums
  __shared__ int flag;
  __shared__ double2 cred[kBlock];
  __shared__ double wsum[kWaves];
  const int g = lb / d.plan.group_size;
  const int size = min(d.plan.group_size, d.plan.tiles - g * d.plan.group_size);
  if (arrive_last(&jb.counters[g * kCounterStride], (unsigned)size, &flag) &&
      tail_group(a, g, cred, &flag))
    tail_final(a, cred, wsum);
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
  int64_t units = ceil_div(count, kTile);  // kTile-pixel sub-tiles
  if (units < 1) units = 1;
  p.sub = ceil_div(units, kMaxTiles);
  p.tiles = ceil_div(units, p.sub);
  p.blocks = p.tiles < block_cap ? p.tiles : block_cap;
  if (p.blocks < 1) p.blocks = 1;
  int gs = 1;
  while (gs * gs < p.tiles) ++gs;
  p.group_size = gs;
  p.ngroups = ceil_div(p.tiles, gs);
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

void launch_set_state(int N, const double* wth, SpotRec* sp, float2* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, wth, sp, coef);
}

void launch_gather(const PixelSet& ps, int32_t* out, hipStream_t s) {
  if (ps.count <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(ceil_div(ps.count, 256)), dim3(256), 0, s, ps, out);
}

int pass_units_per_wave(int N) {
  const LaneMap lm = lane_map(N);
  return ceil_div(lm.U, kWaves);
}

template <int MAXU>
void launch_pass_u(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                   int e_width, hipStream_t s) {
  const dim3 grid(total_blocks), block(kBlock);
  switch (e_width) {
    case 8: hipLaunchKernelGGL((k_pass_batch<MAXU, 8>), grid, block, 0, s, jobs, descs, ndesc); break;
    case 16: hipLaunchKernelGGL((k_pass_batch<MAXU, 16>), grid, block, 0, s, jobs, descs, ndesc); break;
    case 25: hipLaunchKernelGGL((k_pass_batch<MAXU, 25>), grid, block, 0, s, jobs, descs, ndesc); break;
    default: hipLaunchKernelGGL((k_pass_batch<MAXU, 0>), grid, block, 0, s, jobs, descs, ndesc);
  }
}

void launch_pass_batch(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                       int max_units, int e_width, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  if (max_units <= 1) launch_pass_u<1>(jobs, descs, ndesc, total_blocks, e_width, s);
  else if (max_units <= 4) launch_pass_u<4>(jobs, descs, ndesc, total_blocks, e_width, s);
  else launch_pass_u<16>(jobs, descs, ndesc, total_blocks, e_width, s);
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
  p.sub = 1;
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
