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
#include "operand_layout.hpp"
#include "pass_tail.hpp"

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

// Doubled integer offsets of pixel p from the grid centre and Q = Lx^2+Ly^2
// (also as an integer, for the aperture test).
struct PixCoord {
  float Lx, Ly, Q;
  int32_t Qi;
};

__device__ __forceinline__ PixCoord pixel_coord(int32_t p, int W, int H) {
  const int32_t j = p / W;
  const int32_t i = p - j * W;
  const int32_t lx = 2 * i - (W - 1);
  const int32_t ly = 2 * j - (H - 1);
  PixCoord c;
  c.Lx = (float)lx;
  c.Ly = (float)ly;
  c.Qi = lx * lx + ly * ly;
  c.Q = (float)c.Qi;
  return c;
}

// Field of eq. (1) at one pixel over spots [n0, n1): sum A_n e^{i 2 pi (t_n + th_n)}.
// The spot loop index is uniform across the wave, so the records come in
// through scalar loads and feed the vector ALU as scalar operands.
__device__ __forceinline__ float2 backprop_field(const SpotRec* spg, int n0, int n1,
                                                 const PixCoord& c) {
  const HG_CONST SpotRec* sp = as_const(spg);
  float sr = 0.f, si = 0.f;
  // groups of four spots: the four records are requested together, so one
  // wait covers them
  int n = n0;
  for (; n + 3 < n1; n += 4) {
    float scx[4], scy[4], scz[4], sth[4], sA[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      scx[k] = sp[n + k].cx;
      scy[k] = sp[n + k].cy;
      scz[k] = sp[n + k].cz;
      sth[k] = sp[n + k].th;
      sA[k] = sp[n + k].A;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = fmaf(scx[k], c.Lx, fmaf(scy[k], c.Ly, fmaf(scz[k], c.Q, sth[k])));
      float sn, cs;
      sincos_turns(t, sn, cs);
      sr = fmaf(sA[k], cs, sr);
      si = fmaf(sA[k], sn, si);
    }
  }
  for (; n < n1; ++n) {
    const float t = fmaf(sp[n].cx, c.Lx, fmaf(sp[n].cy, c.Ly, fmaf(sp[n].cz, c.Q, sp[n].th)));
    float sn, cs;
    sincos_turns(t, sn, cs);
    sr = fmaf(sp[n].A, cs, sr);
    si = fmaf(sp[n].A, sn, si);
  }
  return make_float2(sr, si);
}

// The same sum with the spot records in LDS (chained launches, where the
// records change between passes of one launch): the four records of a group
// are read together (every lane the same address: broadcast reads).
__device__ __forceinline__ float2 backprop_field_lds(const SpotRec* recs, int n0, int n1,
                                                     const PixCoord& c) {
  float sr = 0.f, si = 0.f;
  int n = n0;
  for (; n + 3 < n1; n += 4) {
    float4 q[4];
    float sA[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      q[k] = *reinterpret_cast<const float4*>(&recs[n + k].cx);
      sA[k] = recs[n + k].A;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t = fmaf(q[k].x, c.Lx, fmaf(q[k].y, c.Ly, fmaf(q[k].z, c.Q, q[k].w)));
      float sn, cs;
      sincos_turns(t, sn, cs);
      sr = fmaf(sA[k], cs, sr);
      si = fmaf(sA[k], sn, si);
    }
  }
  for (; n < n1; ++n) {
    const float t =
        fmaf(recs[n].cx, c.Lx, fmaf(recs[n].cy, c.Ly, fmaf(recs[n].cz, c.Q, recs[n].th)));
    float sn, cs;
    sincos_turns(t, sn, cs);
    sr = fmaf(recs[n].A, cs, sr);
    si = fmaf(recs[n].A, sn, si);
  }
  return make_float2(sr, si);
}

// Mixed-precision back-propagation (eq. 1): the phase of each spot in FP32
// turns with theta folded in, t_n = phi_n(p) / 2 pi + theta_n, its cosine
// and sine from v_sin/v_cos; the two spots of a pair have their cosines,
// their sines and their amplitudes A_n rounded to FP16 and packed, and one
// FP16 dot product accumulated in FP32 (v_dot2_f32_f16) adds each part of
// the pair's terms A_n e^{i 2 pi t_n}: re += (cos_1, cos_2).(A_1, A_2),
// im += (sin_1, sin_2).(A_1, A_2).  A spot left without a partner is paired
// with a zero amplitude.
__device__ __forceinline__ void mx_pair(float t1, float a1, float t2, float a2, float& sr,
                                        float& si) {
  float sn1, cs1, sn2, cs2;
  sincos_turns(t1, sn1, cs1);
  sincos_turns(t2, sn2, cs2);
  const h2v_t a = to_h2(a1, a2);
  sr = __builtin_amdgcn_fdot2(to_h2(cs1, cs2), a, sr, false);
  si = __builtin_amdgcn_fdot2(to_h2(sn1, sn2), a, si, false);
}
__device__ __forceinline__ float turns_of(float cx, float cy, float cz, float th,
                                          const PixCoord& c) {
  return fmaf(cx, c.Lx, fmaf(cy, c.Ly, fmaf(cz, c.Q, th)));
}
// Records by scalar loads, four spots per wait.
__device__ __forceinline__ float2 backprop_field_mx(const SpotRec* spg, int n0, int n1,
                                                    const PixCoord& c) {
  const HG_CONST SpotRec* sp = as_const(spg);
  float sr = 0.f, si = 0.f;
  int n = n0;
  for (; n + 3 < n1; n += 4) {
    float t[4], A[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      t[k] = turns_of(sp[n + k].cx, sp[n + k].cy, sp[n + k].cz, sp[n + k].th, c);
      A[k] = sp[n + k].A;
    }
    mx_pair(t[0], A[0], t[1], A[1], sr, si);
    mx_pair(t[2], A[2], t[3], A[3], sr, si);
  }
  for (; n + 1 < n1; n += 2)
    mx_pair(turns_of(sp[n].cx, sp[n].cy, sp[n].cz, sp[n].th, c), sp[n].A,
            turns_of(sp[n + 1].cx, sp[n + 1].cy, sp[n + 1].cz, sp[n + 1].th, c), sp[n + 1].A,
            sr, si);
  if (n < n1)
    mx_pair(turns_of(sp[n].cx, sp[n].cy, sp[n].cz, sp[n].th, c), sp[n].A, 0.f, 0.f, sr, si);
  return make_float2(sr, si);
}
// Records from LDS (a pending pass's updated state).
__device__ __forceinline__ float2 backprop_field_mx_lds(const SpotRec* recs, int n0, int n1,
                                                        const PixCoord& c) {
  float sr = 0.f, si = 0.f;
  int n = n0;
  for (; n + 3 < n1; n += 4) {
    float t[4], A[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 q = *reinterpret_cast<const float4*>(&recs[n + k].cx);
      t[k] = turns_of(q.x, q.y, q.z, q.w, c);
      A[k] = recs[n + k].A;
    }
    mx_pair(t[0], A[0], t[1], A[1], sr, si);
    mx_pair(t[2], A[2], t[3], A[3], sr, si);
  }
  for (; n + 1 < n1; n += 2)
    mx_pair(turns_of(recs[n].cx, recs[n].cy, recs[n].cz, recs[n].th, c), recs[n].A,
            turns_of(recs[n + 1].cx, recs[n + 1].cy, recs[n + 1].cz, recs[n + 1].th, c),
            recs[n + 1].A, sr, si);
  if (n < n1)
    mx_pair(turns_of(recs[n].cx, recs[n].cy, recs[n].cz, recs[n].th, c), recs[n].A, 0.f, 0.f,
            sr, si);
  return make_float2(sr, si);
}

// ---------------------------------------------------------------- setup ---

// Row tables of the pupil for the random order (one block of kSetupThreads):
// rows[j] = pupil pixels in rows 0..j-1 (j <= H), rows[H + 1 + j] = the first
// pupil column of row j.  Each thread takes a run of consecutive rows; the
// runs' counts are scanned in thread order.
constexpr int kSetupThreads = 256;
__device__ void pupil_rows(const JobDev& jb) {
  __shared__ int32_t run_start[kSetupThreads];
  const int per = (jb.H + kSetupThreads - 1) / kSetupThreads;
  const int j0 = min(jb.H, (int)threadIdx.x * per), j1 = min(jb.H, j0 + per);
  int32_t cnt = 0;
  for (int j = j0; j < j1; ++j) {
    int32_t i0, i1;
    cnt += pupil_run(jb.W, jb.H, jb.ap_q, j, &i0, &i1);
    jb.rows[jb.H + 1 + j] = i0;
  }
  run_start[threadIdx.x] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t total = 0;
    for (int t = 0; t < kSetupThreads; ++t) {
      const int32_t c = run_start[t];
      run_start[t] = total;
      total += c;
    }
    jb.rows[jb.H] = total;  // = P
  }
  __syncthreads();
  int32_t before = run_start[threadIdx.x];
  for (int j = j0; j < j1; ++j) {
    jb.rows[j] = before;
    int32_t i0, i1;
    before += pupil_run(jb.W, jb.H, jb.ap_q, j, &i0, &i1);
  }
}

// The r-th pupil pixel in index order (r < P): the row j with
// rows[j] <= r < rows[j + 1], then the column.
__device__ __forceinline__ int32_t pupil_pixel(const JobDev& jb, uint32_t r) {
  const HG_GLOBAL int32_t* rows = as_global(jb.rows);
  int lo = 0, hi = jb.H;  // rows[lo] <= r < rows[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((uint32_t)rows[mid] <= r) lo = mid;
    else hi = mid;
  }
  return lo * jb.W + rows[jb.H + 1 + lo] + (int32_t)(r - (uint32_t)rows[lo]);
}

// Spot coefficients in FP64, rounded once to FP32; theta^0 from Philox;
// w = 1; pass counters cleared.  Spot values that are not finite, or
// amplitudes that are not positive, raise the argument status flag
// (device-resident inputs cannot be checked on the host).  The job's
// setup blocks after the first fill the Feistel round tables of a
// compressed job whose order is its own (a job of N = 0 builds a shared
// order's tables and pupil rows); all of them clear the exact sums.
__device__ void setup_part(const JobDev& jb, int lb, int nb) {
  if (lb == 0) {
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
    if (jb.rows && !jb.order_shared) pupil_rows(jb);
  }
  // the exact sums start at zero (every block of the job takes a share)
  for (int64_t k = (int64_t)lb * blockDim.x + threadIdx.x; k < jb.acc_len;
       k += (int64_t)nb * blockDim.x)
    jb.acc[k] = 0ull;
  if (lb > 0 && jb.compressed && !jb.order_shared) {
    const int total = kFeistelRounds << jb.h;
    const int stride = (nb - 1) * blockDim.x;
    for (int k = (lb - 1) * blockDim.x + threadIdx.x; k < total; k += stride)
      jb.tab[k] = feistel_table_entry(jb.order_key, k >> jb.h, (uint32_t)k & ((1u << jb.h) - 1u),
                                      jb.h);
  }
}

// ------------------------------------------------- factor tables ---

// Factor tables from FP64 phases (zero outside the grid and beyond N):
//   Fc  back-propagation B operand: part of F_n(col), col 16 cb + l%16,
//       spot n = 2 s + g/2 of K-step s;
//   Ga  G_n(row) for row 16 rb + l%16, spot 2 s + g/2 (forms the A operand);
//   Fn  forward B operand: part of F_n(col), spot 16 sb + l%16, column
//       2 cp + g/2 of column pair cp;
//   Gv  G_n(row) for spot 16 sb + l%16 and rows 16 rb + 4 g + r (V sums).
__device__ void sep_tables_part(const JobDev& jb, int lb, int nb) {
  const int W = jb.W, H = jb.H, N = jb.N;
  const int S16 = jb.mx_steps, Np = 16 * S16, KS = Np / 2;
  const int CB = jb.mx_cblocks, RB = jb.mx_rblocks, CP = 8 * CB;
  const int64_t nF = (int64_t)(16 * CB) * Np, total = nF + (int64_t)(16 * RB) * Np;
  const double lf = jb.lambda_mm * jb.focal_mm;
  const double lf2 = lf * jb.focal_mm;
  const double kxy = jb.pitch_mm / (2.0 * lf), kz = jb.pitch_mm * jb.pitch_mm / (4.0 * lf2);
  for (int64_t k = (int64_t)lb * kSetupThreads + threadIdx.x; k < total; k += (int64_t)nb * kSetupThreads) {
    if (k < nF) {
      const int col = (int)(k / Np), n = (int)(k % Np);
      float fr = 0.f, fi = 0.f;
      if (col < W && n < N) {
        const double L = (double)(2 * col - (W - 1));
        double t = jb.in.x[n] * kxy * L + jb.in.z[n] * kz * L * L;
        t -= rint(t);
        double s, c;
        sincospi(2.0 * t, &s, &c);
        fr = (float)c;
        fi = (float)s;
      }
      const int lgc = (n & 1) << 1, lgn = (col & 1) << 1;
      for (int p = 0; p < 2; ++p) {
        const float v = p ? fi : fr;
        jb.sepFc[op_index4(col >> 4, n >> 1, KS, (col & 15) + 16 * (lgc + p))] = v;
        jb.sepFn[op_index4(n >> 4, col >> 1, CP, (n & 15) + 16 * (lgn + p))] = v;
      }
    } else {
      const int64_t kk = k - nF;
      const int row = (int)(kk / Np), n = (int)(kk % Np);
      float2 g = make_float2(0.f, 0.f);
      if (row < H && n < N) {
        const double L = (double)(2 * row - (H - 1));
        double t = jb.in.y[n] * kxy * L + jb.in.z[n] * kz * L * L;
        t -= rint(t);
        double s, c;
        sincospi(2.0 * t, &s, &c);
        g = make_float2((float)c, (float)s);
      }
      const int lga = (n & 1) << 1;
      for (int p = 0; p < 2; ++p)
        jb.sepGa[op_index4(row >> 4, n >> 1, KS, (row & 15) + 16 * (lga + p))] = g;
      float2* Gv = reinterpret_cast<float2*>(jb.sepGv);
      Gv[op_index(row >> 4, n >> 4, S16, (n & 15) + 16 * ((row & 15) >> 2)) * 4 + (row & 3)] = g;
    }
  }
}

// Factor tables from FP64 phases:
//   Fc: back-propagation B operand, column 16 cb + l % 16, spots of step s;
//   Fn: forward B operand, spot 16 sb + l % 16, columns 16 cb + 4 (l / 16) + q;
//   Ga: G_n(j) for row 16 rb + l % 16, spots of step s (forms the A operand);
//   Gv: G_n(j) for spot 16 sb + l % 16, rows 16 rb + 4 (l / 16) + r (V sums).
// Entries outside the grid or beyond N are zero.
__device__ void mx_tables_part(const JobDev& jb, int lb, int nb) {
  const int W = jb.W, H = jb.H, N = jb.N;
  const int S16 = jb.mx_steps, Np = 16 * S16, CB = jb.mx_cblocks, RB = jb.mx_rblocks;
  const int64_t nF = (int64_t)(16 * CB) * Np, total = nF + (int64_t)(16 * RB) * Np;
  const double lf = jb.lambda_mm * jb.focal_mm;
  const double lf2 = lf * jb.focal_mm;
  const double kxy = jb.pitch_mm / (2.0 * lf), kz = jb.pitch_mm * jb.pitch_mm / (4.0 * lf2);
  uint32_t* Fc = reinterpret_cast<uint32_t*>(jb.mxFc);
  uint32_t* Fn = reinterpret_cast<uint32_t*>(jb.mxFn);
  float2* Ga = reinterpret_cast<float2*>(jb.mxGa);
  float2* Gv = reinterpret_cast<float2*>(jb.mxGv);
  for (int64_t k = (int64_t)lb * kSetupThreads + threadIdx.x; k < total; k += (int64_t)nb * kSetupThreads) {
    if (k < nF) {
      const int col = (int)(k / Np), n = (int)(k % Np);
      uint32_t v = 0u;
      if (col < W && n < N) {
        const double L = (double)(2 * col - (W - 1));
        double t = jb.in.x[n] * kxy * L + jb.in.z[n] * kz * L * L;
        t -= rint(t);
        double s, c;
        sincospi(2.0 * t, &s, &c);
        v = h2_bits((float)c, (float)s);
      }
      const int cb = col >> 4, cl = col & 15, s = n >> 4, nl = n & 15;
      Fc[fc_index(cb, s, S16, cl + 16 * (nl >> 2)) * 4 + (nl & 3)] = v;
      Fn[fn_index(s, cb, CB, nl + 16 * (cl >> 2)) * 4 + (cl & 3)] = v;
    } else {
      const int64_t kk = k - nF;
      const int row = (int)(kk / Np), n = (int)(kk % Np);
      float2 g = make_float2(0.f, 0.f);
      if (row < H && n < N) {
        const double L = (double)(2 * row - (H - 1));
        double t = jb.in.y[n] * kxy * L + jb.in.z[n] * kz * L * L;
        t -= rint(t);
        double s, c;
        sincospi(2.0 * t, &s, &c);
        g = make_float2((float)c, (float)s);
      }
      const int rb = row >> 4, rl = row & 15, s = n >> 4, nl = n & 15;
      Ga[g_index(rb, s, S16, rl + 16 * (nl >> 2)) * 4 + (nl & 3)] = g;
      Gv[g_index(rb, s, S16, nl + 16 * (rl >> 2)) * 4 + (rl & 3)] = g;
    }
  }
}

// The prologue of every job of a launch (PrologueSlice): its setup blocks,
// then the blocks that build the factor tables of its full-grid passes
// (separable FP32 or mixed precision).  The tables depend on the spot
// inputs alone, so both run in one launch.
__global__ __launch_bounds__(kSetupThreads) void k_prologue(const JobDev* __restrict__ jobs,
                                                           const PrologueSlice* __restrict__ slices,
                                                           int nslices) {
  const int si = find_desc(slices, nslices, blockIdx.x);
  const PrologueSlice& sl = slices[si];
  const JobDev& jb = jobs[sl.job];
  const int lb = blockIdx.x - sl.block_begin;
  if (lb < sl.setup_blocks) setup_part(jb, lb, sl.setup_blocks);
  else if (jb.mixed) mx_tables_part(jb, lb - sl.setup_blocks, sl.table_blocks);
  else sep_tables_part(jb, lb - sl.setup_blocks, sl.table_blocks);
}

// pi(k) for every k < P of each compressed job.  With an
// aperture the order runs over the P pupil pixels: pi(k) < P is the index
// of a pupil pixel in index order, mapped to its grid pixel.  With LDS, the Feistel
// tables (h <= 11: 48 KB) are staged in LDS; otherwise read from memory.
//
// The cycle walks have geometric lengths (mean 4^h / M), so a wave that gave
// each lane a fixed set of k would run for its longest walk.  Instead each
// wave takes a chunk of kPermChunk consecutive k and keeps its lanes busy:
// a lane whose walk has ended takes the next k of the chunk.
constexpr int kPermThreads = 512;
constexpr int kPermLdsHalfBits = 11;
constexpr int kPermChunk = 256;  // k per wave
constexpr int kPermPerThread = kPermChunk / 64;

template <bool LDS>
__global__ __launch_bounds__(kPermThreads) void k_perm_batch(const JobDev* __restrict__ jobs,
                                                             const JobSlice* __restrict__ slices,
                                                             int nslices) {
  // the tables as 16-byte words (6 << h is a multiple of 4 for h >= 1)
  constexpr int kTab4 = LDS ? (kFeistelRounds << kPermLdsHalfBits) / 4 : 1;
  constexpr int kTabLoads = (kTab4 + kPermThreads - 1) / kPermThreads;
  __shared__ uint4 tab_s4[kTab4];
  const int si = find_desc(slices, nslices, blockIdx.x);
  const JobDev& jb = jobs[slices[si].job];
  const int lb = blockIdx.x - slices[si].block_begin;
  const uint32_t* tab = jb.tab;
  if (LDS) {
    // every load of this thread is issued before the first is waited for
    const int total4 = (kFeistelRounds << jb.h) / 4;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(jb.tab), (short)0, total4 * 16, 0x00020000);
    uint4 v[kTabLoads];
#pragma unroll
    for (int i = 0; i < kTabLoads; ++i) {
      const int k = threadIdx.x + i * kPermThreads;
      const auto bits = __builtin_amdgcn_raw_buffer_load_b128(rsrc, k * 16, 0, 0);
      __builtin_memcpy(&v[i], &bits, sizeof(uint4));
    }
#pragma unroll
    for (int i = 0; i < kTabLoads; ++i) {
      const int k = threadIdx.x + i * kPermThreads;
      if (k < total4) tab_s4[k] = v[i];
    }
    __syncthreads();
    tab = reinterpret_cast<const uint32_t*>(tab_s4);
  }
  const uint32_t M = (uint32_t)jb.P;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t c0 = ((uint32_t)lb * (kPermThreads / 64) + wave) * kPermChunk;
  if (c0 >= M) return;  // whole wave
  const uint32_t c1 = min(c0 + (uint32_t)kPermChunk, M);
  // lane state: the k being walked and the latest point y of its walk
  uint32_t k = c0 + lane;
  bool active = k < c1;
  uint32_t y = active ? k : 0u;  // an idle lane walks from 0: its table reads stay in range
  uint32_t next = c0 + 64;  // next k of the chunk to hand out (uniform)
  const uint32_t cap = 1u << (2 * jb.h < 32 ? 2 * jb.h : 31);
  uint32_t steps = 0;
  while (__ballot(active) != 0ull) {
    y = feistel(y, tab, jb.h);
    ++steps;
    // the cycle of k contains k < M, so every walk ends within 4^h steps
    if (active && (y < M || steps >= cap)) {
      // (a walk always ends inside; the cap only bounds the loop)
      const uint32_t yk = y < M ? y : k;
      const int32_t p = jb.rows ? pupil_pixel(jb, yk) : (int32_t)yk;
      jb.perm[k] = p;
      active = false;
    }
    const uint64_t idle = __ballot(!active);
    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
    if (!active && next + r < c1) {
      k = next + r;
      y = k;
      steps = 0;
      active = true;
    }
    next += (uint32_t)__popcll(idle);
    if (next > c1) next = c1;
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
//  sums     the tile's per-spot sums (FP32, in a fixed order) are rounded
//           once to 64-bit fixed point and added into the row of the
//           tile's group with integer atomics;
//  tail     the block that completes a group moves the group row into the
//           pass total; the block that completes the last group scales the
//           total by 2^-shift / |Omega| and, when asked, applies the weight
//           update of eqs. (4)-(6).  A deferring pass stops after the group
//           moves and the next pass applies the update at its start.
// A tile's sums do not depend on which block computed it, and integer
// addition does not depend on order, so results depend neither on
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

// CHAIN: the spot records come from LDS (a.recs), the pixel index of this
// thread in the block's first sub-tile may come prefetched (has_pre, pre_p),
// and the block that completes the pass publishes the generation word after
// the update.  PEND: the records come from LDS too (a.recs: the state after
// the previous pass's deferred update), and the first pixel index may come
// prefetched as in CHAIN.  With a.defer the tiles add into the rows of the
// pass's total set and the pass ends there (no counting).
template <int MAXU, bool CHAIN = false, bool PEND = false, bool MX = false>
__device__ void pass_block(const PassCtx& a, unsigned* grab, bool has_pre = false,
                           int32_t pre_p = 0) {
  __shared__ float2 sw[kWaves][kTile];
  __shared__ float4 px[kTile];
  __shared__ float pui[kTile];
  __shared__ float2 red[kWaves * MAXU][64];
  __shared__ int done[kDoneList];
  __shared__ int owned[kMaxGroups];
  __shared__ int ndone, nowned, next_tile, flag;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = a.N;
  const LaneMap lm = lane_map(N);
  const int g = lane % lm.Lg, r = lane / lm.Lg;
  const SpotRec* __restrict__ sp = a.sp;
  if (threadIdx.x == 0) ndone = nowned = 0;
  constexpr bool lds_recs = CHAIN || PEND;

  float cx[MAXU], cy[MAXU], cz[MAXU];
#pragma unroll
  for (int k = 0; k < MAXU; ++k) {
    const int u = wave + k * kWaves;
    const int n = (u / lm.S) * lm.Lg + g;
    cx[k] = cy[k] = cz[k] = 0.f;
    if (u < lm.U && n < N) {
      if (lds_recs) {
        cx[k] = a.recs[n].cx;
        cy[k] = a.recs[n].cy;
        cz[k] = a.recs[n].cz;
      } else {
        const HG_GLOBAL SpotRec* rec = as_global(sp + n);
        cx[k] = rec->cx;
        cy[k] = rec->cy;
        cz[k] = rec->cz;
      }
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
            if (a.ap_q >= 0 || a.ill_a > 0.f) {
              const float wt = pupil_weight(c.Qi, c.Q, a.ap_q, a.ill_a);
              cs *= wt;
              sn *= wt;
            }
            rec = make_float4(c.Lx, c.Ly, c.Q, cs);
            ui = sn;
          }
          px[lane] = rec;
          pui[lane] = ui;
        }
        __syncthreads();
      } else {
        const int32_t p = ((CHAIN || PEND) && has_pre && tile == a.lb && st == 0)
                              ? pre_p
                              : (valid ? pixel_of(a.ps, q) : 0);
        // the next tile is asked for now; the answer is first needed after phase 1
        if (dynamic && st == a.plan.sub - 1 && threadIdx.x == 0) ticket = atomicAdd(grab, 1u);
        PixCoord c{0.f, 0.f, 0.f, 0};
        if (valid) c = pixel_coord(p, a.W, a.H);
        if constexpr (MX)
          sw[wave][lane] = PEND ? backprop_field_mx_lds(a.recs, n_lo, n_hi, c)
                                : backprop_field_mx(sp, n_lo, n_hi, c);
        else
          sw[wave][lane] = lds_recs ? backprop_field_lds(a.recs, n_lo, n_hi, c)
                                    : backprop_field(sp, n_lo, n_hi, c);
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
            if (a.ap_q >= 0 || a.ill_a > 0.f) {
              const float wt = pupil_weight(c.Qi, c.Q, a.ap_q, a.ill_a);
              ur *= wt;
              ui *= wt;
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
          // one unit per wave: four pixels per step, read from LDS
          // together, into two sums (with more units the registers go to
          // the units' sums).  Jobs of one unit per wave always run in the
          // MAXU = 1 launch of their round (LaunchSet), so a hologram sums
          // in the same order alone and beside holograms of more spots.
          float ar = vr[k], ai = vi[k], br = 0.f, bi = 0.f;
          int j = j0;
          if (MAXU == 1 && lm.R == 1) {
            // one replica (r = 0): the pixel loop is uniform across the
            // wave, so its counter and the LDS addresses stay scalar
            int ju = __builtin_amdgcn_readfirstlane(j0);
            const int ju1 = __builtin_amdgcn_readfirstlane(j1);
            for (; ju + 3 < ju1; ju += 4) {
              const float4 p0 = px[ju], p1 = px[ju + 1], p2 = px[ju + 2], p3 = px[ju + 3];
              const float u0 = pui[ju], u1 = pui[ju + 1], u2 = pui[ju + 2], u3 = pui[ju + 3];
              forward_term(cx[k], cy[k], cz[k], p0, u0, ar, ai);
              forward_term(cx[k], cy[k], cz[k], p1, u1, br, bi);
              forward_term(cx[k], cy[k], cz[k], p2, u2, ar, ai);
              forward_term(cx[k], cy[k], cz[k], p3, u3, br, bi);
            }
            j = ju;
          } else if (MAXU == 1)
          for (; j + 3 * lm.R < j1; j += 4 * lm.R) {
            const float4 p0 = px[j], p1 = px[j + lm.R], p2 = px[j + 2 * lm.R],
                         p3 = px[j + 3 * lm.R];
            const float u0 = pui[j], u1 = pui[j + lm.R], u2 = pui[j + 2 * lm.R],
                        u3 = pui[j + 3 * lm.R];
            forward_term(cx[k], cy[k], cz[k], p0, u0, ar, ai);
            forward_term(cx[k], cy[k], cz[k], p1, u1, br, bi);
            forward_term(cx[k], cy[k], cz[k], p2, u2, ar, ai);
            forward_term(cx[k], cy[k], cz[k], p3, u3, br, bi);
          }
          for (; j < j1; j += lm.R) forward_term(cx[k], cy[k], cz[k], px[j], pui[j], ar, ai);
          vr[k] = ar + br;
          vi[k] = ai + bi;
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
      // a deferring pass adds into a row of its total set, others into
      // their tile's group
      const int row = a.defer ? a.tot_row * kAccReplicas + tile % kAccReplicas
                              : kAccGroupRow0 + tile / a.plan.group_size;
      acc_add(a.acc, N, a.plan.shift, row, n, acc);
    }
    if (threadIdx.x == 0) {
      done[ndone++] = tile;
      next_tile = dynamic ? a.plan.blocks + (int)ticket : a.plan.tiles;
    }
    __syncthreads();
    tile = next_tile;
    if (ndone == kDoneList) {
      if (!a.defer) count_tiles(a, done, ndone, owned, &nowned);
      if (threadIdx.x == 0) ndone = 0;
      __syncthreads();
    }
  }
  // a deferring pass is complete when this launch ends: its tiles' sums are
  // not counted (deferring passes have one unit per wave and no chain)
  if constexpr (!CHAIN && MAXU == 1) {
    if (a.defer) return;
  }
  count_tiles(a, done, ndone, owned, &nowned);
  // the pass completes at most once, with this block's last group (the
  // update after the loop keeps the loop's registers free)
  bool last = false;
  for (int i = 0; i < nowned; ++i)
    if (tail_group(a, owned[i], &flag)) last = true;
  if (last) {
    // red (kWaves * MAXU * 64 float2) holds the N <= 256 MAXU spot fields
    tail_final(a, &red[0][0]);
    if (CHAIN) publish_gen(a);
  }
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
      // the next tile is asked for now (the counter's answer is first needed
      // after phase 1)
      if (dynamic && st == a.plan.sub - 1 && threadIdx.x == 0) ticket = atomicAdd(grab, 1u);
      PixCoord c{0.f, 0.f, 0.f, 0};
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
        if (a.ap_q >= 0 || a.ill_a > 0.f) {
          const float wt = pupil_weight(c.Qi, c.Q, a.ap_q, a.ill_a);
          ur *= wt;
          ui *= wt;
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
    if (lane < cnt)
      acc_add(a.acc, N, a.plan.shift, kAccGroupRow0 + tile / a.plan.group_size, n_lo + lane,
              rede[wave][lane]);
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
  bool last = false;  // (at most once, with this block's last group)
  for (int i = 0; i < nowned; ++i)
    if (tail_group(a, owned[i], &flag)) last = true;
  if (last) tail_final(a, &rede[0][0]);  // kWaves * MAXE >= N float2
}

static_assert(kPendMaxSpots <= kBlock, "a pending update takes one spot per thread");

// Batched pass launch: blocks [descs[i].block_begin, descs[i+1].block_begin)
// work on pass i.
// Occupancy target (waves per SIMD): eight for the two-sincos form (all
// blocks of a 1152^2 compressed pass resident with room to spare), six when
// 25 exponentials per lane stay in registers, two for the widest spot maps.
__device__ __forceinline__ void pass_ctx(PassCtx& a, const JobDev& jb, const PassDesc& d) {
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
  a.acc = jb.acc;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = d.from_phi;
  a.ill_a = jb.ill_a;
  a.ap_q = (d.ps.perm == nullptr && d.ps.idx == nullptr) ? jb.ap_q : -1;
}

// A pending pass (one unit per wave): the previous pass's update into LDS
// (with the pixel index of this thread in the block's first sub-tile
// requested before it, so that the two reads overlap), then the pass.
template <bool MX>
__device__ __forceinline__ void pending_pass(PassCtx& a, const JobDev& jb, const PassDesc& d) {
  __shared__ SpotRec recs[kPendMaxSpots];
  bool has_pre = false;
  int32_t pre_p = 0;
  if (!d.from_phi && a.lb < a.plan.tiles) {
    const int32_t q = a.lb * a.plan.sub * kTile + (int)(threadIdx.x & 63);
    pre_p = q < a.ps.count ? pixel_of(a.ps, q) : 0;
    has_pre = true;
  }
  apply_pending(jb, d, a.lb == 0, recs);
  a.recs = recs;
  if (!d.defer) a.pend_row = d.prev_row;
  pass_block<1, false, true, MX>(a, jb.grab + d.grab_slot, has_pre, pre_p);
}

template <int MAXU, int MAXE>
__global__ __launch_bounds__(kBlock, MAXU > 4 ? 2 : (MAXE > 16 ? 6 : 8)) void k_pass_batch(const JobDev* __restrict__ jobs,
                                                       const PassDesc* __restrict__ descs,
                                                       int ndesc) {
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const PassDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  PassCtx a;
  pass_ctx(a, jb, d);
  // the form depends on the job alone (its N, and whether it back-propagates),
  // so a hologram gives the same bits alone and in any batch
  if constexpr (MAXE > 0) {
    if (jb.shared_e && !d.from_phi) {
      pass_block_e<MAXE>(a, jb.grab + d.grab_slot);
      return;
    }
  }
  // deferred updates are only planned for launches of one unit per wave
  // (elsewhere the total row is 0 and no pass defers)
  if constexpr (MAXU == 1) {
    a.tot_row = d.tot_row;
    a.defer = d.defer;
  }
  if (d.pending) {
    if constexpr (MAXU == 1) {
      pending_pass<false>(a, jb, d);
    } else {
      if (a.lb == 0 && threadIdx.x == 0) jb.status[0] = 5;  // HG_EDEVICE
    }
    return;
  }
  pass_block<MAXU>(a, jb.grab + d.grab_slot);
}

// Compressed passes of mixed-precision jobs: the per-pixel pass with the
// back-propagation terms as FP16 products accumulated in FP32, two spots per
// dot product (backprop_field_mx); forward terms, sums, hand-off and update
// as in the FP32 form.
template <int MAXU>
__global__ __launch_bounds__(kBlock, MAXU > 4 ? 2 : 8) void k_pass_mx(const JobDev* __restrict__ jobs,
                                                                    const PassDesc* __restrict__ descs,
                                                                    int ndesc) {
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const PassDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  PassCtx a;
  pass_ctx(a, jb, d);
  if constexpr (MAXU == 1) {
    a.tot_row = d.tot_row;
    a.defer = d.defer;
  }
  if (d.pending) {
    if constexpr (MAXU == 1) {
      pending_pass<true>(a, jb, d);
    } else {
      if (a.lb == 0 && threadIdx.x == 0) jb.status[0] = 5;  // HG_EDEVICE
    }
    return;
  }
  pass_block<MAXU, false, false, true>(a, jb.grab + d.grab_slot);
}

// Compressed passes descs[0..npass) of one job in one cooperative launch;
// every pass has the same grid.  See kernels.hpp (chained compressed passes).
constexpr int kChainSpinLimit = 1 << 20;  // polls of one wait (about a second)
template <int MAXU>
__global__ __launch_bounds__(kBlock, MAXU > 4 ? 2 : 6) void k_pass_chain(
    const JobDev* __restrict__ jobs, const PassDesc* __restrict__ descs, int npass) {
  __shared__ SpotRec recs[kChainMaxSpots];
  __shared__ int stop;
  const JobDev& jb = jobs[descs[0].job];
  bool has_pre = false;
  int32_t pre_p = 0;
  for (int p = 0; p < npass; ++p) {
    __syncthreads();  // the previous pass's use of LDS is over
    if (p > 0) {
      if (threadIdx.x == 0) {
        const unsigned* g = jb.gen + (blockIdx.x % kGenCopies) * kCounterStride;
        int spins = 0;
        while (__hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)p &&
               ++spins < kChainSpinLimit)
          __builtin_amdgcn_s_sleep(2);
        stop = spins >= kChainSpinLimit;
        if (stop) jb.status[0] = 5;  // HG_EDEVICE: the previous pass did not complete
      }
      __syncthreads();
      if (stop) return;
    }
    // the spot state of this pass (written by the previous pass's update)
    load_recs_dev(jb.sp, jb.N, recs);
    __syncthreads();
    const PassDesc& d = descs[p];
    PassCtx a;
    a.sp = jb.sp;
    a.coef = jb.coef;
    a.N = jb.N;
    a.W = jb.W;
    a.H = jb.H;
    a.ps = d.ps;
    a.phi = jb.phi;
    a.plan = d.plan;
    a.lb = blockIdx.x;
    a.partial = jb.partial;
    a.gpart = jb.gpart;
    a.acc = jb.acc;
    a.counters = jb.counters;
    a.inv_count = d.inv_count;
    a.V = d.V;
    a.status = jb.status;
    a.update = d.update;
    a.from_phi = 0;
    a.ill_a = jb.ill_a;
    a.ap_q = (d.ps.perm == nullptr && d.ps.idx == nullptr) ? jb.ap_q : -1;
    a.chain = 1;
    a.recs = recs;
    a.gen = jb.gen;
    a.gen_next = (unsigned)(p + 1);
    pass_block<MAXU, true>(a, jb.grab + d.grab_slot, has_pre, pre_p);
    // the pixel index of the next pass's first sub-tile, requested while the
    // block waits for this pass to complete
    if (p + 1 < npass) {
      const PassDesc& dn = descs[p + 1];
      const int32_t q = blockIdx.x * dn.plan.sub * kTile + (int)(threadIdx.x & 63);
      pre_p = q < dn.ps.count ? pixel_of(dn.ps, q) : 0;
      has_pre = true;
    }
  }
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
  const float phi = atan2f(S.y, S.x);
  as_global_mut(d.out)[q] = phi;
  // the job's final hologram (over all pixels, q = p) with an SLM table
  if (jb.gray) store_gray(jb.gray, q, jb.gray_bits, gray_level(phi, jb.lut, jb.lut_levels));
}

// -------------------------------------------------------------- SLM output ---

// Gray image of a hologram, four consecutive pixels per thread (one 4- or
// 8-byte store where the image is aligned for it).
constexpr int kGrayThreads = 256;
__global__ __launch_bounds__(kGrayThreads) void k_phase_to_gray(const float* __restrict__ phi,
                                                                int64_t count,
                                                                const uint16_t* __restrict__ lut,
                                                                int levels, int bits,
                                                                void* __restrict__ gray) {
  const int64_t p0 = 4 * ((int64_t)blockIdx.x * kGrayThreads + threadIdx.x);
  if (p0 >= count) return;
  if (p0 + 3 < count) {
    const HG_GLOBAL float* src = as_global(phi) + p0;
    const float v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
    const uint32_t g0 = gray_level(v0, lut, levels), g1 = gray_level(v1, lut, levels),
                   g2 = gray_level(v2, lut, levels), g3 = gray_level(v3, lut, levels);
    if (bits == 8 && (reinterpret_cast<uintptr_t>(gray) & 3) == 0) {
      *as_global_mut(reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(gray) + p0)) =
          g0 | (g1 << 8) | (g2 << 16) | (g3 << 24);
      return;
    }
    if (bits == 16 && (reinterpret_cast<uintptr_t>(gray) & 3) == 0) {
      HG_GLOBAL uint32_t* q = as_global_mut(reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(gray) + p0));
      q[0] = g0 | (g1 << 16);
      q[1] = g2 | (g3 << 16);
      return;
    }
  }
  for (int64_t p = p0; p < p0 + 4 && p < count; ++p)
    store_gray(gray, p, bits, gray_level(as_global(phi)[p], lut, levels));
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
// With a pupil, e^{i Phi} is weighted by A = exp(-Q ill_a) and by 0 outside
// the aperture (Q = Lx^2 + Ly^2 > ap_q, ap_q >= 0).
__global__ __launch_bounds__(kMetricThreads) void k_metric_rows(
    const double2* __restrict__ Ex, const double2* __restrict__ Ey, int N, int W, int H,
    const float* __restrict__ phi, int32_t ap_q, double ill_a, double2* __restrict__ partial) {
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
          if (ap_q >= 0 || ill_a > 0.0) {
            const int64_t lx = 2 * (int64_t)(i0 + k) - (W - 1), ly = 2 * (int64_t)j - (H - 1);
            const int64_t Q = lx * lx + ly * ly;
            const double wt = (ap_q >= 0 && Q > ap_q) ? 0.0 : (ill_a > 0.0 ? exp(-(double)Q * ill_a) : 1.0);
            c *= wt;
            s *= wt;
          }
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

int sum_shift(int64_t pixels) {
  int b = 0;  // ceil(log2(pixels))
  while ((int64_t(1) << b) < pixels) ++b;
  return 62 - b;
}

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
  p.shift = sum_shift(count);
  return p;
}

int prologue_setup_blocks(const JobDev& j) {
  if (!j.compressed || j.order_shared) return 1;
  const int total = kFeistelRounds << j.h;
  const int b = ceil_div(total, 256 * 4);
  return 1 + (b > 64 ? 64 : b);
}

int prologue_table_blocks(const JobDev& j) {
  if (!j.sepFc && !j.mxFc) return 0;  // no matrix-core passes
  const int64_t total = (int64_t)16 * (j.mx_cblocks + j.mx_rblocks) * 16 * j.mx_steps;
  return ceil_div(total, kSetupThreads);
}

void launch_prologue(const JobDev* jobs, const PrologueSlice* slices, int nslices,
                     int total_blocks, hipStream_t s) {
  if (nslices <= 0 || total_blocks <= 0) return;
  hipLaunchKernelGGL(k_prologue, dim3(total_blocks), dim3(kSetupThreads), 0, s, jobs, slices,
                     nslices);
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

void launch_pass_mx(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                    int max_units, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  const dim3 grid(total_blocks), block(kBlock);
  if (max_units <= 1) hipLaunchKernelGGL(k_pass_mx<1>, grid, block, 0, s, jobs, descs, ndesc);
  else if (max_units <= 4) hipLaunchKernelGGL(k_pass_mx<4>, grid, block, 0, s, jobs, descs, ndesc);
  else hipLaunchKernelGGL(k_pass_mx<16>, grid, block, 0, s, jobs, descs, ndesc);
}

namespace {
template <int MAXU>
int chain_capacity_u() {
  static int cached = -1;  // per process: the device is the same for every call
  if (cached < 0) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pass_chain<MAXU>, kBlock, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cached = per_cu * cus;
  }
  return cached;
}
template <int MAXU>
hipError_t launch_chain_u(const JobDev* jobs, const PassDesc* descs, int npass, int blocks,
                          hipStream_t s) {
  void* args[] = {(void*)&jobs, (void*)&descs, (void*)&npass};
  return hipLaunchCooperativeKernel((const void*)k_pass_chain<MAXU>, dim3(blocks), dim3(kBlock),
                                    args, 0, s);
}
}  // namespace

int pass_chain_capacity(int max_units) {
  if (max_units <= 1) return chain_capacity_u<1>();
  if (max_units <= 4) return chain_capacity_u<4>();
  return chain_capacity_u<16>();
}

hipError_t launch_pass_chain(const JobDev* jobs, const PassDesc* descs, int npass, int blocks,
                             int max_units, hipStream_t s) {
  if (npass <= 0 || blocks <= 0) return hipSuccess;
  if (max_units <= 1) return launch_chain_u<1>(jobs, descs, npass, blocks, s);
  if (max_units <= 4) return launch_chain_u<4>(jobs, descs, npass, blocks, s);
  return launch_chain_u<16>(jobs, descs, npass, blocks, s);
}

int backprop_blocks(int32_t count) { return ceil_div(count, kBlock); }


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

void launch_phase_to_gray(const float* phi, int64_t count, const uint16_t* lut, int levels,
                          int bits, void* gray, hipStream_t s) {
  if (count <= 0) return;
  const int64_t blocks = ceil_div(count, (int64_t)4 * kGrayThreads);
  hipLaunchKernelGGL(k_phase_to_gray, dim3((unsigned)blocks), dim3(kGrayThreads), 0, s, phi,
                     count, lut, levels, bits, gray);
}

void launch_metric_rows(const double2* Ex, const double2* Ey, int N, int W, int H,
                        const float* phi, int32_t ap_q, double ill_a, double2* partial,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_metric_rows, dim3(metric_blocks(H)), dim3(kMetricThreads), 0, s, Ex, Ey,
                     N, W, H, phi, ap_q, ill_a, partial);
}

void launch_metric_reduce(const double2* partial, int nblk, int N, double inv_count,
                          double2* V_out, hipStream_t s) {
  hipLaunchKernelGGL(k_metric_reduce, dim3(ceil_div(N, 128)), dim3(128), 0, s, partial, nblk, N,
                     inv_count, V_out);
}

}  // namespace hg
