// Mixed-precision passes for gfx950: the separable recast of eqs. (1)-(3)
// on the matrix cores with FP16 operands and FP32 accumulation.
//
// With doubled pixel offsets the phase of eq. (2) splits into a part in the
// column and a part in the row, so e^{i phi_n(i,j)} = F_n(i) G_n(j).  The
// back-propagated field of eq. (1) over the whole grid is then the complex
// matrix product S = B F with B_n(j) = C_n G_n(j), C_n = A_n e^{i theta_n},
// and the forward sums of eq. (3) are V_n = (1/|Omega|) sum_j conj(G_n(j))
// T[j][n] with T = U conj(F)^T, U(j,i) = e^{i Phi(i,j)} on the pixel set and
// 0 elsewhere.  Both products run as v_mfma_f32_16x16x32_f16: a complex
// product is a real one with K = 2 Np, the real and imaginary parts of each
// spot interleaved along K.
//
// Precision: F and B are rounded to FP16 (relative error <= 2^-11 per
// operand), products and sums are FP32, partials are added across tiles with
// compensated (Neumaier) FP32 sums, and the weight update is FP32.  FP64 is
// used only for the factor tables (setup).  The full-grid pass after the
// compressed passes applies the last one's deferred update at its start and
// defers its own to the final hologram, adding its sums exactly (64-bit
// fixed point) into its total set.
#include <math.h>

#include "device_common.hpp"
#include "device_math.hpp"
#include "kernels.hpp"
#include "operand_layout.hpp"
#include "pass_tail.hpp"

namespace hg {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

// (lo, hi) rounded to nearest FP16, packed into one dword.
__device__ __forceinline__ uint32_t pack_h2(float lo, float hi) { return h2_bits(lo, hi); }

__device__ __forceinline__ f4_t mfma16(const u4_t& a, const u4_t& b, const f4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8_t, a),
                                                __builtin_bit_cast(h8_t, b), c, 0, 0, 0);
}

// For a dword holding the half pair (re, im) of z, the pair of -i z: (im, -re).
__device__ __forceinline__ uint32_t times_minus_i(uint32_t v) {
  return ((v >> 16) | (v << 16)) ^ 0x80000000u;
}


// Compensated (Neumaier) FP32 accumulation: the sum is s + c.
__device__ __forceinline__ void ksum(float& s, float& c, float x) {
  const float t = s + x;
  c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// Compensated (Neumaier) sum over rows k0 + s, k0 + s + S, ... (< row_end)
// of column n of a float2 array: (re, im, comp re, comp im).  kMxBatch
// loads are in flight before any is used; rows past row_end fall outside
// the buffer resource and load as zero.
constexpr int kMxBatch = 12;
constexpr int kMxSteps = 2;  // K-steps of the back-propagation product per load group
constexpr int kMxCB = kMxTileW / 16;  // 16-column blocks per tile
__device__ __forceinline__ float4 column_ksum(const ColumnSrc& src, int n, int s, int k0,
                                              int k1, int S) {
  float sr = 0.f, si = 0.f, cr = 0.f, ci = 0.f;
  const int step = S * src.N * (int)sizeof(float2);
  int off = ((k0 + s) * src.N + n) * (int)sizeof(float2);
  for (int k = k0; k < k1; k += S * kMxBatch, off += kMxBatch * step) {
    float2 v[kMxBatch];
#pragma unroll
    for (int b = 0; b < kMxBatch; ++b) {
      const auto bits =
          __builtin_amdgcn_raw_buffer_load_b64(src.rsrc, off + b * step, 0, kDeviceScope);
      __builtin_memcpy(&v[b], &bits, sizeof(float2));
    }
#pragma unroll
    for (int b = 0; b < kMxBatch; ++b) {
      ksum(sr, cr, v[b].x);
      ksum(si, ci, v[b].y);
    }
  }
  return make_float4(sr, si, cr, ci);
}

// The slices' compensated sums of spot lane c, added in slice order.
__device__ __forceinline__ float4 combine_slices(const float4* part, int Npad, int S, int c) {
  float4 t = part[c];
  for (int k = 1; k < S; ++k) {
    const float4 v = part[k * Npad + c];
    ksum(t.x, t.z, v.x);
    ksum(t.y, t.w, v.y);
    t.z += v.z;
    t.w += v.w;
  }
  return t;
}

// Cross-tile reduction and weight update of a mixed-precision pass: the last
// block of each group of tiles adds its group's partials (tile order,
// compensated FP32) and stores the compensated sums rounded to FP32; the
// last group adds those (group order, compensated), scales by 1 / |Omega|
// and, when asked, applies eqs. (4)-(6) in FP32.  The same last-arriver
// hand-off as the FP32 passes; thread (c, s) takes spot lane c of Npad and
// slice s of S.  recs: the state the pass used, when it applied a pending
// update into LDS (else the spot records).
__device__ void mx_tail(const JobDev& jb, const MxDesc& d, int lb, const SpotRec* recs) {
  __shared__ int last;
  __shared__ float wsum[kWaves];
  __shared__ float4 part[kBlock];
  const int N = jb.N;
  int Npad = 1;
  while (Npad < N && Npad < kBlock) Npad <<= 1;
  const int S = kBlock / Npad, c = threadIdx.x % Npad, s = threadIdx.x / Npad;
  const int g = lb / d.plan.group_size;
  const int t0 = g * d.plan.group_size;
  const int t1 = min(t0 + d.plan.group_size, d.plan.tiles);
  float2* gsum = reinterpret_cast<float2*>(jb.gpart);
  if (!arrive_last(&jb.counters[g * kCounterStride], (unsigned)(t1 - t0), &last)) return;
  const ColumnSrc psrc = column_src(jb.partial, t1, N);
  for (int n0 = 0; n0 < N; n0 += Npad) {
    const int n = n0 + c;
    part[threadIdx.x] = n < N ? column_ksum(psrc, n, s, t0, t1, S)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    if (s == 0 && n < N) {
      const float4 t = combine_slices(part, Npad, S, c);
      store_dev(gsum + (int64_t)g * N + n, make_float2(t.x + t.z, t.y + t.w));
    }
    __syncthreads();
  }
  if (!arrive_last(&jb.counters[d.plan.ngroups * kCounterStride], (unsigned)d.plan.ngroups, &last))
    return;
  // this thread's first record, requested before the sums are read (as
  // eight words: a record copied whole into a local would take a stack slot)
  constexpr int kRecWords = (int)(sizeof(SpotRec) / sizeof(float));
  float pre[kRecWords];
#pragma unroll
  for (int k = 0; k < kRecWords; ++k) pre[k] = 0.f;
  if (d.update && s == 0 && c < N) {
    if (recs) {
      const float* q = reinterpret_cast<const float*>(recs + c);
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) pre[k] = q[k];
    } else {
      const HG_GLOBAL float* q = as_global(reinterpret_cast<const float*>(jb.sp + c));
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) pre[k] = q[k];
    }
  }
  const ColumnSrc gsrc = column_src(gsum, d.plan.ngroups, N);
  float msum = 0.f;
  for (int n0 = 0; n0 < N; n0 += Npad) {
    const int n = n0 + c;
    part[threadIdx.x] = n < N ? column_ksum(gsrc, n, s, 0, d.plan.ngroups, S)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    if (s == 0 && n < N) {
      const float4 t = combine_slices(part, Npad, S, c);
      const float vr = (t.x + t.z) * d.inv_count, vi = (t.y + t.w) * d.inv_count;
      d.V[n] = make_double2((double)vr, (double)vi);
      msum += sqrtf(vr * vr + vi * vi);
    }
    __syncthreads();
  }
  // the counters are ready for the next pass (kernel end orders these writes)
  for (int k = threadIdx.x; k <= d.plan.ngroups; k += kBlock) jb.counters[k * kCounterStride] = 0u;
  // the previous pass's total set, which every block has read, is cleared
  if (d.pending) {
    HG_GLOBAL unsigned long long* q =
        as_global_mut(jb.acc + (int64_t)d.prev_row * kAccReplicas * N * kAccSpotWords);
    for (int k = threadIdx.x; k < kAccReplicas * N * kAccSpotWords; k += kBlock)
      __hip_atomic_store(q + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!d.update) return;
  for (int off = 32; off > 0; off >>= 1) msum += __shfl_xor(msum, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = msum;
  __syncthreads();
  float total = wsum[0];
  for (int w = 1; w < kWaves; ++w) total += wsum[w];
  const float mean = total / (float)N;
  if (s != 0) return;
  // eqs. (4)-(6) in FP32: w_n <- w_n mean / |V_n|, theta_n <- arg V_n, A_n = a_n^0 w_n.
  for (int n = c; n < N; n += Npad) {
    const double2 vd = d.V[n];  // written above by this same thread
    const float vr = (float)vd.x, vi = (float)vd.y;
    const float mag = sqrtf(vr * vr + vi * vi);
    float f[kRecWords];
    if (n == c) {
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) f[k] = pre[k];
    } else if (recs) {
      const float* q = reinterpret_cast<const float*>(recs + n);
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) f[k] = q[k];
    } else {
      const HG_GLOBAL float* q = as_global(reinterpret_cast<const float*>(jb.sp + n));
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) f[k] = q[k];
    }
    SpotRec r;
    __builtin_memcpy(&r, f, sizeof(r));
    const float w = r.w * (mean / mag);
    if (!(mag > 0.f) || !isfinite(w)) {
      jb.status[0] = 4;  // HG_ENUMERIC
      if (recs) jb.sp[n] = r;  // the state this pass used
      continue;
    }
    r.w = w;
    r.A = w * r.a0;
    r.th = atan2f(vi, vr) * 0.15915494309189535f;
    jb.sp[n] = r;
    const float Am = r.A / mag;  // C_n = A_n e^{i theta_n} = A_n V_n / |V_n|
    jb.coef[n] = make_float2(Am * vr, Am * vi);
  }
}

// Operands of kMxSteps K-steps of S = B F for one wave: G of its rows and
// the F operand of the tile's 16-column blocks (steps past the last are
// loaded clamped and not used).
struct MxOps {
  f4_t ga[kMxSteps][2];
  u4_t fc[kMxSteps][kMxCB];
};
__device__ __forceinline__ void mx_load(MxOps& o, const f4_t* Ga, const u4_t* Fc, int rb, int tx,
                                        int s0, int S16, int lane) {
#pragma unroll
  for (int q = 0; q < kMxSteps; ++q) {
    const int s = min(s0 + q, S16 - 1);
    const int64_t gi = g_index(rb, s, S16, lane) * 2;
    o.ga[q][0] = as_global(Ga)[gi];
    o.ga[q][1] = as_global(Ga)[gi + 1];
#pragma unroll
    for (int t = 0; t < kMxCB; ++t) o.fc[q][t] = as_global(Fc)[fc_index(kMxCB * tx + t, s, S16, lane)];
  }
}
// A operands conj(B) (real part) and i conj(B) (imaginary part), B = C G.
__device__ __forceinline__ void mx_mma(const MxOps& o, const float2* cs, int s0, int S16, int lg,
                                       f4_t* sr, f4_t* si) {
#pragma unroll
  for (int q = 0; q < kMxSteps; ++q) {
    if (s0 + q < S16) {
      const f4_t g01 = o.ga[q][0], g23 = o.ga[q][1];
      const int n0 = 16 * (s0 + q) + 4 * lg;
      const float2 c0 = cs[n0], c1 = cs[n0 + 1], c2 = cs[n0 + 2], c3 = cs[n0 + 3];
      const float br0 = c0.x * g01[0] - c0.y * g01[1], bi0 = c0.x * g01[1] + c0.y * g01[0];
      const float br1 = c1.x * g01[2] - c1.y * g01[3], bi1 = c1.x * g01[3] + c1.y * g01[2];
      const float br2 = c2.x * g23[0] - c2.y * g23[1], bi2 = c2.x * g23[1] + c2.y * g23[0];
      const float br3 = c3.x * g23[2] - c3.y * g23[3], bi3 = c3.x * g23[3] + c3.y * g23[2];
      const u4_t ar = {pack_h2(br0, -bi0), pack_h2(br1, -bi1), pack_h2(br2, -bi2),
                       pack_h2(br3, -bi3)};
      const u4_t ai = {pack_h2(bi0, br0), pack_h2(bi1, br1), pack_h2(bi2, br2),
                       pack_h2(bi3, br3)};
#pragma unroll
      for (int t = 0; t < kMxCB; ++t) {
        sr[t] = mfma16(ar, o.fc[q][t], sr[t]);
        si[t] = mfma16(ai, o.fc[q][t], si[t]);
      }
    }
  }
}

// One kMxTile x kMxTileW tile per block; wave w owns rows 16 w .. 16 w + 15
// of the tile, so each wave's products, normalisation and forward operands
// stay within the wave until the tile's partial V is formed.
template <int MODE>
__global__ __launch_bounds__(kBlock, 3) void k_mx_pass(const JobDev* __restrict__ jobs,
                                                    const MxDesc* __restrict__ descs, int ndesc) {
  extern __shared__ float2 cs[];                     // [Np] C_n = A_n e^{i theta_n}
  __shared__ uint32_t us[kWaves][16][kMxTileW + 4];  // u of each wave's rows (half pairs)
  __shared__ SpotRec recs[kPendMaxSpots];            // pending: the updated records
  __shared__ float2 red[kWaves][64];
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const MxDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  const int W = jb.W, H = jb.H, N = jb.N, S16 = jb.mx_steps, CB = jb.mx_cblocks;
  const int lb = blockIdx.x - d.block_begin;
  const int tx = lb % d.tiles_x, ty = lb / d.tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int rb = 4 * ty + wave;  // 16-row block of this wave
  const int row0 = 16 * rb, col0 = kMxTileW * tx;

  f4_t sr[kMxCB], si[kMxCB];
#pragma unroll
  for (int t = 0; t < kMxCB; ++t) sr[t] = si[t] = f4_t{0.f, 0.f, 0.f, 0.f};

  if (MODE != kMxFromPhi) {
    if (d.pending) {
      // the previous pass's deferred update, C_n formed as its tail would
      apply_pending(jb, d, lb == 0, recs, cs);
      for (int n = N + threadIdx.x; n < 16 * S16; n += kBlock) cs[n] = make_float2(0.f, 0.f);
    } else {
      for (int n = threadIdx.x; n < 16 * S16; n += kBlock) {
        float2 c = make_float2(0.f, 0.f);
        if (n < N) {
          const HG_GLOBAL float* f = as_global(reinterpret_cast<const float*>(jb.coef + n));
          c = make_float2(f[0], f[1]);
        }
        cs[n] = c;
      }
    }
    __syncthreads();
    // S = B F in groups of kMxSteps K-steps, the next group's operands
    // loaded before the current group's products.
    const u4_t* Fc = reinterpret_cast<const u4_t*>(jb.mxFc);
    const f4_t* Ga = reinterpret_cast<const f4_t*>(jb.mxGa);
    MxOps P, Q;
    mx_load(P, Ga, Fc, rb, tx, 0, S16, lane);
    for (int s0 = 0; s0 < S16; s0 += 2 * kMxSteps) {
      if (s0 + kMxSteps < S16) mx_load(Q, Ga, Fc, rb, tx, s0 + kMxSteps, S16, lane);
      mx_mma(P, cs, s0, S16, lg, sr, si);
      if (s0 + kMxSteps < S16) {
        if (s0 + 2 * kMxSteps < S16) mx_load(P, Ga, Fc, rb, tx, s0 + 2 * kMxSteps, S16, lane);
        mx_mma(Q, cs, s0 + kMxSteps, S16, lg, sr, si);
      }
    }
  }

  if (MODE == kMxFinal) {
    HG_GLOBAL float* out = as_global_mut(d.out);
#pragma unroll
    for (int t = 0; t < kMxCB; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + 4 * lg + r, col = col0 + 16 * t + lr;
        if (row < H && col < W) {
          const float phi = atan2f(si[t][r], sr[t][r]);
          const int64_t p = (int64_t)row * W + col;
          out[p] = phi;
          // the SLM's gray image of the final hologram
          if (jb.gray) store_gray(jb.gray, p, jb.gray_bits, gray_level(phi, jb.lut, jb.lut_levels));
        }
      }
    return;
  }

  // u = e^{i Phi} on every pixel within the pupil (the matrix-core passes
  // cover the whole grid), 0 elsewhere, weighted by the illumination, as
  // half pairs in LDS.
  const bool pupil = jb.ap_q >= 0 || jb.ill_a > 0.f;
#pragma unroll
  for (int t = 0; t < kMxCB; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + 4 * lg + r, col = col0 + 16 * t + lr;
      uint32_t uh = 0u;
      if (row < H && col < W) {
        const int32_t p = row * W + col;
        float wt = 1.f;
        if (pupil) {
          const int32_t lx = 2 * col - (W - 1), ly = 2 * row - (H - 1);
          const int32_t Qi = lx * lx + ly * ly;
          wt = pupil_weight(Qi, (float)Qi, jb.ap_q, jb.ill_a);
        }
        if (wt != 0.f) {  // outside the aperture: never in the set
          float ur = 1.f, ui = 0.f;
          if (MODE == kMxFromPhi) {
            sincos_turns(as_global(jb.phi)[p] * 0.15915494309189535f, ui, ur);
          } else {
            const float m2 = sr[t][r] * sr[t][r] + si[t][r] * si[t][r];
            if (m2 > 0.f) {
              const float inv = rsqrtf(m2);
              ur = sr[t][r] * inv;
              ui = si[t][r] * inv;
            }
          }
          if (pupil) {
            ur *= wt;
            ui *= wt;
          }
          uh = pack_h2(ur, ui);
        }
      }
      us[wave][4 * lg + r][16 * t + lr] = uh;
    }
  __syncthreads();

  // T = U conj(F)^T for this wave's 16 rows, 64 spots per chunk, and the
  // tile's partial V_n = sum_j conj(G_n(j)) T[j][n].  The chunk's F operands
  // are loaded before its products.
  u4_t ua[kMxCB], ub[kMxCB];
#pragma unroll
  for (int ks = 0; ks < kMxCB; ++ks) {
    const uint32_t* src = &us[wave][lr][16 * ks + 4 * lg];
    ua[ks] = u4_t{src[0], src[1], src[2], src[3]};
    ub[ks] = u4_t{times_minus_i(src[0]), times_minus_i(src[1]), times_minus_i(src[2]),
                  times_minus_i(src[3])};
  }
  const u4_t* Fn = reinterpret_cast<const u4_t*>(jb.mxFn);
  const f4_t* Gv = reinterpret_cast<const f4_t*>(jb.mxGv);
  for (int sb0 = 0; sb0 < S16; sb0 += 4) {
    f4_t tr[4], ti[4];
    u4_t fn[kMxCB][4];
#pragma unroll
    for (int ks = 0; ks < kMxCB; ++ks)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        fn[ks][u] = as_global(Fn)[fn_index(min(sb0 + u, S16 - 1), kMxCB * tx + ks, CB, lane)];
#pragma unroll
    for (int u = 0; u < 4; ++u) tr[u] = ti[u] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kMxCB; ++ks)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (sb0 + u < S16) {
          tr[u] = mfma16(ua[ks], fn[ks][u], tr[u]);
          ti[u] = mfma16(ub[ks], fn[ks][u], ti[u]);
        }
      }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float vr = 0.f, vi = 0.f;
      if (sb0 + u < S16) {
        const int64_t gv = g_index(rb, sb0 + u, S16, lane) * 2;
        const f4_t g01 = as_global(Gv)[gv], g23 = as_global(Gv)[gv + 1];
        const float gr[4] = {g01[0], g01[2], g23[0], g23[2]};
        const float gi[4] = {g01[1], g01[3], g23[1], g23[3]};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          vr = fmaf(gr[r], tr[u][r], fmaf(gi[r], ti[u][r], vr));
          vi = fmaf(gr[r], ti[u][r], fmaf(-gi[r], tr[u][r], vi));
        }
      }
      vr += __shfl_xor(vr, 16);
      vi += __shfl_xor(vi, 16);
      vr += __shfl_xor(vr, 32);
      vi += __shfl_xor(vi, 32);
      if (lg == 0) red[wave][16 * u + lr] = make_float2(vr, vi);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      const int n = 16 * sb0 + threadIdx.x;
      if (n < N) {
        float2 v = red[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
          v.x += red[w][threadIdx.x].x;
          v.y += red[w][threadIdx.x].y;
        }
        if (d.defer)
          acc_add(jb.acc, N, d.plan.shift, d.tot_row * kAccReplicas + lb % kAccReplicas, n, v);
        else
          store_dev(jb.partial + (int64_t)lb * N + n, v);
      }
    }
    __syncthreads();
  }
  // a deferring pass is complete when this launch ends (the final hologram
  // applies its update)
  if (d.defer) return;
  mx_tail(jb, d, lb, d.pending ? recs : nullptr);
}

}  // namespace

PassPlan plan_mx(int W, int H) {
  PassPlan p;
  p.tiles = ceil_div(W, kMxTileW) * ceil_div(H, kMxTile);
  p.sub = 1;
  // compensated FP32 sums, except in a pass that defers its update: exact
  // fixed-point sums into its total set (every term has magnitude <= 1)
  p.shift = sum_shift((int64_t)W * H);
  p.blocks = p.tiles;
  int gs = 1;
  while (gs * gs < p.blocks) ++gs;
  p.group_size = gs;
  p.ngroups = ceil_div(p.blocks, gs);
  return p;
}

void launch_mx_pass(const JobDev* jobs, const MxDesc* descs, int ndesc, int total_blocks,
                    int mode, int max_steps, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  const size_t shmem = sizeof(float2) * 16 * (size_t)(max_steps > 0 ? max_steps : 1);
  const dim3 grid(total_blocks), block(kBlock);
  if (mode == kMxFinal)
    hipLaunchKernelGGL(k_mx_pass<kMxFinal>, grid, block, shmem, s, jobs, descs, ndesc);
  else if (mode == kMxFromPhi)
    hipLaunchKernelGGL(k_mx_pass<kMxFromPhi>, grid, block, shmem, s, jobs, descs, ndesc);
  else
    hipLaunchKernelGGL(k_mx_pass<kMxIterate>, grid, block, shmem, s, jobs, descs, ndesc);
}

}  // namespace hg
