// Full-grid FP32 passes as separable products on the gfx950 matrix cores.
//
// With doubled pixel offsets the phase of eq. (2) splits into a part in the
// column and a part in the row: e^{i phi_n(i,j)} = F_n(i) G_n(j).  The
// back-propagated field of eq. (1) over the whole grid is then the complex
// matrix product S = B F with B_n(j) = C_n G_n(j), C_n = A_n e^{i theta_n},
// and the forward sums of eq. (3) over all pixels are
//   V_n = (1/M) sum_j conj(G_n(j)) T[j][n],  T = U conj(F)^T,  U = e^{i Phi}.
// Both products run as v_mfma_f32_16x16x4_f32 (FP32 operands and sums): a
// complex product is a real one with K = 2 Np, the real and imaginary parts
// of each spot (or pixel column) interleaved along K.  The factor tables are
// evaluated once per hologram in FP64 (the spots do not move), so the
// phases are exact to FP32 rounding; C_n comes from the state, or from the
// previous pass's deferred update, which a pending pass (and the final
// hologram) applies at its start.
#include <math.h>

#include "device_common.hpp"
#include "kernels.hpp"
#include "operand_layout.hpp"
#include "pass_tail.hpp"

namespace hg {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4_t mfma4(float a, float b, const f4_t& c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}



constexpr int kSepSteps = 8;  // K-steps of the back-propagation product per load group
constexpr int kSepCols = 8;   // column pairs of the forward product per load group
constexpr int kSepCB = kSepTileW / 16;  // 16-column blocks per tile

// Operands of kSepSteps K-steps of S = B F for one wave: G_n(row) of its
// rows and the F operand of the tile's 16-column blocks.  Loads of the
// next group are issued before the products of the current one.
struct BpOps {
  float2 ga[kSepSteps];
  float fc[kSepSteps][kSepCB];
};
__device__ __forceinline__ void bp_load(BpOps& o, const JobDev& jb, int rb, int tx, int s0, int KS,
                                        int lane) {
  static_assert(kSepSteps % 4 == 0, "groups of whole step quads");
#pragma unroll
  for (int h = 0; h < kSepSteps; h += 4) {
    // four steps of G (float2 each) in two 16-byte loads, four of each F
    // operand in one
    const HG_GLOBAL f4_t* gp =
        as_global(reinterpret_cast<const f4_t*>(jb.sepGa + op_index4(rb, s0 + h, KS, lane)));
    const f4_t g01 = gp[0], g23 = gp[1];
    o.ga[h] = make_float2(g01[0], g01[1]);
    o.ga[h + 1] = make_float2(g01[2], g01[3]);
    o.ga[h + 2] = make_float2(g23[0], g23[1]);
    o.ga[h + 3] = make_float2(g23[2], g23[3]);
#pragma unroll
    for (int t = 0; t < kSepCB; ++t) {
      const f4_t f = as_global(reinterpret_cast<const f4_t*>(
          jb.sepFc + op_index4(kSepCB * tx + t, s0 + h, KS, lane)))[0];
      o.fc[h][t] = f[0];
      o.fc[h + 1][t] = f[1];
      o.fc[h + 2][t] = f[2];
      o.fc[h + 3][t] = f[3];
    }
  }
}
// A operand: part of B (real output: (Br, -Bi)) or of i B (imaginary
// output: (Bi, Br)) with B_n(row) = C_n G_n(row) formed in FP32.
__device__ __forceinline__ void bp_mma(const BpOps& o, const float2* cs, int s0, int lg, int part,
                                       f4_t* sr, f4_t* si) {
#pragma unroll
  for (int q = 0; q < kSepSteps; ++q) {
    const float2 c = cs[2 * (s0 + q) + (lg >> 1)];
    const float br = c.x * o.ga[q].x - c.y * o.ga[q].y, bi = c.x * o.ga[q].y + c.y * o.ga[q].x;
    const float ar = part ? -bi : br, ai = part ? br : bi;
#pragma unroll
    for (int t = 0; t < kSepCB; ++t) {
      sr[t] = mfma4(ar, o.fc[q][t], sr[t]);
      si[t] = mfma4(ai, o.fc[q][t], si[t]);
    }
  }
}

// T = U conj(F)^T for R 16-spot blocks starting at sb0 and the wave's 16
// rows, then the tile's partial V_n = sum_j conj(G_n(j)) T[j][n] of those
// spots, added into row `row` of the exact sums.  Every thread of the block
// calls this with the same sb0 and R.
template <int R>
__device__ void sep_forward(const JobDev& jb, const float2 (*us)[kSepTileW + 1],
                            float2 (*red)[64], int sb0, int rb, int col0, int S16, int CP, int lane,
                            int wave, int shift, int row) {
  const int lr = lane & 15, lg = lane >> 4, part = lg & 1;
  f4_t tr[R], ti[R];
#pragma unroll
  for (int k = 0; k < R; ++k) tr[k] = ti[k] = f4_t{0.f, 0.f, 0.f, 0.f};
  float fa[kSepCols][R], fb[kSepCols][R];
  static_assert(kSepCols % 4 == 0, "load groups of whole column-pair quads");
  auto load = [&](float (*fn)[R], int c0) {  // four column pairs per 16-byte load
#pragma unroll
    for (int q = 0; q < kSepCols; q += 4)
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const f4_t f = as_global(reinterpret_cast<const f4_t*>(
            jb.sepFn + op_index4(sb0 + k, col0 / 2 + c0 + q, CP, lane)))[0];
        fn[q][k] = f[0];
        fn[q + 1][k] = f[1];
        fn[q + 2][k] = f[2];
        fn[q + 3][k] = f[3];
      }
  };
  auto mma = [&](const float (*fn)[R], int c0) {
#pragma unroll
    for (int q = 0; q < kSepCols; ++q) {
      const float2 u = us[lr][2 * (c0 + q) + (lg >> 1)];
      const float ar = part ? u.y : u.x, ai = part ? -u.x : u.y;  // parts of u and of -i u
#pragma unroll
      for (int k = 0; k < R; ++k) {
        tr[k] = mfma4(ar, fn[q][k], tr[k]);
        ti[k] = mfma4(ai, fn[q][k], ti[k]);
      }
    }
  };
  static_assert(kSepTileW / 2 == 2 * kSepCols, "two column groups per tile");
  load(fa, 0);
  load(fb, kSepCols);
  // G of the V sums, requested with F (it does not depend on the products)
  f4_t gva[R], gvb[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int64_t gv = op_index(rb, sb0 + k, S16, lane) * 2;
    gva[k] = as_global(reinterpret_cast<const f4_t*>(jb.sepGv))[gv];
    gvb[k] = as_global(reinterpret_cast<const f4_t*>(jb.sepGv))[gv + 1];
  }
  mma(fa, 0);
  mma(fb, kSepCols);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const f4_t g01 = gva[k], g23 = gvb[k];
    const float gr[4] = {g01[0], g01[2], g23[0], g23[2]};
    const float gi[4] = {g01[1], g01[3], g23[1], g23[3]};
    float vr = 0.f, vi = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      vr = fmaf(gr[r], tr[k][r], fmaf(gi[r], ti[k][r], vr));
      vi = fmaf(gr[r], ti[k][r], fmaf(-gi[r], tr[k][r], vi));
    }
    vr += __shfl_xor(vr, 16);
    vi += __shfl_xor(vi, 16);
    vr += __shfl_xor(vr, 32);
    vi += __shfl_xor(vi, 32);
    if (lg == 0) red[wave][16 * k + lr] = make_float2(vr, vi);
  }
  __syncthreads();
  if ((int)threadIdx.x < 16 * R) {
    const int n = 16 * sb0 + threadIdx.x;
    if (n < jb.N) {
      float2 v = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        v.x += red[w][threadIdx.x].x;
        v.y += red[w][threadIdx.x].y;
      }
      acc_add(jb.acc, jb.N, shift, row, n, v);
    }
  }
  __syncthreads();
}

template <bool FINAL>
__global__ __launch_bounds__(kBlock) void k_sep_pass(const JobDev* __restrict__ jobs,
                                                     const SepDesc* __restrict__ descs,
                                                     int ndesc) {
  extern __shared__ float2 cs[];                      // [Np] C_n = A_n e^{i theta_n}
  __shared__ float2 us[kWaves][16][kSepTileW + 1];    // u of each wave's rows
  __shared__ SpotRec recs[kPendMaxSpots];             // pending: the updated records
  __shared__ float2 red[kWaves][64];
  __shared__ int flag;
  const int di = find_desc(descs, ndesc, blockIdx.x);
  const SepDesc& d = descs[di];
  const JobDev& jb = jobs[d.job];
  const int W = jb.W, H = jb.H, N = jb.N, S16 = jb.mx_steps, KS = 8 * S16;
  const int CP = 8 * jb.mx_cblocks;
  const int lb = blockIdx.x - d.block_begin;
  const int tx = lb % d.tiles_x, ty = lb / d.tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, part = lg & 1;
  const int rb = 4 * ty + wave;
  const int row0 = 16 * rb, col0 = kSepTileW * tx;

  // S = B F, K = 2 Np in groups of kSepSteps steps (KS = 8 S16 is a
  // multiple of kSepSteps), the next group's operands loaded ahead.
  f4_t sr[kSepCB], si[kSepCB];
#pragma unroll
  for (int t = 0; t < kSepCB; ++t) sr[t] = si[t] = f4_t{0.f, 0.f, 0.f, 0.f};
  {
    static_assert(kSepSteps == 8, "K-step groups of 8: KS = 8 S16");
    const int G = KS / kSepSteps;
    // three operand buffers: the loads run two groups ahead of the products;
    // the first two are requested before C_n is staged, so that the two
    // reads overlap
    BpOps P, Q, R;
    bp_load(P, jb, rb, tx, 0, KS, lane);
    if (G > 1) bp_load(Q, jb, rb, tx, kSepSteps, KS, lane);
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
    for (int gi = 0; gi < G; gi += 3) {
      if (gi + 2 < G) bp_load(R, jb, rb, tx, (gi + 2) * kSepSteps, KS, lane);
      bp_mma(P, cs, gi * kSepSteps, lg, part, sr, si);
      if (gi + 1 < G) {
        if (gi + 3 < G) bp_load(P, jb, rb, tx, (gi + 3) * kSepSteps, KS, lane);
        bp_mma(Q, cs, (gi + 1) * kSepSteps, lg, part, sr, si);
      }
      if (gi + 2 < G) {
        if (gi + 4 < G) bp_load(Q, jb, rb, tx, (gi + 4) * kSepSteps, KS, lane);
        bp_mma(R, cs, (gi + 2) * kSepSteps, lg, part, sr, si);
      }
    }
  }

  if (FINAL) {
    HG_GLOBAL float* out = as_global_mut(d.out);
#pragma unroll
    for (int t = 0; t < kSepCB; ++t)
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

  // u = e^{i Phi} over the pupil (0 outside it and outside the grid),
  // weighted by the illumination, in LDS.
  const bool pupil = jb.ap_q >= 0 || jb.ill_a > 0.f;
#pragma unroll
  for (int t = 0; t < kSepCB; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + 4 * lg + r, col = col0 + 16 * t + lr;
      float2 u = make_float2(0.f, 0.f);
      if (row < H && col < W) {
        const float m2 = sr[t][r] * sr[t][r] + si[t][r] * si[t][r];
        u = make_float2(1.f, 0.f);
        if (m2 > 0.f) {
          const float inv = rsqrtf(m2);
          u = make_float2(sr[t][r] * inv, si[t][r] * inv);
        }
        if (pupil) {
          const int32_t lx = 2 * col - (W - 1), ly = 2 * row - (H - 1);
          const int32_t Qi = lx * lx + ly * ly;
          const float wt = pupil_weight(Qi, (float)Qi, jb.ap_q, jb.ill_a);
          u.x *= wt;
          u.y *= wt;
        }
      }
      us[wave][4 * lg + r][16 * t + lr] = u;
    }
  __syncthreads();

  // T and the partial V in groups of four 16-spot blocks, then the rest,
  // into the tile's group row, or, when the pass defers its update, into a
  // row of its total set (no counting: the next launch reads the set)
  const int g = lb / d.plan.group_size;
  const int row =
      d.defer ? d.tot_row * kAccReplicas + lb % kAccReplicas : kAccGroupRow0 + g;
  int sb0 = 0;
  for (; sb0 + 4 <= S16; sb0 += 4)
    sep_forward<4>(jb, us[wave], red, sb0, rb, col0, S16, CP, lane, wave, d.plan.shift, row);
  switch (S16 - sb0) {
    case 3:
      sep_forward<3>(jb, us[wave], red, sb0, rb, col0, S16, CP, lane, wave, d.plan.shift, row);
      break;
    case 2:
      sep_forward<2>(jb, us[wave], red, sb0, rb, col0, S16, CP, lane, wave, d.plan.shift, row);
      break;
    case 1:
      sep_forward<1>(jb, us[wave], red, sb0, rb, col0, S16, CP, lane, wave, d.plan.shift, row);
      break;
    default:
      break;
  }
  if (d.defer) return;

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
  a.acc = jb.acc;
  a.counters = jb.counters;
  a.inv_count = d.inv_count;
  a.V = d.V;
  a.status = jb.status;
  a.update = d.update;
  a.from_phi = 0;
  a.tot_row = d.tot_row;
  if (d.pending) {  // the update starts from the records in LDS
    a.recs = recs;
    a.pend_row = d.prev_row;
  }
  const int size = min(d.plan.group_size, d.plan.tiles - g * d.plan.group_size);
  if (arrive_last(&jb.counters[g * kCounterStride], (unsigned)size, &flag) &&
      tail_group(a, g, &flag))
    tail_final(a, cs);  // the C_n table (Np >= N float2) is no longer read
}

}  // namespace

PassPlan plan_sep(int W, int H) {
  PassPlan p;
  p.tiles = ceil_div(W, kSepTileW) * ceil_div(H, kSepTileH);
  p.sub = 1;
  p.blocks = p.tiles;
  int gs = 1;
  while (gs * gs < p.blocks) ++gs;
  p.group_size = gs;
  p.ngroups = ceil_div(p.blocks, gs);
  p.shift = sum_shift((int64_t)W * H);
  return p;
}

void launch_sep_pass(const JobDev* jobs, const SepDesc* descs, int ndesc, int total_blocks,
                     bool final, int max_steps, hipStream_t s) {
  if (ndesc <= 0 || total_blocks <= 0) return;
  const size_t shmem = sizeof(float2) * 16 * (size_t)(max_steps > 0 ? max_steps : 1);
  if (final)
    hipLaunchKernelGGL(k_sep_pass<true>, dim3(total_blocks), dim3(kBlock), shmem, s, jobs, descs,
                       ndesc);
  else
    hipLaunchKernelGGL(k_sep_pass<false>, dim3(total_blocks), dim3(kBlock), shmem, s, jobs, descs,
                       ndesc);
}

}  // namespace hg
