// HIP kernels of the RS / WGS / CS-WGS hot path for gfx950 (wave64).
//
// Paper section 2: eq. (1) back-propagation, eq. (2) lens-and-prism phase,
// eq. (3) forward projection, eqs. (4)-(6) weight update, eq. (7) metrics.
// Section 3 of the paper recomputes phi_n per pixel instead of storing it;
// the kernels here do the same, in turns, from per-spot coefficients.
#include <math.h>

#include "device_math.hpp"
#include "kernels.hpp"

namespace hg {

namespace {

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

__device__ __forceinline__ int32_t pixel_of(const PixelSet& ps, int32_t q) {
  if (ps.idx) return ps.idx[q];
  if (ps.perm) {
    int64_t k = ps.start + q;
    if (k >= ps.M) k -= ps.M;
    return ps.perm[k];
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

// Field of eq. (1) at one pixel: S = sum_n A_n e^{i 2 pi (t_n + th_n)}.
// The spot loop index is uniform across the wave, so the records come in
// through scalar loads and feed the vector ALU as scalar operands.
__device__ __forceinline__ float2 backprop_field(const SpotRec* __restrict__ sp, int N,
                                                 const PixCoord& c) {
  float sr = 0.f, si = 0.f;
#pragma unroll 4
  for (int n = 0; n < N; ++n) {
    const SpotRec s = sp[n];
    const float t = fmaf(s.cx, c.Lx, fmaf(s.cy, c.Ly, fmaf(s.cz, c.Q, s.th)));
    float sn, cs;
    sincos_turns(t, sn, cs);
    sr = fmaf(s.A, cs, sr);
    si = fmaf(s.A, sn, si);
  }
  return make_float2(sr, si);
}

// Forward partial sums over a tile of pixels held in LDS.  Lanes map to
// spots (64 per chunk), waves split the tile's pixels; the pixel record read
// is uniform across the wave (an LDS broadcast).  Each block writes one
// partial sum per spot: the waves' sums added in wave order.
__device__ __forceinline__ void forward_term(float cx, float cy, float cz, const float4& a,
                                             float ui, float& vr, float& vi) {
  const float t = fmaf(cx, a.x, fmaf(cy, a.y, cz * a.z));
  float sn, cs;
  sincos_turns(t, sn, cs);
  // u * conj(e^{i 2 pi t})
  vr = fmaf(a.w, cs, fmaf(ui, sn, vr));
  vi = fmaf(ui, cs, fmaf(-a.w, sn, vi));
}

__device__ __forceinline__ void forward_tile(const SpotRec* __restrict__ sp, int N,
                                             const float4* __restrict__ px,
                                             const float* __restrict__ pui, int npix,
                                             float2 (*red)[64], float2* __restrict__ partial) {
  // the wave index is uniform across the wave: keep the pixel loop scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  for (int n0 = 0; n0 < N; n0 += 64) {
    const int n = n0 + lane;
    float cx = 0.f, cy = 0.f, cz = 0.f;
    if (n < N) {
      cx = sp[n].cx;
      cy = sp[n].cy;
      cz = sp[n].cz;
    }
    float vr = 0.f, vi = 0.f;
    int k = wave;
    for (; k + 3 * kWaves < npix; k += 4 * kWaves) {
#pragma unroll
      for (int u = 0; u < 4; ++u) forward_term(cx, cy, cz, px[k + u * kWaves], pui[k + u * kWaves], vr, vi);
    }
    for (; k < npix; k += kWaves) forward_term(cx, cy, cz, px[k], pui[k], vr, vi);
    red[wave][lane] = make_float2(vr, vi);
    __syncthreads();
    if (wave == 0 && n < N) {
      float2 acc = red[0][lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        acc.x += red[w][lane].x;
        acc.y += red[w][lane].y;
      }
      partial[(int64_t)blockIdx.x * N + n] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- setup ---

// Spot coefficients in FP64, rounded once to FP32.  Spot values that are not
// finite, or amplitudes that are not positive, raise the argument status
// flag (device-resident inputs cannot be checked on the host).
__global__ void k_setup(SetupArgs a, SpotPtrs in, SpotRec* __restrict__ sp,
                        double* __restrict__ th0, int32_t* __restrict__ status) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  const double x = in.x[n], y = in.y[n], z = in.z[n], amp = in.amp[n];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !(amp > 0.0) || !isfinite(amp))
    status[0] = 1;  // HG_EINVAL
  const double lf = a.lambda_mm * a.focal_mm;
  const double lf2 = lf * a.focal_mm;
  SpotRec r;
  r.cx = (float)(x * a.pitch_mm / (2.0 * lf));
  r.cy = (float)(y * a.pitch_mm / (2.0 * lf));
  r.cz = (float)(z * a.pitch_mm * a.pitch_mm / (4.0 * lf2));
  const double u = theta0_turns(a.seed, (uint64_t)n);
  r.th = (float)u;
  r.A = (float)amp;
  r.a0 = (float)amp;
  r.w = 1.0f;
  r.pad = 0.0f;
  sp[n] = r;
  if (th0) th0[n] = (2.0 * M_PI) * u;
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

__global__ void k_tables(uint64_t seed, int h, uint32_t* __restrict__ tab) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t size = 1u << h;
  if (k >= (uint32_t)kFeistelRounds * size) return;
  const int r = (int)(k >> h);
  const uint32_t R = k & (size - 1u);
  tab[k] = feistel_table_entry(seed, r, R, h);
}

__global__ void k_perm(int32_t M, int h, const uint32_t* __restrict__ tab,
                       int32_t* __restrict__ perm) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  perm[k] = (int32_t)permute((uint32_t)k, (uint32_t)M, tab, h);
}

__global__ void k_gather(PixelSet ps, int32_t* __restrict__ out) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ps.count) return;
  out[q] = pixel_of(ps, q);
}

// ------------------------------------------------------------ iteration ---

// One fused iteration body over a pixel set: back-propagation of eq. (1)
// with the current (A, th), normalised to the unit phasor u = e^{i Phi},
// then the forward partial sums of eq. (3) over the same pixels.  Phi is
// never stored: the next forward step reads it only on these pixels.
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_iter(const SpotRec* __restrict__ sp, int N, int W,
                                                 int H, PixelSet ps,
                                                 float2* __restrict__ partial) {
  __shared__ float4 px[kBlock * PPT];
  __shared__ float pui[kBlock * PPT];
  __shared__ float2 red[kWaves][64];
  const int32_t base = blockIdx.x * (kBlock * PPT);
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int qi = k * kBlock + threadIdx.x;
    const int32_t q = base + qi;
    float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
    float ui = 0.f;
    if (q < ps.count) {
      const PixCoord c = pixel_coord(pixel_of(ps, q), W, H);
      const float2 S = backprop_field(sp, N, c);
      const float m2 = S.x * S.x + S.y * S.y;
      float ur = 1.f;
      if (m2 > 0.f) {
        const float inv = rsqrtf(m2);
        ur = S.x * inv;
        ui = S.y * inv;
      }
      rec = make_float4(c.Lx, c.Ly, c.Q, ur);
    }
    px[qi] = rec;
    pui[qi] = ui;
  }
  __syncthreads();
  const int npix = min(kBlock * PPT, ps.count - base);
  forward_tile(sp, N, px, pui, npix, red, partial);
}

// Forward partial sums of a stored hologram Phi (radians) over a pixel set.
template <int PPT>
__global__ __launch_bounds__(kBlock) void k_forward_phi(const SpotRec* __restrict__ sp, int N,
                                                        int W, int H, PixelSet ps,
                                                        const float* __restrict__ phi,
                                                        float2* __restrict__ partial) {
  __shared__ float4 px[kBlock * PPT];
  __shared__ float pui[kBlock * PPT];
  __shared__ float2 red[kWaves][64];
  const int32_t base = blockIdx.x * (kBlock * PPT);
  constexpr float kInvTwoPi = 0.15915494309189535f;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int qi = k * kBlock + threadIdx.x;
    const int32_t q = base + qi;
    float4 rec = make_float4(0.f, 0.f, 0.f, 0.f);
    float ui = 0.f;
    if (q < ps.count) {
      const int32_t p = pixel_of(ps, q);
      const PixCoord c = pixel_coord(p, W, H);
      float sn, cs;
      sincos_turns(phi[p] * kInvTwoPi, sn, cs);
      rec = make_float4(c.Lx, c.Ly, c.Q, cs);
      ui = sn;
    }
    px[qi] = rec;
    pui[qi] = ui;
  }
  __syncthreads();
  const int npix = min(kBlock * PPT, ps.count - base);
  forward_tile(sp, N, px, pui, npix, red, partial);
}

// Sum the per-block partials of each spot in FP64, in a fixed order:
// slice s of the block's threads adds blocks s, s+S, s+2S, ...; the slices
// are then added in slice order by the slice-0 thread of the spot, which
// writes V_n = sum * inv_count.  Spot n is always finalised by thread
// n mod kChunk; the return value is that thread's sum of |V_n| (0 for the
// other threads).
constexpr int kChunk = 128;
constexpr int kSlices = kUpdateThreads / kChunk;

__device__ double reduce_partials(const float2* __restrict__ partial, int nblk, int N,
                                  double inv_count, double2* __restrict__ V) {
  __shared__ double rre[kSlices][kChunk];
  __shared__ double rim[kSlices][kChunk];
  const int c = threadIdx.x % kChunk;
  const int s = threadIdx.x / kChunk;
  double magsum = 0.0;
  for (int n0 = 0; n0 < N; n0 += kChunk) {
    const int n = n0 + c;
    double are = 0.0, aim = 0.0;
    if (n < N) {
      for (int b = s; b < nblk; b += kSlices) {
        const float2 v = partial[(int64_t)b * N + n];
        are += (double)v.x;
        aim += (double)v.y;
      }
    }
    rre[s][c] = are;
    rim[s][c] = aim;
    __syncthreads();
    if (s == 0 && n < N) {
      double tr = rre[0][c], ti = rim[0][c];
#pragma unroll
      for (int k = 1; k < kSlices; ++k) {
        tr += rre[k][c];
        ti += rim[k][c];
      }
      tr *= inv_count;
      ti *= inv_count;
      V[n] = make_double2(tr, ti);
      magsum += sqrt(tr * tr + ti * ti);
    }
    __syncthreads();
  }
  return magsum;
}

__global__ __launch_bounds__(kUpdateThreads) void k_reduce(const float2* __restrict__ partial,
                                                           int nblk, int N, double inv_count,
                                                           double2* __restrict__ V) {
  reduce_partials(partial, nblk, N, inv_count, V);
}

// eqs. (4)-(6): w_n <- w_n * mean_k |V_k| / |V_n|, theta_n <- arg V_n,
// A_n = a_n^0 w_n.  A spot whose field is zero or not finite keeps its
// state and raises the numeric status flag.  Each spot is updated by the
// thread that finalised its V_n, so V is read back by its own writer.
__global__ __launch_bounds__(kUpdateThreads) void k_update(const float2* __restrict__ partial,
                                                           int nblk, int N, double inv_count,
                                                           SpotRec* __restrict__ sp,
                                                           double2* __restrict__ V,
                                                           int32_t* __restrict__ status) {
  __shared__ double msum[kUpdateThreads];
  msum[threadIdx.x] = reduce_partials(partial, nblk, N, inv_count, V);
  __syncthreads();
  for (int stride = kUpdateThreads / 2; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) msum[threadIdx.x] += msum[threadIdx.x + stride];
    __syncthreads();
  }
  const double mean = msum[0] / (double)N;
  if (threadIdx.x >= kChunk) return;
  for (int n = threadIdx.x; n < N; n += kChunk) {
    const double2 v = V[n];
    const double mag = sqrt(v.x * v.x + v.y * v.y);
    SpotRec r = sp[n];
    const double w = (double)r.w * (mean / mag);
    if (!(mag > 0.0) || !isfinite(w)) {
      status[0] = 4;  // HG_ENUMERIC
      continue;
    }
    r.w = (float)w;
    r.A = (float)(w * (double)r.a0);
    r.th = (float)(atan2(v.y, v.x) / (2.0 * M_PI));
    sp[n] = r;
  }
}

// Final hologram on a pixel set: Phi = atan2(Im S, Re S), written to out[q].
__global__ __launch_bounds__(kBlock) void k_backprop_phi(const SpotRec* __restrict__ sp, int N,
                                                         int W, int H, PixelSet ps,
                                                         float* __restrict__ out) {
  const int32_t q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= ps.count) return;
  const PixCoord c = pixel_coord(pixel_of(ps, q), W, H);
  const float2 S = backprop_field(sp, N, c);
  out[q] = atan2f(S.y, S.x);
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

void launch_setup(const SetupArgs& a, const SpotPtrs& in, SpotRec* sp, double* th0,
                  int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(ceil_div(a.N, 256)), dim3(256), 0, s, a, in, sp, th0, status);
}

void launch_theta0(uint64_t seed, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_theta0, dim3(ceil_div(count, 256)), dim3(256), 0, s, seed, count, out);
}

void launch_set_state(int N, const double* wth, SpotRec* sp, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, wth, sp);
}

void launch_tables(uint64_t seed, int h, uint32_t* tab, hipStream_t s) {
  const int total = kFeistelRounds << h;
  hipLaunchKernelGGL(k_tables, dim3(ceil_div(total, 256)), dim3(256), 0, s, seed, h, tab);
}

void launch_perm(int32_t M, int h, const uint32_t* tab, int32_t* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_perm, dim3(ceil_div(M, 256)), dim3(256), 0, s, M, h, tab, perm);
}

void launch_gather(const PixelSet& ps, int32_t* out, hipStream_t s) {
  if (ps.count <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(ceil_div(ps.count, 256)), dim3(256), 0, s, ps, out);
}

int iter_ppt(int32_t count) {
  // keep at least ~1000 blocks in flight before packing more pixels per block
  if (count >= 4 * 1024 * kBlock) return 4;
  if (count >= 2 * 1024 * kBlock) return 2;
  return 1;
}

int iter_blocks(int32_t count, int ppt) { return ceil_div(count, (int64_t)kBlock * ppt); }

void launch_iter(const SpotRec* sp, int N, int W, int H, const PixelSet& ps, int ppt,
                 float2* partial, hipStream_t s) {
  const dim3 grid(iter_blocks(ps.count, ppt)), block(kBlock);
  switch (ppt) {
    case 4: hipLaunchKernelGGL(k_iter<4>, grid, block, 0, s, sp, N, W, H, ps, partial); break;
    case 2: hipLaunchKernelGGL(k_iter<2>, grid, block, 0, s, sp, N, W, H, ps, partial); break;
    default: hipLaunchKernelGGL(k_iter<1>, grid, block, 0, s, sp, N, W, H, ps, partial); break;
  }
}

void launch_forward_phi(const SpotRec* sp, int N, int W, int H, const PixelSet& ps,
                        const float* phi, int ppt, float2* partial, hipStream_t s) {
  const dim3 grid(iter_blocks(ps.count, ppt)), block(kBlock);
  switch (ppt) {
    case 4:
      hipLaunchKernelGGL(k_forward_phi<4>, grid, block, 0, s, sp, N, W, H, ps, phi, partial);
      break;
    case 2:
      hipLaunchKernelGGL(k_forward_phi<2>, grid, block, 0, s, sp, N, W, H, ps, phi, partial);
      break;
    default:
      hipLaunchKernelGGL(k_forward_phi<1>, grid, block, 0, s, sp, N, W, H, ps, phi, partial);
      break;
  }
}

void launch_update(const float2* partial, int nblk, int N, double inv_count, SpotRec* sp,
                   double2* V, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(1), dim3(kUpdateThreads), 0, s, partial, nblk, N, inv_count,
                     sp, V, status);
}

void launch_reduce(const float2* partial, int nblk, int N, double inv_count, double2* V,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kUpdateThreads), 0, s, partial, nblk, N, inv_count,
                     V);
}

void launch_backprop_phi(const SpotRec* sp, int N, int W, int H, const PixelSet& ps, float* out,
                         hipStream_t s) {
  if (ps.count <= 0) return;
  hipLaunchKernelGGL(k_backprop_phi, dim3(ceil_div(ps.count, kBlock)), dim3(kBlock), 0, s, sp, N,
                     W, H, ps, out);
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
