// Internal interface between the kernels (kernels.hip) and the host runtime
// (api.hip).  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

// Per-spot record read by the back-propagation loop.  All phases are in
// turns (fractions of 2*pi) and use doubled integer pixel offsets
// Lx = 2i - (W-1), Ly = 2j - (H-1) and Q = Lx^2 + Ly^2, so that eq. (2)
// divided by 2*pi reads  phi_n / (2 pi) = cx*Lx + cy*Ly + cz*Q  with
//   cx = x_n pitch / (2 lambda f),  cy = y_n pitch / (2 lambda f),
//   cz = z_n pitch^2 / (4 lambda f^2).
// th = theta_n / (2 pi) and A = a_n^0 w_n complete eq. (1).
struct alignas(32) SpotRec {
  float cx, cy, cz, th;
  float A, a0, w, pad;
};

// Optics and grid constants needed by the setup kernels.
struct SetupArgs {
  int32_t N;
  int32_t W, H;
  double pitch_mm, lambda_mm, focal_mm;
  uint64_t seed;
};

constexpr int kBlock = 256;          // threads per block of the pixel kernels
constexpr int kWaves = kBlock / 64;  // wave64s per block
constexpr int kUpdateThreads = 1024;

// Pixel set of a pass: either all pixels 0..count-1 (perm == nullptr) or
// perm[(start + q) mod M] for q < count, or explicit indices idx[q].
struct PixelSet {
  const int32_t* perm;  // random order of [0, M) or nullptr
  const int32_t* idx;   // explicit pixel list or nullptr
  int64_t start;        // window start in the order (< M)
  int32_t count;        // number of pixels in the set
  int32_t M;            // W*H
};

// Device arrays of the N spot coordinates (mm) and target amplitudes.
struct SpotPtrs {
  const double* x;
  const double* y;
  const double* z;
  const double* amp;
};

// ---- setup (FP64) ----
void launch_setup(const SetupArgs& a, const SpotPtrs& in, SpotRec* sp,
                  double* theta0_out /*nullable*/, int32_t* status, hipStream_t s);
void launch_theta0(uint64_t seed, int count, double* out, hipStream_t s);
void launch_set_state(int N, const double* wth /*w: N, theta: N*/, SpotRec* sp, hipStream_t s);
void launch_tables(uint64_t seed, int h, uint32_t* tab, hipStream_t s);
void launch_perm(int32_t M, int h, const uint32_t* tab, int32_t* perm, hipStream_t s);
void launch_gather(const PixelSet& ps, int32_t* out, hipStream_t s);

// ---- iteration ----
// Launch geometry of one pass over `count` pixels (a function of count only,
// so the summation order of a pass never depends on the batch or device).
struct PassPlan {
  int tiles;       // pixel tiles of 64
  int blocks;      // grid size; block b handles tiles b, b + blocks, ...
  int group_size;  // blocks per first-level reduction group
  int ngroups;
};
PassPlan plan_pass(int32_t count);
// One pass: back-propagation of the state in `sp` (or, with phi != nullptr,
// the stored hologram phi) on the pixel set, forward projection over the same
// set, deterministic reduction to V (N complex, FP64) and, if `update`, the
// weight update of eqs. (4)-(6) written back to sp.  `counters` must be zero
// on entry (ngroups + 1 words) and is zero again when the pass ends.
void launch_pass(const PassPlan& plan, SpotRec* sp, int N, int W, int H, const PixelSet& ps,
                 const float* phi, float2* partial, double2* gpart, unsigned* counters,
                 double2* V, int32_t* status, bool update, hipStream_t s);
void launch_zero_counters(unsigned* counters, int n, hipStream_t s);
// Final hologram: Phi = arg(sum_n A_n e^{i 2 pi (t_n + th_n)}) on the set,
// written compactly (out[q]) or, for all pixels, at out[p].
void launch_backprop_phi(const SpotRec* sp, int N, int W, int H, const PixelSet& ps, float* out,
                         hipStream_t s);

// ---- metrics (FP64) ----
void launch_metric_tables(const SetupArgs& a, const SpotPtrs& in, double2* Ex, double2* Ey,
                          hipStream_t s);
int metric_blocks(int H);
void launch_metric_rows(const double2* Ex, const double2* Ey, int N, int W, int H,
                        const float* phi, double2* partial, hipStream_t s);
void launch_metric_reduce(const double2* partial, int nblk, int N, double inv_count,
                          double2* V_out, hipStream_t s);

}  // namespace hg
