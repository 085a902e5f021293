// Lane-order layouts of the matrix-core operand tables: the prologue writes
// them and the full-grid passes read them, one coalesced access per lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

// FP32 separable passes, v_mfma_f32_16x16x4_f32 (lane l, r < 4):
//   A[l % 16][l / 16],  B[l / 16][l % 16],  D[4 (l / 16) + r][l % 16].
// K-step s of a spot contraction covers spots 2s and 2s + 1; lane group
// g = l / 16 holds part g % 2 (0 real, 1 imaginary) of spot 2 s + g / 2.
// The tables hold, per 16-column (or 16-row) block and K-step, the 64
// lanes' operands contiguously.
__device__ __forceinline__ int64_t op_index(int blk, int step, int steps, int lane) {
  return ((int64_t)blk * steps + step) * 64 + lane;
}
// The same operands with each lane's four consecutive steps next to each
// other (steps a multiple of 4): one 16-byte load per lane covers four
// K-steps of a 4-byte operand, two cover four steps of an 8-byte one.
__device__ __forceinline__ int64_t op_index4(int blk, int step, int steps, int lane) {
  return (((int64_t)blk * (steps >> 2) + (step >> 2)) * 64 + lane) * 4 + (step & 3);
}

// Mixed-precision passes, v_mfma_f32_16x16x32_f16 (lane l, e < 8, r < 4):
//   A[l % 16][8 (l / 16) + e],  B[8 (l / 16) + e][l % 16],  D[4 (l / 16) + r][l % 16].
// With K = 2 Np interleaved (k = 2 n + part), lane l of K-step s covers
// spots 16 s + 4 (l / 16) + q, q < 4, as four (re, im) half pairs.  Entries
// in table units (64-lane operand groups) of a job:
__device__ __forceinline__ int64_t fc_index(int cb, int s, int S16, int lane) {
  return ((int64_t)cb * S16 + s) * 64 + lane;
}
__device__ __forceinline__ int64_t fn_index(int sb, int cb, int CB, int lane) {
  return ((int64_t)sb * CB + cb) * 64 + lane;
}
__device__ __forceinline__ int64_t g_index(int rb, int s, int S16, int lane) {
  return ((int64_t)rb * S16 + s) * 64 + lane;
}

}  // namespace hg
