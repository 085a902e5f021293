// Device helpers shared by the kernels: the counter-based generator, the
// keyed pixel permutation and sin/cos of phases held in turns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64->128-bit
// multiplies with the published multipliers, key advanced between rounds by
// the published Weyl increments.
// ---------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

struct Block4x64 {
  uint64_t v[4];
};

__device__ inline Block4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                          uint64_t c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Block4x64 b;
  b.v[0] = c0;
  b.v[1] = c1;
  b.v[2] = c2;
  b.v[3] = c3;
  return b;
}

// theta_n^0 as a fraction of a turn: u = (word >> 11) * 2^-53, word 0 of the
// block (n, 0, 0, 0) under key (seed, 0).
__device__ inline double theta0_turns(uint64_t seed, uint64_t n) {
  const Block4x64 b = philox4x64_10(n, 0, 0, 0, seed, 0);
  return (double)(b.v[0] >> 11) * 0x1.0p-53;
}

// Feistel round function tables: F_r[R] = word 0 of block (R, r, 0, 0) under
// key (seed, 1), reduced to h bits.
__device__ inline uint32_t feistel_table_entry(uint64_t seed, int r, uint32_t R, int h) {
  const Block4x64 b = philox4x64_10(R, (uint64_t)r, 0, 0, seed, 1);
  return (uint32_t)(b.v[0] & ((1ull << h) - 1));
}

constexpr int kFeistelRounds = 6;

// Six rounds on x < 4^h: (L, R) -> (R, L xor F_r[R]).  tab is [6][2^h].
__device__ inline uint32_t feistel(uint32_t x, const uint32_t* __restrict__ tab, int h) {
  const uint32_t mask = (1u << h) - 1u;
  uint32_t L = x >> h, R = x & mask;
#pragma unroll
  for (int r = 0; r < kFeistelRounds; ++r) {
    const uint32_t nR = L ^ tab[((uint32_t)r << h) | R];
    L = R;
    R = nR;
  }
  return (L << h) | R;
}

// pi(k): walk the Feistel cycle of k until it lands in [0, M).  The cycle of
// k contains k itself, so the walk ends within 4^h steps.
__device__ inline uint32_t permute(uint32_t k, uint32_t M, const uint32_t* __restrict__ tab,
                                   int h) {
  uint32_t y = feistel(k, tab, h);
  const uint32_t cap = 1u << (2 * h < 32 ? 2 * h : 31);
  for (uint32_t step = 0; y >= M && step < cap; ++step) y = feistel(y, tab, h);
  return y;
}

// ---------------------------------------------------------------------------
// sin and cos of 2*pi*t for a phase t held in turns.  The fractional part is
// taken exactly (v_fract), then the hardware sine and cosine, which take
// their argument in turns, are applied on [0, 1).
// ---------------------------------------------------------------------------
// FP16 pairs (round to nearest even) of the mixed-precision products.
typedef _Float16 h2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2v_t to_h2(float lo, float hi) {
  return h2v_t{(_Float16)lo, (_Float16)hi};
}
__device__ __forceinline__ uint32_t h2_bits(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, to_h2(lo, hi));
}

__device__ __forceinline__ void sincos_turns(float t, float& s, float& c) {
  const float r = __builtin_amdgcn_fractf(t);
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}

}  // namespace hg
