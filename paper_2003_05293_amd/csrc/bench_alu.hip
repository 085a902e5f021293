// Issue rates of the vector ALU operations the per-pixel passes are made of:
// FP32 FMA, v_sin_f32, v_cos_f32, v_fract_f32, and the FP16 dot product and
// packing conversion of the mixed-precision back-propagation, each as eight
// independent chains per lane over a grid of 8 waves per SIMD.  Prints lane-operations
// per second over the whole device; the ratios fix the issue slots of a
// (pixel, spot) pair used for the ALU roofline of the passes.
//
//     paper_2003_05293_amd/bench_alu
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

constexpr int kIter = 4096;
constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void k_rate(float* out, float seed) {
  float a[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) a[i] = seed + 0.001f * (float)(threadIdx.x + i);
  const h2_t hv{(_Float16)(seed * 0.5f), (_Float16)(seed * 0.25f)};
  const h2_t hw{(_Float16)0.999f, (_Float16)(-0.001f)};
  for (int it = 0; it < kIter; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if (KIND == 0) a[i] = fmaf(a[i], 0.999f, 0.0001f);
      if (KIND == 1) a[i] = __builtin_amdgcn_sinf(a[i]);
      if (KIND == 2) a[i] = __builtin_amdgcn_cosf(a[i]);
      if (KIND == 3) a[i] = __builtin_amdgcn_fractf(a[i]) + 0.25f;
      if (KIND == 4) a[i] = __builtin_amdgcn_fdot2(hv, hw, a[i], false);  // v_dot2c_f32_f16
      if (KIND == 5)  // v_cvt_pk_f16_f32 of two chains, then the pair's bits as the next input
        a[i] = __builtin_bit_cast(float, h2_t{(_Float16)a[i], (_Float16)a[(i + 1) % kChains]});
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));        \
      return -1.0;                                                        \
    }                                                                     \
  } while (0)

// Lane-operations per second of kernel KIND (ops per step: 1, or 2 for fract + add).
template <int KIND>
double rate(float* d, int blocks, int ops_per_step) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_rate<KIND>, dim3(blocks), dim3(256), 0, 0, d, 0.3f);
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  constexpr int kReps = 5;
  for (int r = 0; r < kReps; ++r) hipLaunchKernelGGL(k_rate<KIND>, dim3(blocks), dim3(256), 0, 0, d, 0.3f);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return (double)kReps * blocks * 256 * kIter * kChains * ops_per_step / (ms * 1e-3);
}

}  // namespace

int main() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  const int blocks = cus * 4 * 8;  // 8 waves per SIMD
  float* d = nullptr;
  if (hipMalloc(&d, sizeof(float) * (size_t)blocks * 256) != hipSuccess) return 1;
  const double fma = rate<0>(d, blocks, 1), sn = rate<1>(d, blocks, 1), cs = rate<2>(d, blocks, 1),
               fr = rate<3>(d, blocks, 2), dt = rate<4>(d, blocks, 1), cv = rate<5>(d, blocks, 1);
  if (fma < 0 || sn < 0 || cs < 0 || fr < 0 || dt < 0 || cv < 0) return 1;
  std::printf("compute units        %d\n", cus);
  std::printf("v_fma_f32            %.2f T lane-ops/s\n", fma / 1e12);
  std::printf("v_sin_f32            %.2f T lane-ops/s (%.3f of FMA)\n", sn / 1e12, sn / fma);
  std::printf("v_cos_f32            %.2f T lane-ops/s (%.3f of FMA)\n", cs / 1e12, cs / fma);
  std::printf("v_fract_f32 + v_add  %.2f T lane-ops/s\n", fr / 1e12);
  std::printf("v_dot2c_f32_f16      %.2f T lane-ops/s (%.3f of FMA)\n", dt / 1e12, dt / fma);
  std::printf("v_cvt_pk_f16_f32     %.2f T lane-ops/s (%.3f of FMA)\n", cv / 1e12, cv / fma);
  (void)hipFree(d);
  return 0;
}
