// Fixed costs behind the pass hand-off: back-to-back launches of an empty
// kernel, of a kernel whose every block adds 1 to one word with a
// device-scope atomic, and of a kernel that stores one float per thread, at
// several grid sizes (256 threads per block).  Prints microseconds per
// launch (HIP events around 2000 launches on one stream).
//
//     paper_2003_05293_amd/bench_launch
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

__global__ void k_empty(int* p) {
  if (p == nullptr) return;
}
__global__ void k_one_word(unsigned* c) {
  if (threadIdx.x == 0) atomicAdd(c, 1u);
}
__global__ __launch_bounds__(256) void k_store(float* o) { o[blockIdx.x * 256 + threadIdx.x] = 1.f; }

template <typename F>
double us_per_launch(F launch, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  for (int i = 0; i < 20; ++i) launch();
  if (hipDeviceSynchronize() != hipSuccess || hipEventRecord(a, 0) != hipSuccess) return -1.0;
  for (int i = 0; i < reps; ++i) launch();
  float ms = 0.f;
  if (hipEventRecord(b, 0) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
      hipEventElapsedTime(&ms, a, b) != hipSuccess)
    return -1.0;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return 1000.0 * ms / reps;
}

}  // namespace

int main() {
  constexpr int kMaxGrid = 4096;
  unsigned* c = nullptr;
  float* o = nullptr;
  if (hipMalloc(&c, 256) != hipSuccess || hipMemset(c, 0, 256) != hipSuccess ||
      hipMalloc(&o, sizeof(float) * kMaxGrid * 256) != hipSuccess)
    return 1;
  const int grids[] = {1, 64, 256, 1296, 2048, kMaxGrid};
  std::printf("%6s %12s %16s %12s\n", "blocks", "empty us", "one-word atomic", "store us");
  for (int g : grids) {
    const double e = us_per_launch([&] { hipLaunchKernelGGL(k_empty, dim3(g), dim3(256), 0, 0, (int*)c); }, 2000);
    const double t = us_per_launch([&] { hipLaunchKernelGGL(k_one_word, dim3(g), dim3(256), 0, 0, c); }, 2000);
    const double s = us_per_launch([&] { hipLaunchKernelGGL(k_store, dim3(g), dim3(256), 0, 0, o); }, 2000);
    if (e < 0 || t < 0 || s < 0) return 1;
    std::printf("%6d %12.2f %16.2f %12.2f\n", g, e, t, s);
  }
  (void)hipFree(c);
  (void)hipFree(o);
  return 0;
}
