// C ABI of libhg (include/hg.h): argument validation, per-stream scratch
// memory and the RS / WGS / CS-WGS schedules of the paper's section 2.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hg.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

hg_status fail(hg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HG_HIP(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(e_ == hipErrorOutOfMemory ? HG_ENOMEM : HG_EDEVICE,                \
                  std::string(#expr) + " failed: " + hipGetErrorString(e_));         \
  } while (0)

#define HG_TRY(expr)              \
  do {                            \
    hg_status st_ = (expr);       \
    if (st_ != HG_OK) return st_; \
  } while (0)

// Device buffer that grows on demand and is never shrunk.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  hg_status reserve(size_t n) {
    if (n <= cap) return HG_OK;
    if (p) {
      HG_HIP(hipFree(p));
      p = nullptr;
      cap = 0;
    }
    HG_HIP(hipMalloc((void**)&p, n * sizeof(T)));
    cap = n;
    return HG_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// ----------------------------------------------------------------- timing --

std::atomic<bool> g_timing{false};

struct TimedLaunch {
  const char* name;
  hipEvent_t start, stop;
};

struct TimingTotals {
  double ms = 0.0;
  int64_t launches = 0;
};

std::mutex g_tmu;
std::map<std::string, TimingTotals> g_totals;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event() {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scratch of one (device, stream).  Calls on the same stream run in stream
// order, so its buffers can be reused from call to call; the pinned staging
// area is refilled only after the previous upload from it has completed.
// `status` is sticky: kernels raise it, blocking calls report and clear it.
struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  DevBuf<double> raw;             // x, y, z, amp, then w, theta: 6N
  DevBuf<hg::SpotRec> sp;         // N
  DevBuf<uint32_t> tab;           // 6 * 2^h Feistel tables
  DevBuf<int32_t> perm;           // M random order
  DevBuf<float2> partial;         // blocks * N
  DevBuf<double2> gpart;          // groups * N
  DevBuf<unsigned> counters;      // groups + 1, zero between passes
  DevBuf<double2> V;              // N, or iterations * N when tracing
  DevBuf<int32_t> status;         // 1
  DevBuf<double2> Ex, Ey, mpart;  // metrics
  double* pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  std::vector<TimedLaunch> timed;

  hg_status init_status() {
    if (status.p) return HG_OK;
    HG_TRY(status.reserve(1));
    HG_HIP(hipMemsetAsync(status.p, 0, sizeof(int32_t), stream));
    return HG_OK;
  }

  // After the stream has been synchronised: report and clear the flag.
  hg_status take_status() {
    int32_t st = 0;
    HG_HIP(hipMemcpy(&st, status.p, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (st == 0) return HG_OK;
    HG_HIP(hipMemset(status.p, 0, sizeof(int32_t)));
    if (st == HG_EINVAL)
      return fail(HG_EINVAL, "device-resident spot values were not finite or an amplitude was "
                             "not positive (in this or an earlier call on this stream)");
    return fail(HG_ENUMERIC, "a spot field came out zero or not finite (in this or an earlier "
                             "call on this stream)");
  }

  hg_status stage(size_t ndoubles) {
    if (staged_pending) {
      HG_HIP(hipEventSynchronize(staged));
      staged_pending = false;
    }
    if (ndoubles > pinned_cap) {
      if (pinned) HG_HIP(hipHostFree(pinned));
      pinned = nullptr;
      pinned_cap = 0;
      HG_HIP(hipHostMalloc((void**)&pinned, ndoubles * sizeof(double), hipHostMallocDefault));
      pinned_cap = ndoubles;
    }
    if (!staged) HG_HIP(hipEventCreateWithFlags(&staged, hipEventDisableTiming));
    return HG_OK;
  }

  // Runs `launch` bracketed by events when timing is on.
  template <typename F>
  void timed_launch(const char* name, F&& launch) {
    if (!g_timing.load(std::memory_order_relaxed)) {
      launch();
      return;
    }
    hipEvent_t a = pool_event(), b = pool_event();
    if (a && b) (void)hipEventRecord(a, stream);
    launch();
    if (a && b) {
      (void)hipEventRecord(b, stream);
      timed.push_back(TimedLaunch{name, a, b});
    }
  }

  void drain_timing() {
    for (const TimedLaunch& t : timed) {
      float ms = 0.f;
      if (hipEventSynchronize(t.stop) == hipSuccess &&
          hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_tmu);
        TimingTotals& tt = g_totals[t.name];
        tt.ms += ms;
        tt.launches += 1;
      }
      std::lock_guard<std::mutex> lk(g_tmu);
      g_event_pool.push_back(t.start);
      g_event_pool.push_back(t.stop);
    }
    timed.clear();
  }

  void release() {
    drain_timing();
    raw.release();
    sp.release();
    tab.release();
    perm.release();
    partial.release();
    gpart.release();
    counters.release();
    V.release();
    status.release();
    Ex.release();
    Ey.release();
    mpart.release();
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_cap = 0;
    if (staged) (void)hipEventDestroy(staged);
    staged = nullptr;
    staged_pending = false;
  }
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

hg_status get_workspace(void* stream, Workspace** out) {
  int dev = 0;
  HG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, (hipStream_t)stream);
  auto it = g_ws.find(key);
  if (it == g_ws.end()) {
    auto ws = std::make_unique<Workspace>();
    ws->device = dev;
    ws->stream = (hipStream_t)stream;
    it = g_ws.emplace(key, std::move(ws)).first;
  }
  *out = it->second.get();
  return HG_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

hg_status validate(const hg_grid* g, const hg_optics* o, const hg_spots* s, bool on_device) {
  if (!g || !o || !s) return fail(HG_EINVAL, "grid, optics and spots must be non-NULL");
  if (g->W < 1 || g->H < 1 || g->W > 8192 || g->H > 8192)
    return fail(HG_EINVAL, "grid W and H must be in [1, 8192]");
  if (!finite_pos(g->pitch_mm)) return fail(HG_EINVAL, "pitch_mm must be positive and finite");
  if (!finite_pos(o->lambda_mm) || !finite_pos(o->focal_mm))
    return fail(HG_EINVAL, "lambda_mm and focal_mm must be positive and finite");
  if (s->n < 1 || s->n > HG_MAX_SPOTS)
    return fail(HG_EINVAL, "spot count must be in [1, HG_MAX_SPOTS]");
  if (!s->x_mm || !s->y_mm || !s->z_mm || !s->amp)
    return fail(HG_EINVAL, "spot arrays must be non-NULL");
  if (on_device) return HG_OK;  // values are checked by the setup kernel
  for (int n = 0; n < s->n; ++n) {
    if (!std::isfinite(s->x_mm[n]) || !std::isfinite(s->y_mm[n]) || !std::isfinite(s->z_mm[n]))
      return fail(HG_EINVAL, "spot coordinates must be finite");
    if (!finite_pos(s->amp[n])) return fail(HG_EINVAL, "spot amplitudes must be positive and finite");
  }
  return HG_OK;
}

hg_status validate_flags(uint32_t flags, uint32_t allowed_extra) {
  if (flags & ~(HG_PREC_MASK | allowed_extra))
    return fail(HG_EINVAL, "flags: unknown bits set");
  if ((flags & HG_PREC_MASK) != HG_PREC_FP32)
    return fail(HG_EINVAL, "flags: only HG_PREC_FP32 is available in this build");
  return HG_OK;
}

int half_bits(int64_t M) {
  int h = 1;
  while ((int64_t(1) << (2 * h)) < M) ++h;
  return h;
}

int32_t subset_size(int64_t M, double c) { return (int32_t)std::ceil(c * (double)M); }

hg::SetupArgs setup_args(const hg_grid* g, const hg_optics* o, const hg_spots* s, uint64_t seed) {
  hg::SetupArgs a;
  a.N = s->n;
  a.W = g->W;
  a.H = g->H;
  a.pitch_mm = g->pitch_mm;
  a.lambda_mm = o->lambda_mm;
  a.focal_mm = o->focal_mm;
  a.seed = seed;
  return a;
}

// Brings the spot arrays (and optionally w, theta) to the device and runs the
// FP64 coefficient setup.  Host arrays go through the pinned staging area;
// device-resident arrays are read in place.  Returns the device pointers.
hg_status upload_spots(Workspace* ws, const hg_grid* g, const hg_optics* o, const hg_spots* s,
                       uint64_t seed, bool on_device, const double* w, const double* theta,
                       hg::SpotPtrs* dev) {
  const int N = s->n;
  HG_TRY(ws->init_status());
  HG_TRY(ws->sp.reserve(N));
  hg::SpotPtrs in;
  if (on_device) {
    in = hg::SpotPtrs{s->x_mm, s->y_mm, s->z_mm, s->amp};
  } else {
    const size_t nd = (size_t)6 * N;
    HG_TRY(ws->stage(nd));
    std::memcpy(ws->pinned + 0 * N, s->x_mm, N * sizeof(double));
    std::memcpy(ws->pinned + 1 * N, s->y_mm, N * sizeof(double));
    std::memcpy(ws->pinned + 2 * N, s->z_mm, N * sizeof(double));
    std::memcpy(ws->pinned + 3 * N, s->amp, N * sizeof(double));
    if (w) std::memcpy(ws->pinned + 4 * N, w, N * sizeof(double));
    if (theta) std::memcpy(ws->pinned + 5 * N, theta, N * sizeof(double));
    HG_TRY(ws->raw.reserve(nd));
    HG_HIP(hipMemcpyAsync(ws->raw.p, ws->pinned, nd * sizeof(double), hipMemcpyHostToDevice,
                          ws->stream));
    HG_HIP(hipEventRecord(ws->staged, ws->stream));
    ws->staged_pending = true;
    in = hg::SpotPtrs{ws->raw.p, ws->raw.p + N, ws->raw.p + 2 * N, ws->raw.p + 3 * N};
  }
  hg::launch_setup(setup_args(g, o, s, seed), in, ws->sp.p, nullptr, ws->status.p, ws->stream);
  if (w && theta) hg::launch_set_state(N, ws->raw.p + 4 * N, ws->sp.p, ws->stream);
  if (dev) *dev = in;
  return HG_OK;
}

hg_status build_order(Workspace* ws, int64_t M, uint64_t seed) {
  const int h = half_bits(M);
  HG_TRY(ws->tab.reserve((size_t)6 << h));
  HG_TRY(ws->perm.reserve((size_t)M));
  hg::launch_tables(seed, h, ws->tab.p, ws->stream);
  hg::launch_perm((int32_t)M, h, ws->tab.p, ws->perm.p, ws->stream);
  return HG_OK;
}

// Scratch of a pass of `count` pixels; counters are cleared by a fill kernel
// (never by a memset node) so that the sequence can be graph-captured.
hg_status reserve_pass(Workspace* ws, const hg::PassPlan& plan, int N) {
  HG_TRY(ws->partial.reserve((size_t)plan.blocks * N));
  HG_TRY(ws->gpart.reserve((size_t)plan.ngroups * N));
  const size_t before = ws->counters.cap;
  HG_TRY(ws->counters.reserve((size_t)plan.ngroups + 1));
  if (ws->counters.cap != before) hg::launch_zero_counters(ws->counters.p, (int)ws->counters.cap, ws->stream);
  return HG_OK;
}

hg::PixelSet all_pixels(int32_t M) {
  hg::PixelSet ps;
  ps.perm = nullptr;
  ps.idx = nullptr;
  ps.start = 0;
  ps.count = M;
  ps.M = M;
  return ps;
}

hg::PixelSet index_set(const int32_t* idx, int32_t m, int32_t M) {
  if (!idx) return all_pixels(M);
  hg::PixelSet ps = all_pixels(M);
  ps.idx = idx;
  ps.count = m;
  return ps;
}

hg_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(HG_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return HG_OK;
}

// The shared schedule of RS (I = 0), WGS (c < 0) and CS-WGS.
hg_status run_iterations(const hg_grid* g, const hg_optics* o, const hg_spots* s,
                         int32_t iterations, double c, uint64_t seed, uint32_t flags, float* phi,
                         double* trace_host, void* stream) {
  const bool on_device = (flags & HG_SPOTS_ON_DEVICE) != 0;
  HG_TRY(validate(g, o, s, on_device));
  if (iterations < 0 || iterations > HG_MAX_ITERATIONS)
    return fail(HG_EINVAL, "iterations must be in [0, HG_MAX_ITERATIONS]");
  if (!phi) return fail(HG_EINVAL, "phi_dev must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  const int N = s->n;
  const int32_t M = g->W * g->H;
  const bool compressed = c > 0.0 && iterations >= 2;
  const int32_t m = compressed ? subset_size(M, c) : M;

  HG_TRY(upload_spots(ws, g, o, s, seed, on_device, nullptr, nullptr, nullptr));
  if (compressed) HG_TRY(build_order(ws, M, seed));
  const hg::PassPlan plan_all = hg::plan_pass(M);
  const hg::PassPlan plan_sub = hg::plan_pass(m);
  HG_TRY(reserve_pass(ws, plan_all, N));
  HG_TRY(reserve_pass(ws, plan_sub, N));
  HG_TRY(ws->V.reserve((size_t)N * (trace_host && iterations > 0 ? iterations : 1)));

  for (int32_t j = 1; j <= iterations; ++j) {
    hg::PixelSet ps = all_pixels(M);
    const bool sub = compressed && j < iterations;
    if (sub) {
      ps.perm = ws->perm.p;
      ps.start = (int64_t)(j - 1) * m % M;
      ps.count = m;
    }
    double2* Vj = ws->V.p + (trace_host ? (size_t)(j - 1) * N : 0);
    ws->timed_launch(sub ? "k_pass_subset" : "k_pass_full", [&] {
      hg::launch_pass(sub ? plan_sub : plan_all, ws->sp.p, N, g->W, g->H, ps, nullptr,
                      ws->partial.p, ws->gpart.p, ws->counters.p, Vj, ws->status.p, true,
                      ws->stream);
    });
  }
  ws->timed_launch("k_backprop_phi", [&] {
    hg::launch_backprop_phi(ws->sp.p, N, g->W, g->H, all_pixels(M), phi, ws->stream);
  });
  HG_TRY(check_launch());
  if (trace_host) {
    if (iterations > 0)
      HG_HIP(hipMemcpyAsync(trace_host, ws->V.p, sizeof(double2) * (size_t)N * iterations,
                            hipMemcpyDeviceToHost, ws->stream));
    HG_HIP(hipStreamSynchronize(ws->stream));
    HG_TRY(ws->take_status());
  }
  return HG_OK;
}

hg_status check_set(const hg_grid* grid, const int32_t* idx_dev, int32_t m) {
  if (idx_dev && (m < 1 || (int64_t)m > (int64_t)grid->W * grid->H))
    return fail(HG_EINVAL, "m must be in [1, W*H] when idx_dev is given");
  return HG_OK;
}

hg_status check_state(const hg_spots* spots, const double* w, const double* theta) {
  if (!w || !theta) return fail(HG_EINVAL, "w and theta must be non-NULL");
  for (int n = 0; n < spots->n; ++n)
    if (!finite_pos(w[n]) || !std::isfinite(theta[n]))
      return fail(HG_EINVAL, "w must be positive and finite, theta finite");
  return HG_OK;
}

}  // namespace

extern "C" {

const char* hg_last_error(void) { return g_err.c_str(); }

const char* hg_version(void) { return "libhg 0.1 (gfx950)"; }

hg_status hg_rs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                uint64_t seed, float* phi_dev, void* stream) {
  return run_iterations(grid, optics, spots, 0, -1.0, seed, 0, phi_dev, nullptr, stream);
}

hg_status hg_wgs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                 int32_t iterations, uint64_t seed, float* phi_dev, void* stream) {
  return run_iterations(grid, optics, spots, iterations, -1.0, seed, 0, phi_dev, nullptr,
                        stream);
}

hg_status hg_cswgs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                   int32_t iterations, double compression, uint64_t seed, float* phi_dev,
                   void* stream) {
  if (!(compression > 0.0 && compression <= 1.0))
    return fail(HG_EINVAL, "compression must be in (0, 1]");
  return run_iterations(grid, optics, spots, iterations, compression, seed, 0, phi_dev, nullptr,
                        stream);
}

hg_status hg_cswgs_ex(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                      const hg_params* params, float* phi_dev, void* stream) {
  if (!params) return fail(HG_EINVAL, "params must be non-NULL");
  if (!(params->compression > 0.0 && params->compression <= 1.0))
    return fail(HG_EINVAL, "compression must be in (0, 1]");
  HG_TRY(validate_flags(params->flags, HG_SPOTS_ON_DEVICE));
  return run_iterations(grid, optics, spots, params->iterations, params->compression,
                        params->seed, params->flags, phi_dev, params->trace_V, stream);
}

hg_status hg_metrics(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                     const float* phi_dev, double* e, double* u, double* intensities,
                     void* stream) {
  HG_TRY(validate(grid, optics, spots, false));
  if (!phi_dev || !e || !u) return fail(HG_EINVAL, "phi_dev, e and u must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  const int N = spots->n;
  hg::SpotPtrs in;
  HG_TRY(upload_spots(ws, grid, optics, spots, 0, false, nullptr, nullptr, &in));
  HG_TRY(ws->Ex.reserve((size_t)grid->W * N));
  HG_TRY(ws->Ey.reserve((size_t)grid->H * N));
  const int nblk = hg::metric_blocks(grid->H);
  HG_TRY(ws->mpart.reserve((size_t)nblk * N));
  HG_TRY(ws->V.reserve(N));
  hg::launch_metric_tables(setup_args(grid, optics, spots, 0), in, ws->Ex.p, ws->Ey.p,
                           ws->stream);
  hg::launch_metric_rows(ws->Ex.p, ws->Ey.p, N, grid->W, grid->H, phi_dev, ws->mpart.p,
                         ws->stream);
  hg::launch_metric_reduce(ws->mpart.p, nblk, N, 1.0 / ((double)grid->W * grid->H), ws->V.p,
                           ws->stream);
  HG_TRY(check_launch());
  std::vector<double> V(2 * (size_t)N);
  HG_HIP(hipMemcpyAsync(V.data(), ws->V.p, sizeof(double2) * N, hipMemcpyDeviceToHost,
                        ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  HG_TRY(ws->take_status());
  double sum = 0.0, lo = INFINITY, hi = -INFINITY;
  for (int n = 0; n < N; ++n) {
    const double I = V[2 * n] * V[2 * n] + V[2 * n + 1] * V[2 * n + 1];
    if (intensities) intensities[n] = I;
    sum += I;
    lo = I < lo ? I : lo;
    hi = I > hi ? I : hi;
  }
  *e = sum;
  *u = (hi + lo) > 0.0 ? 1.0 - (hi - lo) / (hi + lo) : 0.0;
  return HG_OK;
}

hg_status hg_theta0(uint64_t seed, int32_t count, double* out_host) {
  if (count < 1 || count > HG_MAX_SPOTS || !out_host)
    return fail(HG_EINVAL, "count must be in [1, HG_MAX_SPOTS] and out_host non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(nullptr, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->raw.reserve((size_t)6 * count));
  hg::launch_theta0(seed, count, ws->raw.p, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipMemcpyAsync(out_host, ws->raw.p, sizeof(double) * count, hipMemcpyDeviceToHost,
                        ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  return HG_OK;
}

hg_status hg_subset(const hg_grid* grid, uint64_t seed, int32_t j, double compression,
                    int32_t* idx_dev, int32_t* m_out, void* stream) {
  if (!grid || grid->W < 1 || grid->H < 1 || grid->W > 8192 || grid->H > 8192)
    return fail(HG_EINVAL, "grid W and H must be in [1, 8192]");
  if (j < 1) return fail(HG_EINVAL, "j must be >= 1");
  if (!(compression > 0.0 && compression <= 1.0))
    return fail(HG_EINVAL, "compression must be in (0, 1]");
  if (!idx_dev || !m_out) return fail(HG_EINVAL, "idx_dev and m_out must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  const int32_t M = grid->W * grid->H;
  const int32_t m = subset_size(M, compression);
  HG_TRY(build_order(ws, M, seed));
  hg::PixelSet ps = all_pixels(M);
  ps.perm = ws->perm.p;
  ps.start = (int64_t)(j - 1) * m % M;
  ps.count = m;
  hg::launch_gather(ps, idx_dev, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipStreamSynchronize(ws->stream));
  *m_out = m;
  return HG_OK;
}

hg_status hg_forward(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                     const float* phi_dev, const int32_t* idx_dev, int32_t m, uint32_t flags,
                     double* V_out, void* stream) {
  HG_TRY(validate(grid, optics, spots, false));
  HG_TRY(validate_flags(flags, 0));
  HG_TRY(check_set(grid, idx_dev, m));
  if (!phi_dev || !V_out) return fail(HG_EINVAL, "phi_dev and V_out must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  const int N = spots->n;
  const int32_t M = grid->W * grid->H;
  HG_TRY(upload_spots(ws, grid, optics, spots, 0, false, nullptr, nullptr, nullptr));
  const hg::PixelSet ps = index_set(idx_dev, m, M);
  const hg::PassPlan plan = hg::plan_pass(ps.count);
  HG_TRY(reserve_pass(ws, plan, N));
  HG_TRY(ws->V.reserve(N));
  hg::launch_pass(plan, ws->sp.p, N, grid->W, grid->H, ps, phi_dev, ws->partial.p, ws->gpart.p,
                  ws->counters.p, ws->V.p, ws->status.p, false, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipMemcpyAsync(V_out, ws->V.p, sizeof(double2) * N, hipMemcpyDeviceToHost, ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  return ws->take_status();
}

hg_status hg_backward(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                      const double* w, const double* theta, const int32_t* idx_dev, int32_t m,
                      uint32_t flags, float* phi_dev, void* stream) {
  HG_TRY(validate(grid, optics, spots, false));
  HG_TRY(validate_flags(flags, 0));
  HG_TRY(check_state(spots, w, theta));
  HG_TRY(check_set(grid, idx_dev, m));
  if (!phi_dev) return fail(HG_EINVAL, "phi_dev must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(upload_spots(ws, grid, optics, spots, 0, false, w, theta, nullptr));
  hg::launch_backprop_phi(ws->sp.p, spots->n, grid->W, grid->H,
                          index_set(idx_dev, m, grid->W * grid->H), phi_dev, ws->stream);
  return check_launch();
}

hg_status hg_step(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                  const double* w, const double* theta, const int32_t* idx_dev, int32_t m,
                  uint32_t flags, double* V_out, void* stream) {
  HG_TRY(validate(grid, optics, spots, false));
  HG_TRY(validate_flags(flags, 0));
  HG_TRY(check_state(spots, w, theta));
  HG_TRY(check_set(grid, idx_dev, m));
  if (!V_out) return fail(HG_EINVAL, "V_out must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  const int N = spots->n;
  HG_TRY(upload_spots(ws, grid, optics, spots, 0, false, w, theta, nullptr));
  const hg::PixelSet ps = index_set(idx_dev, m, grid->W * grid->H);
  const hg::PassPlan plan = hg::plan_pass(ps.count);
  HG_TRY(reserve_pass(ws, plan, N));
  HG_TRY(ws->V.reserve(N));
  hg::launch_pass(plan, ws->sp.p, N, grid->W, grid->H, ps, nullptr, ws->partial.p, ws->gpart.p,
                  ws->counters.p, ws->V.p, ws->status.p, false, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipMemcpyAsync(V_out, ws->V.p, sizeof(double2) * N, hipMemcpyDeviceToHost, ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  return ws->take_status();
}

hg_status hg_timing_enable(int on) {
  g_timing.store(on != 0);
  return HG_OK;
}

static void drain_all_timing() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    std::lock_guard<std::mutex> wl(kv.second->mu);
    kv.second->drain_timing();
  }
}

hg_status hg_timing_reset(void) {
  drain_all_timing();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_totals.clear();
  return HG_OK;
}

hg_status hg_timing_read(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return fail(HG_EINVAL, "arguments must be non-NULL");
  drain_all_timing();
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_totals.find(name);
  *total_ms = it == g_totals.end() ? 0.0 : it->second.ms;
  *launches = it == g_totals.end() ? 0 : it->second.launches;
  return HG_OK;
}

hg_status hg_release(void) {
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    std::lock_guard<std::mutex> wl(kv.second->mu);
    (void)hipSetDevice(kv.second->device);
    (void)hipDeviceSynchronize();
    kv.second->release();
  }
  g_ws.clear();
  if (have_cur) (void)hipSetDevice(cur);
  return HG_OK;
}

}  // extern "C"
