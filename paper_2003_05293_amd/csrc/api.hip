// C ABI of libhg (include/hg.h): per-stream workspaces and the entry points.
// Every algorithm call is a batch of one hologram on the stream's workspace.
#include <hip/hip_runtime.h>

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
#include "runtime.hpp"

// Device memory of hg_cswgs_static, which works in this array instead of
// allocated memory (zero at load; each GPU holds its own copy).  In host
// code `scratch` names a host-side stand-in, not the device array: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
static __device__ __align__(256) char scratch[HG_STATIC_SCRATCH_BYTES];

namespace {

using hg::set_error;

// Scratch of one (device, stream).  Calls on the same stream run in stream
// order, so the buffers are reused from call to call.  `status` is sticky:
// kernels raise it, blocking calls report and clear it.
struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  hg::Batch batch;
  hg::DevBuf<int32_t> status;
  hg::DevBuf<double> raw;             // metrics: spot inputs; theta0 output
  hg::DevBuf<double2> Ex, Ey, mpart, V;
  hg::Staging staging;

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
      return set_error(HG_EINVAL, "device-resident spot values were not finite or an amplitude "
                                  "was not positive (in this or an earlier call on this stream)");
    return set_error(HG_ENUMERIC, "a spot field came out zero or not finite (in this or an "
                                  "earlier call on this stream)");
  }

  void release() {
    batch.release();
    status.release();
    raw.release();
    Ex.release();
    Ey.release();
    mpart.release();
    V.release();
    staging.release();
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

hg_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(HG_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return HG_OK;
}

hg_status validate_flags(uint32_t flags, uint32_t allowed_extra) {
  if (flags & ~(HG_PREC_MASK | allowed_extra)) return set_error(HG_EINVAL, "flags: unknown bits set");
  const uint32_t prec = flags & HG_PREC_MASK;
  if (prec != HG_PREC_FP32 && prec != HG_PREC_MIXED)
    return set_error(HG_EINVAL, "flags: precision must be HG_PREC_FP32 or HG_PREC_MIXED");
  if (prec == HG_PREC_MIXED && (flags & HG_FULL_DIRECT))
    return set_error(HG_EINVAL, "flags: HG_FULL_DIRECT applies to HG_PREC_FP32 only");
  return HG_OK;
}

hg_status check_compression(double c) {
  if (!(c > 0.0 && c <= 1.0)) return set_error(HG_EINVAL, "compression must be in (0, 1]");
  return HG_OK;
}

hg::TuneParams tune_params(const hg_tune* t) {
  hg::TuneParams tp;
  if (t && t->full_block_cap > 0) tp.full_block_cap = t->full_block_cap;
  if (t && t->subset_block_cap > 0) tp.subset_block_cap = t->subset_block_cap;
  if (t) tp.pass_form = t->pass_form;
  if (t) tp.chain_passes = t->chain_passes != 0;
  return tp;
}

// The shared schedule of RS (I = 0), WGS (c < 0) and CS-WGS: a batch of one.
hg_status run_one(const hg_grid* g, const hg_optics* o, const hg_spots* s, int32_t iterations,
                  double c, uint64_t seed, uint32_t flags, float* phi, double* trace_host,
                  void* stream, const hg::TuneParams& tp = hg::TuneParams{},
                  const hg_lut* lut = nullptr, void* gray = nullptr) {
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(g, o, s, iterations, c, seed, flags, phi, trace_host, &spec));
  HG_TRY(hg::apply_lut(lut, gray, &spec));
  if (!phi) return set_error(HG_EINVAL, "phi_dev must be non-NULL");
  HG_TRY(hg::attach_shared_order(&spec));
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(&spec, 1, tp, ws->status.p, /*allow_chain=*/true));
  HG_TRY(ws->batch.enqueue(ws->stream));
  if (trace_host) {
    HG_TRY(ws->batch.fetch_traces(ws->stream));
    HG_HIP(hipStreamSynchronize(ws->stream));
    HG_TRY(ws->take_status());
  }
  return HG_OK;
}

hg_status check_params(const hg_params* params) {
  if (!params) return set_error(HG_EINVAL, "params must be non-NULL");
  HG_TRY(check_compression(params->compression));
  HG_TRY(validate_flags(params->flags, HG_SPOTS_ON_DEVICE | HG_FULL_DIRECT));
  if (params->tune.full_block_cap < 0 || params->tune.subset_block_cap < 0 ||
      params->tune.pass_form < 0 || params->tune.pass_form > 1 ||
      params->tune.chain_passes < 0 || params->tune.chain_passes > 1)
    return set_error(HG_EINVAL, "tune caps must be >= 0, pass_form and chain_passes 0 or 1");
  return HG_OK;
}

// ------------------------------------------------ static scratch (no alloc) --
// Layout of one copy of `scratch`: [0, 256) the status word, then the job
// scratch, and the descriptor tables in the last kStaticTableBytes.
constexpr size_t kStaticTableBytes = size_t(1) << 20;
constexpr size_t kStaticArenaOffset = 256;
constexpr int kStaticMaxDevices = 64;
static_assert(HG_STATIC_SCRATCH_BYTES > kStaticArenaOffset + kStaticTableBytes, "scratch layout");

struct StaticScratch {
  std::mutex mu;
  bool ready = false;
  char* dev = nullptr;          // this device's copy of `scratch`
  hipEvent_t copied = nullptr;  // the last descriptor upload has read `host`
  hg::Batch batch;
  char host[kStaticTableBytes];  // descriptor staging
};

std::mutex g_static_mu;
StaticScratch* g_static[kStaticMaxDevices] = {};

// Set-up of the current device (first call on it): the address of its copy
// of the array and the upload event.  The status word is zero from load;
// no call of this path reads it.
hg_status static_scratch(StaticScratch** out) {
  int dev = 0;
  HG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kStaticMaxDevices)
    return set_error(HG_EINVAL, "hg_cswgs_static supports devices 0.." +
                                    std::to_string(kStaticMaxDevices - 1));
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static[dev]) g_static[dev] = new StaticScratch();
  StaticScratch* st = g_static[dev];
  if (!st->ready) {
    void* p = nullptr;
    HG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(HG_EDEVICE, "hipGetSymbolAddress gave no address for the scratch");
    HG_HIP(hipEventCreateWithFlags(&st->copied, hipEventDisableTiming));
    st->dev = static_cast<char*>(p);
    st->batch.adopt(st->dev + kStaticArenaOffset,
                    HG_STATIC_SCRATCH_BYTES - kStaticArenaOffset - kStaticTableBytes,
                    st->dev + HG_STATIC_SCRATCH_BYTES - kStaticTableBytes, kStaticTableBytes,
                    st->host, kStaticTableBytes, st->copied);
    st->ready = true;
  }
  *out = st;
  return HG_OK;
}

hg_status check_set(const hg_grid* grid, const int32_t* idx_dev, int32_t m) {
  if (idx_dev && (m < 1 || (int64_t)m > (int64_t)grid->W * grid->H))
    return set_error(HG_EINVAL, "m must be in [1, W*H] when idx_dev is given");
  return HG_OK;
}

hg_status check_state(const hg_spots* spots, const double* w, const double* theta) {
  if (!w || !theta) return set_error(HG_EINVAL, "w and theta must be non-NULL");
  for (int n = 0; n < spots->n; ++n)
    if (!(std::isfinite(w[n]) && w[n] > 0.0) || !std::isfinite(theta[n]))
      return set_error(HG_EINVAL, "w must be positive and finite, theta finite");
  return HG_OK;
}

// The mixed-precision passes work on the whole grid (or a window of the
// random order), not on explicit pixel lists.
hg_status check_mixed_set(uint32_t flags, const int32_t* idx_dev) {
  if ((flags & HG_PREC_MASK) == HG_PREC_MIXED && idx_dev)
    return set_error(HG_EINVAL, "HG_PREC_MIXED hooks take the whole grid: idx_dev must be NULL");
  return HG_OK;
}

hg::PixelSet pixel_set(const int32_t* idx, int32_t m, int32_t M) {
  hg::PixelSet ps;
  ps.perm = nullptr;
  ps.idx = idx;
  ps.start = 0;
  ps.count = idx ? m : M;
  ps.M = M;
  return ps;
}

// Sets the state of the batch's single job to (w, theta) (host arrays).
hg_status set_state(Workspace* ws, int N, const double* w, const double* theta) {
  HG_TRY(ws->raw.reserve(2 * (size_t)N));
  HG_TRY(ws->staging.acquire(sizeof(double) * 2 * N));
  double* st = reinterpret_cast<double*>(ws->staging.p);
  std::memcpy(st, w, sizeof(double) * N);
  std::memcpy(st + N, theta, sizeof(double) * N);
  HG_HIP(hipMemcpyAsync(ws->raw.p, st, sizeof(double) * 2 * N, hipMemcpyHostToDevice,
                        ws->stream));
  HG_TRY(ws->staging.mark_copied(ws->stream));
  hg::launch_set_state(N, ws->raw.p, ws->batch.job(0).sp, ws->batch.job(0).coef, ws->stream);
  return HG_OK;
}

// One pass of the single job over a pixel set, without the weight update;
// V (N complex) is copied to the host.
hg_status single_pass(Workspace* ws, const hg::PixelSet& ps, bool from_phi, double* V_out) {
  const hg::JobDev& j = ws->batch.job(0);
  hg::PassDesc d;
  d.block_begin = 0;
  d.job = 0;
  d.ps = ps;
  d.plan = hg::plan_pass(ps.count, hg::kDefaultBlockCap);
  d.update = 0;
  d.from_phi = from_phi ? 1 : 0;
  d.grab_slot = 0;
  // eq. (3): the mean over the set (the whole grid stands for the pupil)
  d.inv_count = 1.0 / (double)(ps.idx ? ps.count : j.P);
  d.V = j.V;
  void* dev = nullptr;
  HG_TRY(ws->batch.upload_custom(&d, sizeof(d), ws->stream, &dev));
  hg::launch_pass_batch(ws->batch.jobs_device(), reinterpret_cast<const hg::PassDesc*>(dev), 1,
                        d.plan.blocks, hg::pass_units_per_wave(j.N),
                        from_phi || !j.shared_e ? 0 : hg::pass_e_width(j.N), ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipMemcpyAsync(V_out, j.V, sizeof(double2) * j.N, hipMemcpyDeviceToHost, ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  return ws->take_status();
}

// Runs a launch set built for the batch's single job (test hooks).
hg_status single_set(Workspace* ws, hg::LaunchSet& set) {
  char* dev = nullptr;
  HG_TRY(ws->batch.custom_device(set.bytes(), &dev));
  std::vector<char> host(std::max<size_t>(set.bytes(), 1));
  set.stage(host.data(), dev);
  void* up = nullptr;
  HG_TRY(ws->batch.upload_custom(host.data(), host.size(), ws->stream, &up));
  set.launch(ws->batch.jobs_device(), ws->stream, false);
  return check_launch();
}


hg_status job_specs(int32_t count, const hg_job* jobs, const hg_tune* tune,
                    std::vector<hg::JobSpec>* out) {
  if (count < 1 || !jobs) return set_error(HG_EINVAL, "count must be >= 1 and jobs non-NULL");
  if (tune && (tune->full_block_cap < 0 || tune->subset_block_cap < 0 || tune->pass_form < 0 ||
               tune->pass_form > 1 || tune->chain_passes < 0 || tune->chain_passes > 1))
    return set_error(HG_EINVAL, "tune caps must be >= 0, pass_form and chain_passes 0 or 1");
  out->resize(count);
  for (int32_t i = 0; i < count; ++i) {
    const hg_job& j = jobs[i];
    hg_status st = check_compression(j.compression);
    if (st == HG_OK) st = validate_flags(j.flags, HG_SPOTS_ON_DEVICE | HG_FULL_DIRECT);
    if (st == HG_OK)
      st = hg::make_spec(&j.grid, &j.optics, &j.spots, j.iterations, j.compression, j.seed,
                         j.flags, j.phi_dev, j.trace_V, &(*out)[i]);
    if (st == HG_OK && !j.phi_dev) st = set_error(HG_EINVAL, "phi_dev must be non-NULL");
    if (st == HG_OK) st = hg::apply_lut(j.lut, j.gray_dev, &(*out)[i]);
    if (st == HG_OK) st = hg::attach_shared_order(&(*out)[i]);
    if (st != HG_OK) return set_error(st, "job " + std::to_string(i) + ": " + hg::last_error());
  }
  return HG_OK;
}

}  // namespace

// A planned batch that owns its scratch; runs replay a captured graph.
struct hg_batch {
  int device = 0;
  hg::Batch batch;
  hg::DevBuf<int32_t> status;
  bool use_graph = false;
  hipStream_t captured_on = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::mutex mu;
};

extern "C" {

const char* hg_last_error(void) { return hg::last_error(); }

const char* hg_version(void) { return "libhg 0.2 (gfx950)"; }

hg_status hg_rs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                uint64_t seed, float* phi_dev, void* stream) {
  return run_one(grid, optics, spots, 0, -1.0, seed, 0, phi_dev, nullptr, stream);
}

hg_status hg_wgs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                 int32_t iterations, uint64_t seed, float* phi_dev, void* stream) {
  return run_one(grid, optics, spots, iterations, -1.0, seed, 0, phi_dev, nullptr, stream);
}

hg_status hg_cswgs(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                   int32_t iterations, double compression, uint64_t seed, float* phi_dev,
                   void* stream) {
  HG_TRY(check_compression(compression));
  return run_one(grid, optics, spots, iterations, compression, seed, 0, phi_dev, nullptr, stream);
}

hg_status hg_cswgs_ex(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                      const hg_params* params, float* phi_dev, void* stream) {
  HG_TRY(check_params(params));
  return run_one(grid, optics, spots, params->iterations, params->compression, params->seed,
                 params->flags, phi_dev, params->trace_V, stream, tune_params(&params->tune),
                 params->lut, params->gray_dev);
}

hg_status hg_cswgs_static(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                          const hg_params* params, float* phi_dev, void* stream) {
  HG_TRY(check_params(params));
  if (!(params->flags & HG_SPOTS_ON_DEVICE))
    return set_error(HG_EINVAL, "hg_cswgs_static takes device-resident spots: params->flags "
                                "must have HG_SPOTS_ON_DEVICE");
  if (params->trace_V)
    return set_error(HG_EINVAL, "hg_cswgs_static takes no trace: params->trace_V must be NULL");
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(grid, optics, spots, params->iterations, params->compression,
                       params->seed, params->flags, phi_dev, nullptr, &spec));
  HG_TRY(hg::apply_lut(params->lut, params->gray_dev, &spec));
  if (!phi_dev) return set_error(HG_EINVAL, "phi_dev must be non-NULL");
  StaticScratch* st = nullptr;
  HG_TRY(static_scratch(&st));
  std::lock_guard<std::mutex> lk(st->mu);
  HG_TRY(st->batch.build(&spec, 1, tune_params(&params->tune), reinterpret_cast<int32_t*>(st->dev),
                         /*allow_chain=*/true));
  return st->batch.enqueue(static_cast<hipStream_t>(stream));
}

hg_status hg_metrics(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                     const float* phi_dev, double* e, double* u, double* intensities,
                     void* stream) {
  HG_TRY(hg::validate_spec(grid, optics, spots, false));
  if (!phi_dev || !e || !u) return set_error(HG_EINVAL, "phi_dev, e and u must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  const int N = spots->n;
  HG_TRY(ws->raw.reserve(4 * (size_t)N));
  HG_TRY(ws->staging.acquire(sizeof(double) * 4 * N));
  double* st = reinterpret_cast<double*>(ws->staging.p);
  std::memcpy(st, spots->x_mm, sizeof(double) * N);
  std::memcpy(st + N, spots->y_mm, sizeof(double) * N);
  std::memcpy(st + 2 * N, spots->z_mm, sizeof(double) * N);
  std::memcpy(st + 3 * N, spots->amp, sizeof(double) * N);
  HG_HIP(hipMemcpyAsync(ws->raw.p, st, sizeof(double) * 4 * N, hipMemcpyHostToDevice,
                        ws->stream));
  HG_TRY(ws->staging.mark_copied(ws->stream));
  const hg::SpotPtrs in{ws->raw.p, ws->raw.p + N, ws->raw.p + 2 * N, ws->raw.p + 3 * N};
  hg::SetupArgs a;
  a.N = N;
  a.W = grid->W;
  a.H = grid->H;
  a.pitch_mm = grid->pitch_mm;
  a.lambda_mm = optics->lambda_mm;
  a.focal_mm = optics->focal_mm;
  HG_TRY(ws->Ex.reserve((size_t)grid->W * N));
  HG_TRY(ws->Ey.reserve((size_t)grid->H * N));
  const int nblk = hg::metric_blocks(grid->H);
  HG_TRY(ws->mpart.reserve((size_t)nblk * N));
  HG_TRY(ws->V.reserve(N));
  hg::launch_metric_tables(a, in, ws->Ex.p, ws->Ey.p, ws->stream);
  // the pupil: V* is the mean over Omega of A e^{i(Phi - phi_n)}
  const int32_t ap_q = hg::aperture_bound(optics);
  const double ill_a = hg::illumination_exponent(grid->pitch_mm, optics->waist_mm);
  const int64_t P = hg::pupil_count(grid->W, grid->H, ap_q);
  hg::launch_metric_rows(ws->Ex.p, ws->Ey.p, N, grid->W, grid->H, phi_dev, ap_q, ill_a,
                         ws->mpart.p, ws->stream);
  hg::launch_metric_reduce(ws->mpart.p, nblk, N, 1.0 / (double)P, ws->V.p, ws->stream);
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
  // the fraction of the power on the SLM, mean_Omega(A^2), in the spots
  *e = sum / hg::pupil_power(grid->W, grid->H, ap_q, ill_a);
  *u = (hi + lo) > 0.0 ? 1.0 - (hi - lo) / (hi + lo) : 0.0;
  return HG_OK;
}

hg_status hg_lut_create(const uint16_t* gray, int32_t levels, int32_t bits, hg_lut** out) {
  if (!gray || !out) return set_error(HG_EINVAL, "gray and out must be non-NULL");
  if (levels < 1 || levels > 65536) return set_error(HG_EINVAL, "levels must be in [1, 65536]");
  if (bits != 8 && bits != 16) return set_error(HG_EINVAL, "bits must be 8 or 16");
  if (bits == 8)
    for (int32_t k = 0; k < levels; ++k)
      if (gray[k] > 255) return set_error(HG_EINVAL, "8-bit tables hold values <= 255");
  std::unique_ptr<hg_lut> lut(new hg_lut());
  lut->levels = levels;
  lut->bits = bits;
  HG_HIP(hipGetDevice(&lut->device));
  HG_HIP(hipMalloc(reinterpret_cast<void**>(&lut->dev), sizeof(uint16_t) * (size_t)levels));
  const hipError_t e =
      hipMemcpy(lut->dev, gray, sizeof(uint16_t) * (size_t)levels, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(lut->dev);
    return set_error(HG_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *out = lut.release();
  return HG_OK;
}

hg_status hg_lut_destroy(hg_lut* lut) {
  if (!lut) return HG_OK;
  int cur = 0;
  HG_HIP(hipGetDevice(&cur));
  HG_HIP(hipSetDevice(lut->device));
  const hipError_t e = hipFree(lut->dev);
  (void)hipSetDevice(cur);
  delete lut;
  if (e != hipSuccess) return set_error(HG_EDEVICE, std::string("hipFree: ") + hipGetErrorString(e));
  return HG_OK;
}

hg_status hg_phase_to_gray(const hg_lut* lut, const float* phi_dev, int64_t count, void* gray_dev,
                           void* stream) {
  if (!lut || !lut->dev || !phi_dev || !gray_dev)
    return set_error(HG_EINVAL, "lut, phi_dev and gray_dev must be non-NULL");
  if (count < 0) return set_error(HG_EINVAL, "count must be >= 0");
  hg::launch_phase_to_gray(phi_dev, count, lut->dev, lut->levels, lut->bits, gray_dev,
                           static_cast<hipStream_t>(stream));
  return check_launch();
}

hg_status hg_theta0(uint64_t seed, int32_t count, double* out_host) {
  if (count < 1 || count > HG_MAX_SPOTS || !out_host)
    return set_error(HG_EINVAL, "count must be in [1, HG_MAX_SPOTS] and out_host non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(nullptr, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->raw.reserve((size_t)count));
  hg::launch_theta0(seed, count, ws->raw.p, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipMemcpyAsync(out_host, ws->raw.p, sizeof(double) * count, hipMemcpyDeviceToHost,
                        ws->stream));
  HG_HIP(hipStreamSynchronize(ws->stream));
  return HG_OK;
}

hg_status hg_subset(const hg_grid* grid, const hg_optics* optics, uint64_t seed, int32_t j,
                    double compression, int32_t* idx_dev, int32_t* m_out, void* stream) {
  HG_TRY(hg::validate_grid(grid));
  if (j < 1) return set_error(HG_EINVAL, "j must be >= 1");
  HG_TRY(check_compression(compression));
  if (!idx_dev || !m_out) return set_error(HG_EINVAL, "idx_dev and m_out must be non-NULL");
  // a one-spot job carries the random order of this grid, pupil and seed
  const double zero = 0.0, one = 1.0;
  const hg_spots s{1, &zero, &zero, &zero, &one};
  const hg_optics o{1.0, 1.0, 0.0, optics ? optics->aperture_px : 0.0};
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(grid, &o, &s, 2, compression, seed, 0, nullptr, nullptr, &spec));
  spec.order_key = seed;
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(&spec, 1, hg::TuneParams{}, ws->status.p));
  HG_TRY(ws->batch.enqueue_prologue(ws->stream));
  const hg::JobDev& jb = ws->batch.job(0);
  hg::PixelSet ps = pixel_set(nullptr, 0, jb.P);
  ps.perm = jb.perm;
  ps.start = (int64_t)(j - 1) * jb.m % jb.P;
  ps.count = jb.m;
  hg::launch_gather(ps, idx_dev, ws->stream);
  HG_TRY(check_launch());
  HG_HIP(hipStreamSynchronize(ws->stream));
  *m_out = jb.m;
  return HG_OK;
}

hg_status hg_forward(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                     const float* phi_dev, const int32_t* idx_dev, int32_t m, uint32_t flags,
                     double* V_out, void* stream) {
  HG_TRY(validate_flags(flags, 0));
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(grid, optics, spots, 0, -1.0, 0, flags, const_cast<float*>(phi_dev),
                       nullptr, &spec));
  spec.hook = true;
  HG_TRY(check_set(grid, idx_dev, m));
  HG_TRY(check_mixed_set(flags, idx_dev));
  if (!phi_dev || !V_out) return set_error(HG_EINVAL, "phi_dev and V_out must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(&spec, 1, hg::TuneParams{}, ws->status.p));
  HG_TRY(ws->batch.enqueue_prologue(ws->stream));
  if (spec.precision == HG_PREC_MIXED) {
    const hg::JobDev& j = ws->batch.job(0);
    hg::LaunchSet set;
    set.add_forward_mx(j, ws->batch.layout(0), 0);
    HG_TRY(single_set(ws, set));
    HG_HIP(hipMemcpyAsync(V_out, j.V, sizeof(double2) * j.N, hipMemcpyDeviceToHost, ws->stream));
    HG_HIP(hipStreamSynchronize(ws->stream));
    return ws->take_status();
  }
  return single_pass(ws, pixel_set(idx_dev, m, grid->W * grid->H), true, V_out);
}

hg_status hg_backward(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                      const double* w, const double* theta, const int32_t* idx_dev, int32_t m,
                      uint32_t flags, float* phi_dev, void* stream) {
  HG_TRY(validate_flags(flags, HG_FULL_DIRECT));
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(grid, optics, spots, 0, -1.0, 0, flags, idx_dev ? nullptr : phi_dev,
                       nullptr, &spec));
  spec.hook = true;
  HG_TRY(check_state(spots, w, theta));
  HG_TRY(check_set(grid, idx_dev, m));
  HG_TRY(check_mixed_set(flags, idx_dev));
  if (!phi_dev) return set_error(HG_EINVAL, "phi_dev must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(&spec, 1, hg::TuneParams{}, ws->status.p));
  HG_TRY(ws->batch.enqueue_prologue(ws->stream));
  HG_TRY(set_state(ws, spots->n, w, theta));
  if (!idx_dev && !(flags & HG_FULL_DIRECT)) {
    hg::LaunchSet set;
    set.add_final(ws->batch.job(0), ws->batch.layout(0), 0);
    return single_set(ws, set);
  }
  hg::BackDesc d;
  d.block_begin = 0;
  d.job = 0;
  d.ps = pixel_set(idx_dev, m, grid->W * grid->H);
  d.out = phi_dev;
  void* dev = nullptr;
  HG_TRY(ws->batch.upload_custom(&d, sizeof(d), ws->stream, &dev));
  hg::launch_backprop_batch(ws->batch.jobs_device(), reinterpret_cast<const hg::BackDesc*>(dev), 1,
                            hg::backprop_blocks(d.ps.count), ws->stream);
  return check_launch();
}

hg_status hg_step(const hg_grid* grid, const hg_optics* optics, const hg_spots* spots,
                  const double* w, const double* theta, const int32_t* idx_dev, int32_t m,
                  uint32_t flags, double* V_out, void* stream) {
  HG_TRY(validate_flags(flags, HG_FULL_DIRECT));
  hg::JobSpec spec;
  HG_TRY(hg::make_spec(grid, optics, spots, 0, -1.0, 0, flags, nullptr, nullptr, &spec));
  spec.hook = true;
  HG_TRY(check_state(spots, w, theta));
  HG_TRY(check_set(grid, idx_dev, m));
  HG_TRY(check_mixed_set(flags, idx_dev));
  if (!V_out) return set_error(HG_EINVAL, "V_out must be non-NULL");
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(&spec, 1, hg::TuneParams{}, ws->status.p));
  HG_TRY(ws->batch.enqueue_prologue(ws->stream));
  HG_TRY(set_state(ws, spots->n, w, theta));
  if (!idx_dev && !(flags & HG_FULL_DIRECT)) {
    // one full-grid iteration body with the separable products, no update
    const hg::JobDev& j = ws->batch.job(0);
    hg::JobDev jj = j;
    jj.iterations = 1;
    hg::LaunchSet set;
    set.add_iteration(jj, ws->batch.layout(0), 1, 0);
    if (!set.sep.empty()) set.sep[0].update = 0;
    if (!set.mx.empty()) set.mx[0].update = 0;
    HG_TRY(single_set(ws, set));
    HG_HIP(hipMemcpyAsync(V_out, j.V, sizeof(double2) * j.N, hipMemcpyDeviceToHost, ws->stream));
    HG_HIP(hipStreamSynchronize(ws->stream));
    return ws->take_status();
  }
  return single_pass(ws, pixel_set(idx_dev, m, grid->W * grid->H), false, V_out);
}

hg_status hg_cswgs_batch(int32_t count, const hg_job* jobs, const hg_tune* tune, void* stream) {
  std::vector<hg::JobSpec> specs;
  HG_TRY(job_specs(count, jobs, tune, &specs));
  Workspace* ws = nullptr;
  HG_TRY(get_workspace(stream, &ws));
  std::lock_guard<std::mutex> lk(ws->mu);
  HG_TRY(ws->init_status());
  HG_TRY(ws->batch.build(specs.data(), count, tune_params(tune), ws->status.p));
  HG_TRY(ws->batch.enqueue(ws->stream));
  bool trace = false;
  for (const auto& s : specs) trace = trace || s.trace_host;
  if (trace) {
    HG_TRY(ws->batch.fetch_traces(ws->stream));
    HG_TRY(ws->take_status());
  }
  return HG_OK;
}

hg_status hg_batch_create(int32_t count, const hg_job* jobs, const hg_tune* tune,
                          int32_t use_graph, hg_batch** out) {
  if (!out) return set_error(HG_EINVAL, "out must be non-NULL");
  std::vector<hg::JobSpec> specs;
  HG_TRY(job_specs(count, jobs, tune, &specs));
  for (int32_t i = 0; i < count; ++i) {
    if (!specs[i].spots_on_device)
      return set_error(HG_EINVAL, "hg_batch_create: every job needs HG_SPOTS_ON_DEVICE");
    if (specs[i].trace_host) return set_error(HG_EINVAL, "hg_batch_create: traces are not allowed");
  }
  auto b = std::make_unique<hg_batch>();
  HG_HIP(hipGetDevice(&b->device));
  b->use_graph = use_graph != 0;
  HG_TRY(b->status.reserve(1));
  HG_HIP(hipMemset(b->status.p, 0, sizeof(int32_t)));
  HG_TRY(b->batch.build(specs.data(), count, tune_params(tune), b->status.p));
  *out = b.release();
  return HG_OK;
}

hg_status hg_batch_run(hg_batch* b, void* stream) {
  if (!b) return set_error(HG_EINVAL, "batch must be non-NULL");
  std::lock_guard<std::mutex> lk(b->mu);
  hipStream_t s = (hipStream_t)stream;
  if (!b->use_graph) return b->batch.enqueue(s);
  if (!s) return set_error(HG_EINVAL, "graph runs need a non-NULL stream");
  if (b->exec && b->captured_on != s) {
    (void)hipGraphExecDestroy(b->exec);
    (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
  }
  if (!b->exec) {
    HG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hg_status st = b->batch.enqueue(s, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != HG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess)
      return set_error(HG_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    b->graph = g;
    HG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->captured_on = s;
  }
  hg::timed(s, "hg_batch", [&] { (void)hipGraphLaunch(b->exec, s); });
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(HG_EDEVICE, std::string("graph launch failed: ") + hipGetErrorString(e));
  return HG_OK;
}

hg_status hg_batch_destroy(hg_batch* b) {
  if (!b) return HG_OK;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->batch.release();
    b->status.release();
    if (have_cur) (void)hipSetDevice(cur);
  }
  delete b;
  return HG_OK;
}

hg_status hg_timing_enable(int on) {
  hg::timing_enable(on != 0);
  return HG_OK;
}

hg_status hg_timing_reset(void) { return hg::timing_reset(); }

hg_status hg_timing_read(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return set_error(HG_EINVAL, "arguments must be non-NULL");
  return hg::timing_read(name, total_ms, launches);
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
  hg::release_shared_orders();
  return HG_OK;
}

}  // extern "C"
