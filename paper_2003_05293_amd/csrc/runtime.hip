// Host runtime of libhg: error state, staging, validation, batch planning and
// the RS / WGS / CS-WGS schedules (paper section 2) as batched launches.
#include "runtime.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace hg {

// ------------------------------------------------------------------ errors --

namespace {
thread_local std::string g_err;
}

hg_status set_error(hg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

const char* last_error() { return g_err.c_str(); }

// ----------------------------------------------------------------- staging --

hg_status Staging::acquire(size_t bytes) {
  if (pending) {
    HG_HIP(hipEventSynchronize(done));
    pending = false;
  }
  if (bytes > cap && adopted)
    return set_error(HG_ENOMEM, "the request needs " + std::to_string(bytes) +
                                    " bytes of descriptor staging, more than the " +
                                    std::to_string(cap) + " of the static area");
  if (bytes > cap) {
    if (p) HG_HIP(hipHostFree(p));
    p = nullptr;
    cap = 0;
    HG_HIP(hipHostMalloc((void**)&p, bytes, hipHostMallocDefault));
    cap = bytes;
  }
  if (!done) HG_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  return HG_OK;
}

hg_status Staging::mark_copied(hipStream_t s) {
  HG_HIP(hipEventRecord(done, s));
  pending = true;
  return HG_OK;
}

void Staging::adopt(char* q, size_t n, hipEvent_t ev) {
  p = q;
  cap = n;
  done = ev;
  pending = false;
  adopted = true;
}

void Staging::release() {
  if (pending && done) (void)hipEventSynchronize(done);
  if (p && !adopted) (void)hipHostFree(p);
  if (done && !adopted) (void)hipEventDestroy(done);
  p = nullptr;
  cap = 0;
  done = nullptr;
  pending = false;
  adopted = false;
}

// -------------------------------------------------------------- validation --

namespace {
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }
}  // namespace

hg_status validate_grid(const hg_grid* g) {
  if (!g) return set_error(HG_EINVAL, "grid must be non-NULL");
  if (g->W < 1 || g->H < 1 || g->W > 8192 || g->H > 8192)
    return set_error(HG_EINVAL, "grid W and H must be in [1, 8192]");
  if (!finite_pos(g->pitch_mm)) return set_error(HG_EINVAL, "pitch_mm must be positive and finite");
  return HG_OK;
}

int32_t aperture_bound(const hg_optics* o) {
  const double D = o->aperture_px;
  if (!(D > 0.0)) return -1;
  const double q = std::floor(D * D);  // Lx^2 + Ly^2 <= D^2 for integers
  return q >= 2147483647.0 ? 2147483647 : (int32_t)q;
}

int64_t pupil_count(int32_t W, int32_t H, int32_t q) {
  int64_t n = 0;
  for (int32_t j = 0; j < H; ++j) {
    int32_t i0, i1;
    n += pupil_run(W, H, q, j, &i0, &i1);
  }
  return n;
}

double illumination_exponent(double pitch_mm, double waist_mm) {
  // A = exp(-(x'^2 + y'^2) / w^2) with x'^2 + y'^2 = Q pitch^2 / 4
  return waist_mm > 0.0 ? pitch_mm * pitch_mm / (4.0 * waist_mm * waist_mm) : 0.0;
}

double pupil_power(int32_t W, int32_t H, int32_t q, double ill_a) {
  if (!(ill_a > 0.0)) return 1.0;
  // A^2 = exp(-2 a Lx^2) exp(-2 a Ly^2), summed over each row's run
  std::vector<double> ex((size_t)W);
  for (int32_t i = 0; i < W; ++i) {
    const double lx = 2.0 * i - (W - 1);
    ex[(size_t)i] = std::exp(-2.0 * ill_a * lx * lx);
  }
  double total = 0.0;
  int64_t count = 0;
  for (int32_t j = 0; j < H; ++j) {
    int32_t i0, i1;
    const int32_t c = pupil_run(W, H, q, j, &i0, &i1);
    if (c == 0) continue;
    const double ly = 2.0 * j - (H - 1);
    double row = 0.0;
    for (int32_t i = i0; i <= i1; ++i) row += ex[(size_t)i];
    total += row * std::exp(-2.0 * ill_a * ly * ly);
    count += c;
  }
  return total / (double)count;
}

hg_status validate_spec(const hg_grid* g, const hg_optics* o, const hg_spots* s, bool on_device) {
  if (!g || !o || !s) return set_error(HG_EINVAL, "grid, optics and spots must be non-NULL");
  HG_TRY(validate_grid(g));
  if (!finite_pos(o->lambda_mm) || !finite_pos(o->focal_mm))
    return set_error(HG_EINVAL, "lambda_mm and focal_mm must be positive and finite");
  if (!std::isfinite(o->waist_mm) || !(o->waist_mm >= 0.0) || !std::isfinite(o->aperture_px) ||
      !(o->aperture_px >= 0.0))
    return set_error(HG_EINVAL, "waist_mm and aperture_px must be finite and >= 0");
  if (pupil_count(g->W, g->H, aperture_bound(o)) == 0)
    return set_error(HG_EINVAL, "the aperture contains no pixel");
  if (s->n < 1 || s->n > HG_MAX_SPOTS)
    return set_error(HG_EINVAL, "spot count must be in [1, HG_MAX_SPOTS]");
  if (!s->x_mm || !s->y_mm || !s->z_mm || !s->amp)
    return set_error(HG_EINVAL, "spot arrays must be non-NULL");
  if (on_device) return HG_OK;  // values are checked by the setup kernel
  for (int n = 0; n < s->n; ++n) {
    if (!std::isfinite(s->x_mm[n]) || !std::isfinite(s->y_mm[n]) || !std::isfinite(s->z_mm[n]))
      return set_error(HG_EINVAL, "spot coordinates must be finite");
    if (!finite_pos(s->amp[n]))
      return set_error(HG_EINVAL, "spot amplitudes must be positive and finite");
  }
  return HG_OK;
}

hg_status apply_lut(const hg_lut* lut, void* gray, JobSpec* spec) {
  if (!lut && !gray) return HG_OK;
  if (!lut || !gray) return set_error(HG_EINVAL, "lut and gray_dev must be both NULL or both set");
  if (!lut->dev || lut->levels < 1 || (lut->bits != 8 && lut->bits != 16))
    return set_error(HG_EINVAL, "lut is not a live table of hg_lut_create");
  spec->lut = lut->dev;
  spec->lut_levels = lut->levels;
  spec->gray_bits = lut->bits;
  spec->gray = gray;
  return HG_OK;
}

hg_status make_spec(const hg_grid* g, const hg_optics* o, const hg_spots* s, int32_t iterations,
                    double compression, uint64_t seed, uint32_t flags, float* phi,
                    double* trace_host, JobSpec* out) {
  const bool on_device = (flags & HG_SPOTS_ON_DEVICE) != 0;
  HG_TRY(validate_spec(g, o, s, on_device));
  if (iterations < 0 || iterations > HG_MAX_ITERATIONS)
    return set_error(HG_EINVAL, "iterations must be in [0, HG_MAX_ITERATIONS]");
  JobSpec j;
  j.W = g->W;
  j.H = g->H;
  j.pitch_mm = g->pitch_mm;
  j.lambda_mm = o->lambda_mm;
  j.focal_mm = o->focal_mm;
  j.waist_mm = o->waist_mm;
  j.ap_q = aperture_bound(o);
  j.pupil_n = (int32_t)pupil_count(g->W, g->H, j.ap_q);
  j.N = s->n;
  j.x = s->x_mm;
  j.y = s->y_mm;
  j.z = s->z_mm;
  j.amp = s->amp;
  j.spots_on_device = on_device;
  j.iterations = iterations;
  j.compression = compression;
  j.seed = seed;
  j.precision = flags & HG_PREC_MASK;
  j.full_direct = (flags & HG_FULL_DIRECT) != 0;
  j.phi = phi;
  j.trace_host = trace_host;
  *out = j;
  return HG_OK;
}

// ------------------------------------------------------------------ timing --

namespace {
std::atomic<bool> g_timing{false};
struct TimedLaunch {
  const char* name;
  hipEvent_t start, stop;
  int count;  // launches between the two events
};
struct Totals {
  double ms = 0.0;
  int64_t launches = 0;
};
std::mutex g_tmu;
std::vector<TimedLaunch> g_pending;
std::map<std::string, Totals> g_totals;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_locked() {
  for (const TimedLaunch& t : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
      Totals& tt = g_totals[t.name];
      tt.ms += ms;
      tt.launches += t.count;
    }
    g_pool.push_back(t.start);
    g_pool.push_back(t.stop);
  }
  g_pending.clear();
}
}  // namespace

bool timing_enabled() { return g_timing.load(std::memory_order_relaxed); }
void timing_enable(bool on) { g_timing.store(on); }

hipEvent_t timing_start(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_tmu);
  hipEvent_t e = pool_event();
  if (e) (void)hipEventRecord(e, s);
  return e;
}

void timing_stop(hipStream_t s, const char* name, hipEvent_t start, int count) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!start) return;
  hipEvent_t e = pool_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_pending.push_back(TimedLaunch{name, start, e, count});
}

hg_status timing_reset() {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  g_totals.clear();
  return HG_OK;
}

hg_status timing_read(const char* name, double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_tmu);
  drain_locked();
  auto it = g_totals.find(name);
  *total_ms = it == g_totals.end() ? 0.0 : it->second.ms;
  *launches = it == g_totals.end() ? 0 : it->second.launches;
  return HG_OK;
}

// ------------------------------------------------------------------- batch --

namespace {

int half_bits(int64_t M) {
  int h = 1;
  while ((int64_t(1) << (2 * h)) < M) ++h;
  return h;
}

bool job_compressed(const JobSpec& s) { return s.compression > 0.0 && s.iterations >= 2; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

// ---------------------------------------------------- shared random orders --

namespace {
struct OrderId {
  int dev;
  int32_t W, H, ap_q;
  uint64_t key;
  bool operator<(const OrderId& o) const {
    return std::tie(dev, W, H, ap_q, key) < std::tie(o.dev, o.W, o.H, o.ap_q, o.key);
  }
};
// Device memory of one order: [JobDev][JobSlice][PrologueSlice][tables][perm][rows].
struct OrderEntry {
  int dev = 0;
  DevBuf<char> mem;
  uint32_t* tab = nullptr;
  int32_t* perm = nullptr;
  int32_t* rows = nullptr;
};
std::mutex g_order_mu;
std::map<OrderId, std::unique_ptr<OrderEntry>> g_orders;
std::map<int, hipStream_t> g_order_streams;  // per device, default priority

// Builds the order with the setup and permutation kernels of the jobs (a
// job of no spots whose tables, pupil rows and permutation are the order's)
// on the device's own stream, and waits for it.
hg_status build_order(OrderEntry& e, const JobSpec& s, int dev) {
  JobDev od = JobDev{};
  od.W = s.W;
  od.H = s.H;
  od.M = s.W * s.H;
  od.P = s.pupil_n > 0 ? s.pupil_n : od.M;
  od.ap_q = s.ap_q;
  od.compressed = 1;
  od.h = half_bits(od.P);
  od.order_key = s.order_key;
  const size_t o_slice = align_up(sizeof(JobDev), 256);
  const size_t o_pro = align_up(o_slice + sizeof(JobSlice), 256);
  const size_t o_tab = align_up(o_pro + sizeof(PrologueSlice), 256);
  const size_t o_perm = align_up(o_tab + sizeof(uint32_t) * ((size_t)kFeistelRoundsHost << od.h), 256);
  const size_t o_rows = align_up(o_perm + sizeof(int32_t) * (size_t)od.P, 256);
  const size_t total = o_rows + (s.ap_q >= 0 ? sizeof(int32_t) * (2 * (size_t)s.H + 1) : 0);
  HG_TRY(e.mem.reserve(total));
  e.dev = dev;
  e.tab = reinterpret_cast<uint32_t*>(e.mem.p + o_tab);
  e.perm = reinterpret_cast<int32_t*>(e.mem.p + o_perm);
  e.rows = s.ap_q >= 0 ? reinterpret_cast<int32_t*>(e.mem.p + o_rows) : nullptr;
  od.tab = e.tab;
  od.perm = e.perm;
  od.rows = e.rows;
  const JobSlice slice{0, 0};
  const PrologueSlice pro{0, 0, prologue_setup_blocks(od), 0};
  HG_HIP(hipMemcpy(e.mem.p, &od, sizeof(JobDev), hipMemcpyHostToDevice));
  HG_HIP(hipMemcpy(e.mem.p + o_slice, &slice, sizeof(JobSlice), hipMemcpyHostToDevice));
  HG_HIP(hipMemcpy(e.mem.p + o_pro, &pro, sizeof(PrologueSlice), hipMemcpyHostToDevice));
  hipStream_t& st = g_order_streams[dev];
  if (!st) HG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  const JobDev* jd = reinterpret_cast<const JobDev*>(e.mem.p);
  launch_prologue(jd, reinterpret_cast<const PrologueSlice*>(e.mem.p + o_pro), 1,
                  pro.setup_blocks, st);
  launch_perm_batch(jd, reinterpret_cast<const JobSlice*>(e.mem.p + o_slice), 1, perm_blocks(od.P),
                    od.h <= 11, st);
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess)
    return set_error(HG_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(le));
  HG_HIP(hipStreamSynchronize(st));
  return HG_OK;
}
}  // namespace

hg_status attach_shared_order(JobSpec* s) {
  if (!job_compressed(*s)) return HG_OK;
  int dev = 0;
  HG_HIP(hipGetDevice(&dev));
  const OrderId id{dev, s->W, s->H, s->ap_q, s->order_key};
  std::lock_guard<std::mutex> lk(g_order_mu);
  auto it = g_orders.find(id);
  if (it == g_orders.end()) {
    auto e = std::make_unique<OrderEntry>();
    const hg_status st = build_order(*e, *s, dev);
    if (st != HG_OK) {
      e->mem.release();
      return st;
    }
    it = g_orders.emplace(id, std::move(e)).first;
  }
  s->shared_tab = it->second->tab;
  s->shared_perm = it->second->perm;
  s->shared_rows = it->second->rows;
  return HG_OK;
}

void release_shared_orders() {
  std::lock_guard<std::mutex> lk(g_order_mu);
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : g_orders) {
    (void)hipSetDevice(kv.second->dev);
    (void)hipDeviceSynchronize();
    kv.second->mem.release();
  }
  g_orders.clear();
  for (auto& kv : g_order_streams) {
    (void)hipSetDevice(kv.first);
    (void)hipStreamDestroy(kv.second);
  }
  g_order_streams.clear();
  if (have_cur) (void)hipSetDevice(cur);
}

PixelSet all_pixels(int32_t M) {
  PixelSet ps;
  ps.perm = nullptr;
  ps.idx = nullptr;
  ps.start = 0;
  ps.count = M;
  ps.M = M;
  return ps;
}

JobLayout layout_job(const JobSpec& s, const TuneParams& tp, int32_t* status_dev,
                     bool raw_inline) {
  JobLayout L;
  JobDev& j = L.dev;
  j = JobDev{};
  j.W = s.W;
  j.H = s.H;
  j.N = s.N;
  j.M = s.W * s.H;
  j.P = s.pupil_n > 0 ? s.pupil_n : j.M;
  j.ap_q = s.ap_q;
  j.ill_a = (float)illumination_exponent(s.pitch_mm, s.waist_mm);
  j.iterations = s.iterations;
  j.compressed = job_compressed(s) ? 1 : 0;
  // the random order runs over the pupil's P pixels
  j.m = j.compressed ? (int32_t)std::ceil(s.compression * (double)j.P) : j.P;
  j.h = j.compressed ? half_bits(j.P) : 0;
  j.seed = s.seed;
  j.order_key = s.order_key;
  j.order_shared = (j.compressed && s.shared_perm) ? 1 : 0;
  j.pitch_mm = s.pitch_mm;
  j.lambda_mm = s.lambda_mm;
  j.focal_mm = s.focal_mm;
  j.phi = s.phi;
  j.lut = s.lut;
  j.lut_levels = s.lut_levels;
  j.gray_bits = s.gray_bits;
  j.gray = s.gray;
  j.trace = s.trace_host ? 1 : 0;
  j.status = status_dev;
  j.mixed = s.precision == HG_PREC_MIXED ? 1 : 0;
  j.shared_e = (!j.mixed && tp.pass_form == 1 && pass_e_width(s.N) > 0) ? 1 : 0;
  L.separable = !j.mixed && tp.separable_full && !s.full_direct;
  L.plan_all = plan_pass(j.M, tp.full_block_cap);
  L.plan_sub = j.compressed ? plan_pass(j.m, tp.subset_block_cap) : L.plan_all;
  L.plan_sep = plan_sep(j.W, j.H);
  L.plan_mx = plan_mx(j.W, j.H);
  // partial-sum rows: one per tile of the largest pass the job can run
  int max_rows = 0, max_groups = 0;
  if (j.mixed || L.separable) {  // operand tables of the matrix-core passes
    static_assert(kSepTileH == kMxTile && kMxTile % kSepTileW == 0,
                  "one table geometry for both full-grid forms");
    j.mx_steps = (s.N + 15) / 16;
    j.mx_cblocks = (s.W + kMxTile - 1) / kMxTile * (kMxTile / 16);
    j.mx_rblocks = (s.H + kMxTile - 1) / kMxTile * (kMxTile / 16);
  }
  int acc_groups = 0;  // groups of the exact-sum passes
  if (j.mixed) {
    // matrix-core passes over the whole grid (compensated FP32 sums), and
    // per-pixel compressed passes (exact sums)
    max_rows = L.plan_mx.tiles;
    max_groups = L.plan_mx.ngroups;
    if (j.compressed) acc_groups = L.plan_sub.ngroups;
  } else {
    // direct full-grid passes: without the separable form, and for the
    // single-pass entry points
    if (!L.separable || s.hook) {
      max_rows = L.plan_all.tiles;
      max_groups = L.plan_all.ngroups;
    }
    if (j.compressed) {
      max_rows = std::max(max_rows, L.plan_sub.tiles);
      max_groups = std::max(max_groups, L.plan_sub.ngroups);
    }
  }
  if (L.separable) {
    max_rows = std::max(max_rows, L.plan_sep.tiles);
    max_groups = std::max(max_groups, L.plan_sep.ngroups);
  }
  if (!j.mixed) acc_groups = max_groups;
  L.grab_offset = (std::max(max_groups, acc_groups) + 1) * kCounterStride;
  L.gen_offset = (L.grab_offset + s.iterations + 2 + kCounterStride - 1) / kCounterStride *
                 kCounterStride;
  j.counters_len = L.gen_offset + kGenCopies * kCounterStride;
  size_t bytes = 0;
  auto take = [&](size_t n) {
    bytes = align_up(bytes, 256);
    const size_t o = bytes;
    bytes += n;
    return o;
  };
  L.raw_inline = raw_inline && !s.spots_on_device;
  L.off_raw = L.raw_inline ? take(sizeof(double) * 4 * (size_t)s.N) : 0;
  L.off_sp = take(sizeof(SpotRec) * (size_t)s.N);
  L.off_sp_alt = take(sizeof(SpotRec) * (size_t)s.N);
  L.off_coef = take(sizeof(float2) * (size_t)s.N);
  const bool own_order = j.compressed && !j.order_shared;
  L.off_tab = own_order ? take(sizeof(uint32_t) * ((size_t)kFeistelRoundsHost << j.h)) : 0;
  L.off_perm = own_order ? take(sizeof(int32_t) * (size_t)j.P) : 0;
  L.off_rows = (own_order && j.ap_q >= 0) ? take(sizeof(int32_t) * (2 * (size_t)j.H + 1)) : 0;
  if (j.mixed) {
    const size_t ops = (size_t)j.mx_steps * 64;  // operand groups per 16-row/column block
    L.off_mxFc = take(16 * ops * j.mx_cblocks);
    L.off_mxFn = take(16 * ops * j.mx_cblocks);
    L.off_mxGa = take(32 * ops * j.mx_rblocks);
    L.off_mxGv = take(32 * ops * j.mx_rblocks);
  }
  if (j.mixed) {  // compensated FP32 sums of the matrix-core passes
    L.off_partial = take(sizeof(float2) * (size_t)max_rows * s.N);
    L.off_gpart = take(sizeof(double2) * (size_t)max_groups * s.N);
  }
  if (!j.mixed || j.compressed) {  // exact fixed-point sums of the per-pixel passes
    j.acc_len = (int64_t)(kAccGroupRow0 + acc_groups) * s.N * kAccSpotWords;
    L.off_acc = take(sizeof(unsigned long long) * (size_t)j.acc_len);
  }
  L.off_counters = take(sizeof(unsigned) * (size_t)j.counters_len);
  L.off_V = take(sizeof(double2) * (size_t)s.N *
                 (s.trace_host && s.iterations > 0 ? s.iterations : 1));
  if (L.separable) {
    const size_t ops = (size_t)j.mx_steps * 64;  // operand lanes per 16-row/column block
    L.off_sepFc = take(sizeof(float) * 8 * ops * j.mx_cblocks);
    L.off_sepFn = take(sizeof(float) * 8 * ops * j.mx_cblocks);
    L.off_sepGa = take(sizeof(float2) * 8 * ops * j.mx_rblocks);
    L.off_sepGv = take(sizeof(float2) * 4 * ops * j.mx_rblocks);
  }
  L.bytes = align_up(bytes, 256);
  return L;
}

JobDev bind_job(const JobLayout& L, const JobSpec& s, char* base, const double* raw_ext) {
  JobDev j = L.dev;
  if (s.spots_on_device) {
    j.in = SpotPtrs{s.x, s.y, s.z, s.amp};
  } else {
    const double* r = L.raw_inline ? reinterpret_cast<const double*>(base + L.off_raw) : raw_ext;
    j.in = SpotPtrs{r, r + s.N, r + 2 * s.N, r + 3 * s.N};
  }
  j.sp = reinterpret_cast<SpotRec*>(base + L.off_sp);
  j.sp_alt = reinterpret_cast<SpotRec*>(base + L.off_sp_alt);
  // jobs of one spot unit per wave run in the one-unit pass launch of each
  // round, whose kernel applies deferred updates
  j.defer_ok = pass_units_per_wave(s.N) == 1 ? 1 : 0;
  j.coef = reinterpret_cast<float2*>(base + L.off_coef);
  if (j.order_shared) {
    j.tab = s.shared_tab;
    j.perm = s.shared_perm;
    j.rows = s.shared_rows;
  } else {
    j.tab = j.compressed ? reinterpret_cast<uint32_t*>(base + L.off_tab) : nullptr;
    j.perm = j.compressed ? reinterpret_cast<int32_t*>(base + L.off_perm) : nullptr;
    j.rows = (j.compressed && j.ap_q >= 0) ? reinterpret_cast<int32_t*>(base + L.off_rows) : nullptr;
  }
  j.partial = j.mixed ? reinterpret_cast<float2*>(base + L.off_partial) : nullptr;
  j.gpart = j.mixed ? reinterpret_cast<double2*>(base + L.off_gpart) : nullptr;
  j.acc = (!j.mixed || j.compressed) ? reinterpret_cast<unsigned long long*>(base + L.off_acc)
                                      : nullptr;
  j.counters = reinterpret_cast<unsigned*>(base + L.off_counters);
  j.grab = j.counters + L.grab_offset;
  j.gen = j.counters + L.gen_offset;
  j.V = reinterpret_cast<double2*>(base + L.off_V);
  if (L.separable) {
    j.sepFc = reinterpret_cast<float*>(base + L.off_sepFc);
    j.sepFn = reinterpret_cast<float*>(base + L.off_sepFn);
    j.sepGa = reinterpret_cast<float2*>(base + L.off_sepGa);
    j.sepGv = reinterpret_cast<float4*>(base + L.off_sepGv);
  }
  if (j.mixed) {
    j.mxFc = reinterpret_cast<uint4*>(base + L.off_mxFc);
    j.mxFn = reinterpret_cast<uint4*>(base + L.off_mxFn);
    j.mxGa = reinterpret_cast<float4*>(base + L.off_mxGa);
    j.mxGv = reinterpret_cast<float4*>(base + L.off_mxGv);
  }
  return j;
}

namespace {
// Deferred updates.  Pass it of job j (1..I; I + 1 is the final hologram)
// can apply the previous pass's update at its start, and so let that pass
// stop after its sums: the per-pixel compressed passes of one spot unit per
// wave (FP32 or mixed), the FP32 separable full-grid passes and final
// hologram, and the mixed full-grid pass and final hologram of a CS-WGS
// job, for N <= kPendMaxSpots.
bool pend_capable(const JobDev& j, const JobLayout& L, int it) {
  if (j.N > kPendMaxSpots || !j.sp_alt) return false;
  if (j.compressed && it < j.iterations) return j.defer_ok && !j.shared_e;
  // mixed CS-WGS: the full-grid pass and the final hologram (the exact sums
  // of a mixed job are kept only with compressed passes)
  if (j.mixed) return j.compressed && (it == j.iterations || (it > j.iterations && j.phi));
  if (!L.separable) return false;
  return it <= j.iterations || j.phi != nullptr;
}
bool defers(const JobDev& j, const JobLayout& L, int it) {
  return it <= j.iterations && pend_capable(j, L, it) && pend_capable(j, L, it + 1);
}
// 2^-shift / count of pass it's sums, as its tail would scale them
double pass_inv(const JobDev& j, const JobLayout& L, int it) {
  const bool sub = j.compressed && it < j.iterations;
  const int shift = sub ? L.plan_sub.shift : j.mixed ? L.plan_mx.shift : L.plan_sep.shift;
  return std::ldexp(1.0, -shift) * (1.0 / (double)(sub ? j.m : j.P));
}
// A pending pass it reads the state X_{it-2} that the previous pass used
// and, when it defers in turn (or is the final hologram), stores X_{it-1},
// which it formed, for the next.  In a run of pending passes s, s+1, ...
// (pass s-1 defers without being pending, so X_{s-2} is in the spot records
// sp, where the setup or a pass's own update left it) pass it reads buffer
// (it - s) mod 2 and writes the other (0: sp, 1: sp_alt).
template <typename D>
void plan_deferral(D& d, const JobDev& j, const JobLayout& L, int it) {
  const bool df = defers(j, L, it), pd = it >= 2 && defers(j, L, it - 1);
  if (!df && !pd) return;
  SpotRec* const buf[2] = {j.sp, j.sp_alt};
  d.tot_row = it % kAccTotalRows;
  d.defer = df ? 1 : 0;
  if (pd) {
    int s = it;  // the first pending pass of this run
    while (s - 1 >= 2 && defers(j, L, s - 2)) --s;
    d.pending = 1;
    d.prev_row = (it - 1) % kAccTotalRows;
    d.clear_row = (it + 1) % kAccTotalRows;
    d.prev_inv = pass_inv(j, L, it - 1);
    d.st_in = buf[(it - s) % 2];
    d.st_out = (df || it > j.iterations) ? buf[(it - s + 1) % 2] : nullptr;
    d.prev_V = j.trace ? j.V + (size_t)(it - 2) * j.N : nullptr;
  }
}
template <typename D>
void clear_deferral(D& d) {
  d.defer = d.pending = d.tot_row = d.prev_row = 0;
  d.clear_row = -1;
  d.prev_inv = 0.0;
  d.st_in = nullptr;
  d.st_out = nullptr;
  d.prev_V = nullptr;
}
}  // namespace

PassDesc iteration_desc(const JobDev& j, const JobLayout& L, int it, int index, int block_begin) {
  const bool sub = j.compressed && it < j.iterations;
  PassDesc d;
  d.block_begin = block_begin;
  d.job = index;
  d.ps = all_pixels(j.M);  // the whole grid: the pupil weights drop the pixels outside it
  if (sub) {
    d.ps.perm = j.perm;
    d.ps.start = (int64_t)(it - 1) * j.m % j.P;
    d.ps.count = j.m;
    d.ps.M = j.P;
  }
  d.plan = sub ? L.plan_sub : L.plan_all;
  d.update = 1;
  d.from_phi = 0;
  d.grab_slot = it;
  d.inv_count = 1.0 / (double)(sub ? j.m : j.P);  // eq. (3): the mean over the set
  d.V = j.V + (j.trace ? (size_t)(it - 1) * j.N : 0);
  // Deferred updates: consecutive compressed passes, and the last of them
  // with the separable full-grid pass and the final hologram after it
  if (sub) plan_deferral(d, j, L, it);
  return d;
}

// ------------------------------------------------------------- launch sets --

namespace {
SepDesc sep_desc(const JobDev& j, const JobLayout& L, int index, int block_begin) {
  SepDesc d;
  d.block_begin = block_begin;
  d.job = index;
  d.tiles_x = (j.W + kSepTileW - 1) / kSepTileW;
  d.tiles_y = (j.H + kSepTileH - 1) / kSepTileH;
  d.plan = L.plan_sep;
  d.update = 0;
  d.inv_count = 1.0 / (double)j.P;
  d.V = j.V;
  d.out = nullptr;
  return d;
}
}  // namespace

namespace {
MxDesc mx_desc(const JobDev& j, const JobLayout& L, int index, int block_begin) {
  MxDesc d;
  d.block_begin = block_begin;
  d.job = index;
  d.tiles_x = (j.W + kMxTileW - 1) / kMxTileW;
  d.tiles_y = (j.H + kMxTile - 1) / kMxTile;
  d.plan = L.plan_mx;
  d.update = 0;
  d.inv_count = 1.0f / (float)j.P;
  d.V = j.V;
  d.out = nullptr;
  return d;
}
}  // namespace

void LaunchSet::add_forward_mx(const JobDev& j, const JobLayout& L, int index) {
  mx.push_back(mx_desc(j, L, index, mx_blocks));
  mx_blocks += L.plan_mx.blocks;
  mx_steps = std::max(mx_steps, j.mx_steps);
  mx_mode = kMxFromPhi;
}

void LaunchSet::add_iteration(const JobDev& j, const JobLayout& L, int it, int index) {
  const bool sub = j.compressed && it < j.iterations;
  if (j.mixed && sub) {  // per-pixel compressed pass, FP16 back-propagation
    const int u = pass_units_per_wave(j.N);
    const PassDesc d = iteration_desc(j, L, it, index, u > 1 ? mxw_blocks : mxp_blocks);
    if (u > 1) {
      mxw.push_back(d);
      mxw_blocks += d.plan.blocks;
      mxw_units = std::max(mxw_units, u);
    } else {
      mxp.push_back(d);
      mxp_blocks += d.plan.blocks;
    }
    return;
  }
  if (j.mixed) {
    MxDesc d = mx_desc(j, L, index, mx_blocks);
    mx_full += 1;
    d.update = 1;
    d.V = j.V + (j.trace ? (size_t)(it - 1) * j.N : 0);
    plan_deferral(d, j, L, it);
    mx.push_back(d);
    mx_blocks += d.plan.blocks;
    mx_steps = std::max(mx_steps, j.mx_steps);
    return;
  }
  if (!sub && L.separable) {
    SepDesc d = sep_desc(j, L, index, sep_blocks);
    d.update = 1;
    d.V = j.V + (j.trace ? (size_t)(it - 1) * j.N : 0);
    plan_deferral(d, j, L, it);
    sep.push_back(d);
    sep_blocks += d.plan.blocks;
    sep_steps = std::max(sep_steps, j.mx_steps);
    return;
  }
  const int u = j.shared_e ? 1 : pass_units_per_wave(j.N);
  if (u > 1) {
    const PassDesc d = iteration_desc(j, L, it, index, wide_blocks);
    wide.push_back(d);
    wide_blocks += d.plan.blocks;
    wide_units = std::max(wide_units, u);
    return;
  }
  const PassDesc d = iteration_desc(j, L, it, index, pass_blocks);
  pass.push_back(d);
  pass_blocks += d.plan.blocks;
  if (j.shared_e) e_width = std::max(e_width, pass_e_width(j.N));
}

void LaunchSet::add_final(const JobDev& j, const JobLayout& L, int index) {
  if (j.mixed) {
    MxDesc d = mx_desc(j, L, index, mx_blocks);
    d.out = j.phi;
    plan_deferral(d, j, L, j.iterations + 1);
    mx.push_back(d);
    mx_blocks += d.plan.blocks;
    mx_steps = std::max(mx_steps, j.mx_steps);
    mx_mode = kMxFinal;
    return;
  }
  if (L.separable) {
    SepDesc d = sep_desc(j, L, index, sep_blocks);
    d.out = j.phi;
    plan_deferral(d, j, L, j.iterations + 1);
    sep.push_back(d);
    sep_blocks += d.plan.blocks;
    sep_steps = std::max(sep_steps, j.mx_steps);
    sep_final = true;
    return;
  }
  BackDesc b;
  b.block_begin = back_blocks;
  b.job = index;
  b.ps = all_pixels(j.M);
  b.out = j.phi;
  back.push_back(b);
  back_blocks += backprop_blocks(j.M);
}

size_t LaunchSet::bytes() const {
  return align_up(sizeof(PassDesc) * pass.size(), 256) + align_up(sizeof(PassDesc) * wide.size(), 256) +
         align_up(sizeof(SepDesc) * sep.size(), 256) +
         align_up(sizeof(BackDesc) * back.size(), 256) + align_up(sizeof(MxDesc) * mx.size(), 256) +
         align_up(sizeof(PassDesc) * mxp.size(), 256) + align_up(sizeof(PassDesc) * mxw.size(), 256);
}

size_t LaunchSet::stage(char* host, char* dev) {
  size_t o = 0;
  auto put = [&](const void* src, size_t n) {
    const size_t at = o;
    if (n) std::memcpy(host + at, src, n);
    o = align_up(o + n, 256);
    return dev + at;
  };
  d_pass = reinterpret_cast<const PassDesc*>(put(pass.data(), sizeof(PassDesc) * pass.size()));
  d_wide = reinterpret_cast<const PassDesc*>(put(wide.data(), sizeof(PassDesc) * wide.size()));
  d_sep = reinterpret_cast<const SepDesc*>(put(sep.data(), sizeof(SepDesc) * sep.size()));
  d_back = reinterpret_cast<const BackDesc*>(put(back.data(), sizeof(BackDesc) * back.size()));
  d_mx = reinterpret_cast<const MxDesc*>(put(mx.data(), sizeof(MxDesc) * mx.size()));
  d_mxp = reinterpret_cast<const PassDesc*>(put(mxp.data(), sizeof(PassDesc) * mxp.size()));
  d_mxw = reinterpret_cast<const PassDesc*>(put(mxw.data(), sizeof(PassDesc) * mxw.size()));
  return o;
}

namespace {
const char* pass_name(const std::vector<PassDesc>& a, const std::vector<PassDesc>& b) {
  bool any_full = false, any_sub = false;
  for (const auto* v : {&a, &b})
    for (const PassDesc& d : *v) (d.ps.count == d.ps.M && !d.ps.perm ? any_full : any_sub) = true;
  return any_full && any_sub ? "k_pass_mixed" : any_sub ? "k_pass_subset" : "k_pass_full";
}
}  // namespace

const char* LaunchSet::pass_only_name() const {
  const bool fp32 = !pass.empty() || !wide.empty(), mixed = !mxp.empty() || !mxw.empty();
  if (fp32 == mixed || !sep.empty() || !back.empty() || !mx.empty()) return nullptr;
  return fp32 ? pass_name(pass, wide) : "k_mxp_subset";
}

void LaunchSet::launch(const JobDev* jobs, hipStream_t s, bool capture) const {
  auto run = [&](const char* name, auto&& f) {
    if (capture) f();
    else timed(s, name, f);
  };
  if (!sep.empty())
    run(sep_final ? "k_sep_final" : "k_sep_pass", [&] {
      launch_sep_pass(jobs, d_sep, (int)sep.size(), sep_blocks, sep_final, sep_steps, s);
    });
  if (!pass.empty())
    run(pass_name(pass, {}),
        [&] { launch_pass_batch(jobs, d_pass, (int)pass.size(), pass_blocks, 1, e_width, s); });
  if (!wide.empty())
    run(pass_name(wide, {}), [&] {
      launch_pass_batch(jobs, d_wide, (int)wide.size(), wide_blocks, wide_units, 0, s);
    });
  if (!back.empty())
    run("k_backprop_phi",
        [&] { launch_backprop_batch(jobs, d_back, (int)back.size(), back_blocks, s); });
  if (!mxp.empty())
    run("k_mxp_subset", [&] { launch_pass_mx(jobs, d_mxp, (int)mxp.size(), mxp_blocks, 1, s); });
  if (!mxw.empty())
    run("k_mxp_subset",
        [&] { launch_pass_mx(jobs, d_mxw, (int)mxw.size(), mxw_blocks, mxw_units, s); });
  if (!mx.empty()) {
    const char* name = "k_mx_forward";
    if (mx_mode == kMxFinal) name = "k_mx_final";
    else if (mx_mode == kMxIterate) name = "k_mx_full";
    run(name, [&] { launch_mx_pass(jobs, d_mx, (int)mx.size(), mx_blocks, mx_mode, mx_steps, s); });
  }
}

// ------------------------------------------------------------------- batch --

hg_status Batch::build(const JobSpec* specs, int count, const TuneParams& tp,
                       int32_t* status_dev, bool allow_chain) {
  specs_.assign(specs, specs + count);
  jobs_.assign(count, JobDev{});
  layouts_.resize(count);
  std::vector<size_t> raw_off(count, 0), base_off(count, 0);
  // host-resident spot inputs first, contiguous, so that one copy moves them
  host_spot_bytes_ = 0;
  for (int i = 0; i < count; ++i)
    if (!specs[i].spots_on_device) {
      raw_off[i] = host_spot_bytes_;
      host_spot_bytes_ += sizeof(double) * 4 * (size_t)specs[i].N;
    }
  size_t bytes = align_up(host_spot_bytes_, 256);
  int max_rounds = 0;
  perm_lds_ = true;
  for (int i = 0; i < count; ++i) {
    layouts_[i] = layout_job(specs[i], tp, status_dev, false);
    base_off[i] = bytes;
    bytes += layouts_[i].bytes;
    max_rounds = std::max(max_rounds, specs[i].iterations);
    const JobDev& j = layouts_[i].dev;
    if (j.compressed && !j.order_shared) {
      if (j.h > 11) perm_lds_ = false;
    }
  }
  raw_base_ = 0;
  HG_TRY(arena_.reserve(std::max<size_t>(bytes, 256)));
  for (int i = 0; i < count; ++i)
    jobs_[i] = bind_job(layouts_[i], specs[i], arena_.p + base_off[i],
                        reinterpret_cast<const double*>(arena_.p + raw_off[i]));
  // iteration rounds: round r runs iteration r + 1 of every job with I > r
  rounds_.assign(max_rounds, LaunchSet{});
  for (int r = 0; r < max_rounds; ++r)
    for (int i = 0; i < count; ++i)
      if (r < jobs_[i].iterations) rounds_[r].add_iteration(jobs_[i], layouts_[i], r + 1, i);
  final_ = LaunchSet{};
  perm_.clear();
  perm_blocks_ = 0;
  pro_.clear();
  pro_blocks_ = 0;
  for (int i = 0; i < count; ++i) {
    const JobDev& j = jobs_[i];
    if (j.phi) final_.add_final(j, layouts_[i], i);
    if (j.compressed && !j.order_shared) {
      perm_.push_back(JobSlice{perm_blocks_, i});
      perm_blocks_ += perm_blocks(j.P);
    }
    const PrologueSlice ps{pro_blocks_, i, prologue_setup_blocks(j), prologue_table_blocks(j)};
    pro_.push_back(ps);
    pro_blocks_ += ps.setup_blocks + ps.table_blocks;
  }
  // chained launch of a single FP32 job's compressed passes
  chain_descs_.clear();
  chain_rounds_ = 0;
  if (allow_chain && tp.chain_passes && count == 1) {
    const JobDev& j = jobs_[0];
    const int passes = j.iterations - 1;  // iterations 1..I-1 are compressed
    const int units = pass_units_per_wave(j.N);
    if (j.compressed && !j.mixed && !j.shared_e && j.N <= kChainMaxSpots && passes >= 2 &&
        layouts_[0].plan_sub.blocks <= pass_chain_capacity(units)) {
      for (int r = 0; r < passes; ++r) {
        // a chained launch hands the state over inside the launch
        PassDesc d = rounds_[r].pass.at(0);
        clear_deferral(d);
        chain_descs_.push_back(d);
      }
      // and the passes after it update in their own tails (the chain's
      // last pass leaves the state in the spot records); so does the last
      // compressed pass of the one-launch-per-pass form that stands in when
      // the cooperative launch is refused
      if ((size_t)passes < rounds_.size())
        for (SepDesc& d : rounds_[passes].sep) clear_deferral(d);
      for (SepDesc& d : final_.sep) clear_deferral(d);
      for (PassDesc& d : rounds_[passes - 1].pass) {
        d.defer = 0;
        d.st_out = nullptr;
      }
      chain_rounds_ = passes;
      chain_blocks_ = layouts_[0].plan_sub.blocks;
      chain_units_ = units;
    }
  }
  // descriptor tables: [JobDev][JobSlice perm][PrologueSlice][chain passes]
  // [rounds...][final]
  size_t tb = align_up(sizeof(JobDev) * count, 256);
  const size_t t_perm = tb;
  tb = align_up(tb + sizeof(JobSlice) * perm_.size(), 256);
  const size_t t_pro = tb;
  tb = align_up(tb + sizeof(PrologueSlice) * pro_.size(), 256);
  const size_t t_chain = tb;
  tb = align_up(tb + sizeof(PassDesc) * chain_descs_.size(), 256);
  const size_t t_sets = tb;
  for (const LaunchSet& ls : rounds_) tb += ls.bytes();
  tb += final_.bytes();
  table_bytes_ = tb;
  HG_TRY(table_.reserve(std::max<size_t>(tb, 256)));
  HG_TRY(staging_.acquire(tb + host_spot_bytes_));
  std::memset(staging_.p, 0, tb);
  jobs_dev_ = reinterpret_cast<JobDev*>(table_.p);
  perm_dev_ = reinterpret_cast<JobSlice*>(table_.p + t_perm);
  std::memcpy(staging_.p, jobs_.data(), sizeof(JobDev) * count);
  if (!perm_.empty()) std::memcpy(staging_.p + t_perm, perm_.data(), sizeof(JobSlice) * perm_.size());
  pro_dev_ = reinterpret_cast<PrologueSlice*>(table_.p + t_pro);
  std::memcpy(staging_.p + t_pro, pro_.data(), sizeof(PrologueSlice) * pro_.size());
  chain_dev_ = reinterpret_cast<PassDesc*>(table_.p + t_chain);
  if (!chain_descs_.empty())
    std::memcpy(staging_.p + t_chain, chain_descs_.data(), sizeof(PassDesc) * chain_descs_.size());
  size_t o = t_sets;
  for (LaunchSet& ls : rounds_) o += ls.stage(staging_.p + o, table_.p + o);
  o += final_.stage(staging_.p + o, table_.p + o);
  for (int i = 0; i < count; ++i) {
    const JobSpec& s = specs[i];
    if (s.spots_on_device) continue;
    double* dst = reinterpret_cast<double*>(staging_.p + tb + raw_off[i]);
    std::memcpy(dst, s.x, sizeof(double) * s.N);
    std::memcpy(dst + s.N, s.y, sizeof(double) * s.N);
    std::memcpy(dst + 2 * s.N, s.z, sizeof(double) * s.N);
    std::memcpy(dst + 3 * s.N, s.amp, sizeof(double) * s.N);
  }
  return HG_OK;
}

hg_status Batch::enqueue_prologue(hipStream_t s, bool capture) {
  HG_HIP(hipMemcpyAsync(table_.p, staging_.p, table_bytes_, hipMemcpyHostToDevice, s));
  if (host_spot_bytes_)
    HG_HIP(hipMemcpyAsync(arena_.p + raw_base_, staging_.p + table_bytes_, host_spot_bytes_,
                          hipMemcpyHostToDevice, s));
  if (!capture) HG_TRY(staging_.mark_copied(s));
  const bool quiet = capture || untimed_;
  auto run = [&](const char* name, auto&& launch) {
    if (quiet) launch();
    else timed(s, name, launch);
  };
  run("k_prologue",
      [&] { launch_prologue(jobs_dev_, pro_dev_, (int)pro_.size(), pro_blocks_, s); });
  if (perm_blocks_ > 0)
    run("k_perm", [&] {
      launch_perm_batch(jobs_dev_, perm_dev_, (int)perm_.size(), perm_blocks_, perm_lds_, s);
    });
  return HG_OK;
}

hg_status Batch::enqueue(hipStream_t s, bool capture) {
  HG_TRY(enqueue_prologue(s, capture));
  size_t r0 = 0;
  const bool quiet = capture || untimed_;
  if (chain_rounds_ > 0 && !capture) {
    hipError_t ce = hipSuccess;
    auto chain = [&] {
      ce = launch_pass_chain(jobs_dev_, chain_dev_, chain_rounds_, chain_blocks_, chain_units_, s);
    };
    if (quiet) chain();
    else timed(s, "k_pass_chain", chain);
    if (ce == hipSuccess) r0 = (size_t)chain_rounds_;
    else (void)hipGetLastError();  // not launched: one launch per pass instead
  }
  // Runs of rounds that launch the same per-pixel pass kernel and nothing
  // else are timed as one group (two events around the run), so that the
  // average per launch is that of back-to-back launches.
  size_t r = r0;
  while (r < rounds_.size()) {
    const char* kind = rounds_[r].pass_only_name();
    if (quiet || !timing_enabled() || !kind) {
      rounds_[r].launch(jobs_dev_, s, quiet);
      ++r;
      continue;
    }
    size_t r1 = r;
    while (r1 < rounds_.size() && rounds_[r1].pass_only_name() &&
           std::strcmp(rounds_[r1].pass_only_name(), kind) == 0)
      ++r1;
    hipEvent_t a = timing_start(s);
    for (size_t k = r; k < r1; ++k) rounds_[k].launch(jobs_dev_, s, /*capture=*/true);
    timing_stop(s, kind, a, (int)(r1 - r));
    r = r1;
  }
  final_.launch(jobs_dev_, s, quiet);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return set_error(HG_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return HG_OK;
}

hg_status Batch::fetch_traces(hipStream_t s) {
  bool any = false;
  for (size_t i = 0; i < specs_.size(); ++i) {
    const JobSpec& sp = specs_[i];
    if (!sp.trace_host || sp.iterations <= 0) continue;
    HG_HIP(hipMemcpyAsync(sp.trace_host, jobs_[i].V,
                          sizeof(double2) * (size_t)sp.N * sp.iterations, hipMemcpyDeviceToHost,
                          s));
    any = true;
  }
  if (any) HG_HIP(hipStreamSynchronize(s));
  return HG_OK;
}

hg_status Batch::upload_custom(const void* bytes, size_t size, hipStream_t s, void** dev) {
  HG_TRY(custom_staging_.acquire(size));
  std::memcpy(custom_staging_.p, bytes, size);
  HG_TRY(custom_.reserve(size));
  HG_HIP(hipMemcpyAsync(custom_.p, custom_staging_.p, size, hipMemcpyHostToDevice, s));
  HG_TRY(custom_staging_.mark_copied(s));
  *dev = custom_.p;
  return HG_OK;
}

hg_status Batch::custom_device(size_t size, char** dev) {
  HG_TRY(custom_.reserve(std::max<size_t>(size, 256)));
  *dev = custom_.p;
  return HG_OK;
}

void Batch::adopt(char* arena, size_t arena_bytes, char* table, size_t table_bytes, char* host,
                  size_t host_bytes, hipEvent_t copied) {
  release();
  arena_.adopt(arena, arena_bytes);
  table_.adopt(table, table_bytes);
  staging_.adopt(host, host_bytes, copied);
  untimed_ = true;
}

void Batch::release() {
  untimed_ = false;
  staging_.release();
  custom_staging_.release();
  arena_.release();
  table_.release();
  custom_.release();
  jobs_dev_ = nullptr;
  perm_dev_ = nullptr;
  pro_dev_ = nullptr;
  chain_dev_ = nullptr;
}

}  // namespace hg
