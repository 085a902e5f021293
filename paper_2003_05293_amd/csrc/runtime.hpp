// Host runtime of libhg: device buffers, batch planning and the RS / WGS /
// CS-WGS schedules (paper section 2) enqueued as batched launches.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hg.h"
#include "kernels.hpp"

// A phase-to-gray table of the SLM resident on one device (hg_lut_create).
struct hg_lut {
  uint16_t* dev = nullptr;  // [levels]
  int32_t levels = 0;
  int32_t bits = 0;         // 8 or 16: element type of the gray images
  int device = 0;
};

namespace hg {

// Thread-local error message of the C ABI.
hg_status set_error(hg_status st, const std::string& msg);
const char* last_error();

#define HG_HIP(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::hg::set_error(e_ == hipErrorOutOfMemory ? HG_ENOMEM : HG_EDEVICE,     \
                             std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

#define HG_TRY(expr)              \
  do {                            \
    hg_status st_ = (expr);       \
    if (st_ != HG_OK) return st_; \
  } while (0)

// Device buffer that grows on demand and is never shrunk.  Growing waits for
// the device first: queued kernels may still be reading the old buffer.
// An adopted buffer is memory the library does not own (a fixed region of
// static device memory): it never grows, and a request beyond it fails with
// HG_ENOMEM instead of allocating.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t cap = 0;
  bool adopted = false;
  hg_status reserve(size_t n) {
    if (n <= cap) return HG_OK;
    if (adopted)
      return set_error(HG_ENOMEM, "the request needs " + std::to_string(n * sizeof(T)) +
                                      " bytes of static scratch in one region, which holds " +
                                      std::to_string(cap * sizeof(T)));
    if (p) HG_HIP(hipDeviceSynchronize());
    release();
    HG_HIP(hipMalloc((void**)&p, n * sizeof(T)));
    cap = n;
    return HG_OK;
  }
  void adopt(T* q, size_t n) {
    p = q;
    cap = n;
    adopted = true;
  }
  void release() {
    if (p && !adopted) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    adopted = false;
  }
};

// Host staging area whose refill waits for the copy that last read it:
// pinned memory that grows on demand, or an adopted fixed host region with
// its event (which then never grows).
struct Staging {
  char* p = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  bool adopted = false;
  hg_status acquire(size_t bytes);             // waits for the previous copy, grows
  hg_status mark_copied(hipStream_t s);        // records the event after the copies
  void adopt(char* q, size_t n, hipEvent_t ev);
  void release();
};

// Host description of one hologram.
struct JobSpec {
  int32_t W = 0, H = 0;
  double pitch_mm = 0, lambda_mm = 0, focal_mm = 0;
  double waist_mm = 0;      // illumination waist (0: uniform)
  int32_t ap_q = -1;        // aperture bound on Lx^2 + Ly^2 (-1: none)
  int32_t pupil_n = 0;      // pixels of the pupil (W*H without an aperture)
  int32_t N = 0;
  const double *x = nullptr, *y = nullptr, *z = nullptr, *amp = nullptr;
  bool spots_on_device = false;
  int32_t iterations = 0;
  double compression = -1.0;  // <= 0: plain WGS (no random order)
  uint64_t seed = 0;                  // theta^0
  uint64_t order_key = HG_ORDER_KEY;  // the random order (compressed jobs)
  // the random order shared by every hologram of this grid and pupil on
  // the device (attach_shared_order); null: the job builds its own
  int32_t* shared_perm = nullptr;
  uint32_t* shared_tab = nullptr;
  int32_t* shared_rows = nullptr;
  uint32_t precision = HG_PREC_FP32;
  bool full_direct = false;   // full-grid passes with the per-pixel kernels
  bool hook = false;          // single-pass entry point (any pixel set up to W*H)
  float* phi = nullptr;       // output hologram (device)
  double* trace_host = nullptr;
  // SLM output: the final pass also writes the gray image (device)
  const uint16_t* lut = nullptr;
  int32_t lut_levels = 0;
  int32_t gray_bits = 0;
  void* gray = nullptr;
};

// The random pixel order of a compressed job's grid, pupil and order key,
// shared by every hologram that has them on the current device: built on
// first use (the call blocks until it is complete) and kept until
// release_shared_orders.  Leaves jobs without a random order unchanged.
hg_status attach_shared_order(JobSpec* s);
void release_shared_orders();

// Launch-geometry parameters (chosen per shape by the autotuner).
struct TuneParams {
  int32_t full_block_cap = kDefaultBlockCap;
  int32_t subset_block_cap = kDefaultBlockCap;
  bool separable_full = true;  // full-grid passes as separable products
  int32_t pass_form = 0;       // 1: shared-exponential compressed passes where N allows
  bool chain_passes = false;   // chained launch of a single job's compressed passes
};

// Pupil of an hg_optics (validated): the aperture bound q = floor(D^2)
// (-1 without an aperture), the pupil's pixel count, the FP64 illumination
// exponent pitch^2 / (4 w^2) per unit of Q (0 without a waist), and the
// power mean_Omega(A^2) (1 without a waist).
int32_t aperture_bound(const hg_optics* o);
int64_t pupil_count(int32_t W, int32_t H, int32_t q);
double illumination_exponent(double pitch_mm, double waist_mm);
double pupil_power(int32_t W, int32_t H, int32_t q, double ill_a);

// SLM output of a hologram: the table and the gray image (both or neither).
hg_status apply_lut(const hg_lut* lut, void* gray, JobSpec* spec);

// Validation of the host-visible parts of a hologram description.
hg_status validate_grid(const hg_grid* g);
hg_status validate_spec(const hg_grid* g, const hg_optics* o, const hg_spots* s, bool on_device);
hg_status make_spec(const hg_grid* g, const hg_optics* o, const hg_spots* s, int32_t iterations,
                    double compression, uint64_t seed, uint32_t flags, float* phi,
                    double* trace_host, JobSpec* out);

// Device scratch of one job, laid out relative to the job's base address.
struct JobLayout {
  JobDev dev;  // every field but the pointers
  PassPlan plan_all, plan_sub, plan_sep, plan_mx;
  bool separable = false;
  size_t off_raw = 0, off_sp = 0, off_sp_alt = 0, off_coef = 0, off_tab = 0, off_perm = 0, off_partial = 0,
         off_gpart = 0, off_acc = 0, off_counters = 0, off_V = 0, off_sepFc = 0, off_sepFn = 0,
         off_sepGa = 0, off_sepGv = 0, off_mxFc = 0, off_mxFn = 0, off_mxGa = 0, off_mxGv = 0,
         off_rows = 0;
  size_t bytes = 0;
  bool raw_inline = false;  // the job's own scratch holds a copy of its spot arrays
  int grab_offset = 0;      // the pass tile counters follow the group counters
  int gen_offset = 0;       // then the generation words of chained launches
};
// raw_inline: reserve room for the 4N input doubles of host-resident spots.
JobLayout layout_job(const JobSpec& s, const TuneParams& tp, int32_t* status_dev,
                     bool raw_inline);
// The JobDev of a job whose scratch starts at `base` (host spot copies at
// raw_ext when the layout does not hold them itself).
JobDev bind_job(const JobLayout& L, const JobSpec& s, char* base, const double* raw_ext);
// Descriptor of iteration `it` (1-based) of job `index` in a launch.
PassDesc iteration_desc(const JobDev& j, const JobLayout& L, int it, int index, int block_begin);
PixelSet all_pixels(int32_t M);

// The launches of one iteration round (or of the final phase) of a set of
// jobs: compressed passes (k_pass_batch), separable full-grid passes
// (k_sep_pass, on the factor tables built by the prologue), direct full-grid final phases (k_backprop_batch) and the
// passes of mixed-precision jobs (k_mx_pass).
struct LaunchSet {
  // per-pixel passes in two launches: jobs of one spot unit per wave (and
  // the shared-exponential form) in `pass`, wider jobs in `wide`, so that
  // every job runs in the same kernel form alone and in any batch
  std::vector<PassDesc> pass;
  int pass_blocks = 0;
  int e_width = 0;  // widest shared-exponential form among the passes (0: none)
  std::vector<PassDesc> wide;
  int wide_blocks = 0, wide_units = 1;
  std::vector<SepDesc> sep;
  int sep_blocks = 0, sep_steps = 0;
  bool sep_final = false;
  std::vector<BackDesc> back;
  int back_blocks = 0;
  std::vector<MxDesc> mx;
  int mx_blocks = 0, mx_steps = 0, mx_full = 0;
  int mx_mode = kMxIterate;
  // compressed passes of mixed-precision jobs (per-pixel, FP16
  // back-propagation): one unit per wave in mxp, wider jobs in mxw
  std::vector<PassDesc> mxp;
  int mxp_blocks = 0;
  std::vector<PassDesc> mxw;
  int mxw_blocks = 0, mxw_units = 1;
  // device copies, set by stage()
  const PassDesc* d_pass = nullptr;
  const PassDesc* d_wide = nullptr;
  const SepDesc* d_sep = nullptr;
  const BackDesc* d_back = nullptr;
  const MxDesc* d_mx = nullptr;
  const PassDesc* d_mxp = nullptr;
  const PassDesc* d_mxw = nullptr;

  void add_iteration(const JobDev& j, const JobLayout& L, int it, int index);
  void add_final(const JobDev& j, const JobLayout& L, int index);
  // Forward projection of the job's stored hologram (mixed precision, all
  // pixels, no update).
  void add_forward_mx(const JobDev& j, const JobLayout& L, int index);
  bool empty() const {
    return pass.empty() && wide.empty() && sep.empty() && back.empty() && mx.empty() &&
           mxp.empty() && mxw.empty();
  }
  // Timing name of the set's per-pixel pass launch when that is all the set
  // launches, else nullptr.
  const char* pass_only_name() const;
  size_t bytes() const;
  // Copies the descriptors into host staging at `host` and points the
  // device copies at `dev` (same offsets); returns the bytes used.
  size_t stage(char* host, char* dev);
  // Launches the set's kernels.  `capture`: no timing.
  void launch(const JobDev* jobs, hipStream_t s, bool capture) const;
};

// Kernel timing (hg_timing_*).  While enabled, `timed` brackets a launch
// with two events recorded on its stream; hg_timing_read drains them.
bool timing_enabled();
void timing_enable(bool on);
hipEvent_t timing_start(hipStream_t s);
void timing_stop(hipStream_t s, const char* name, hipEvent_t start, int count = 1);
hg_status timing_reset();
hg_status timing_read(const char* name, double* total_ms, int64_t* launches);

template <typename F>
void timed(hipStream_t s, const char* name, F&& launch) {
  if (!timing_enabled()) {
    launch();
    return;
  }
  hipEvent_t a = timing_start(s);
  launch();
  timing_stop(s, name, a);
}

// A batch of holograms planned for one launch sequence.  Plans, device
// scratch and the descriptor tables are kept and reused by later builds.
class Batch {
 public:
  // Plans the jobs and lays out their scratch; allocates as needed.
  // allow_chain: a single FP32 job may run its compressed passes as one
  // chained launch (not for schedules captured into a graph).
  hg_status build(const JobSpec* specs, int count, const TuneParams& tp, int32_t* status_dev,
                  bool allow_chain = false);
  // Uploads the tables (and host spot arrays), then the whole schedule:
  // setup, random orders, one pass launch per iteration round, final phase.
  // With `capture`, the enqueue is being recorded into a graph: no event is
  // recorded and no launch is timed.
  hg_status enqueue(hipStream_t s, bool capture = false);
  // Setup and random orders only (for the single-step calls).
  hg_status enqueue_prologue(hipStream_t s, bool capture = false);
  // Copies the traces of the jobs that asked for one and waits for them.
  hg_status fetch_traces(hipStream_t s);

  int count() const { return (int)specs_.size(); }
  const JobDev& job(int i) const { return jobs_[i]; }
  const JobLayout& layout(int i) const { return layouts_[i]; }
  const JobDev* jobs_device() const { return jobs_dev_; }
  // A descriptor area on the device for ad-hoc single launches.
  hg_status upload_custom(const void* bytes, size_t size, hipStream_t s, void** dev);
  // Reserves the custom area and returns its device address.
  hg_status custom_device(size_t size, char** dev);
  // Makes the batch work in fixed memory that it does not own: job scratch
  // in [arena, arena + arena_bytes), descriptor tables in [table, table +
  // table_bytes) on the device, their host staging in [host, host +
  // host_bytes) guarded by `copied`.  Later builds allocate nothing (a
  // schedule that does not fit fails with HG_ENOMEM) and launches are
  // never timed.  Not for batches that use upload_custom.
  void adopt(char* arena, size_t arena_bytes, char* table, size_t table_bytes, char* host,
             size_t host_bytes, hipEvent_t copied);
  void release();

 private:
  std::vector<JobSpec> specs_;
  std::vector<JobDev> jobs_;
  std::vector<JobLayout> layouts_;
  std::vector<LaunchSet> rounds_;        // one per iteration round
  LaunchSet final_;                      // final phases
  std::vector<JobSlice> perm_;
  int perm_blocks_ = 0;
  std::vector<PrologueSlice> pro_;       // setup and factor tables, one launch
  int pro_blocks_ = 0;
  PrologueSlice* pro_dev_ = nullptr;
  // chained launch of the compressed passes (single job): iterations
  // 1..chain_rounds_ run in one k_pass_chain launch instead of rounds_
  std::vector<PassDesc> chain_descs_;
  PassDesc* chain_dev_ = nullptr;
  int chain_rounds_ = 0, chain_blocks_ = 0, chain_units_ = 1;
  bool perm_lds_ = true;
  size_t host_spot_bytes_ = 0;
  size_t raw_base_ = 0;
  DevBuf<char> arena_;
  DevBuf<char> table_;
  DevBuf<char> custom_;
  JobDev* jobs_dev_ = nullptr;
  JobSlice* perm_dev_ = nullptr;
  size_t table_bytes_ = 0;
  Staging staging_;
  Staging custom_staging_;
  bool untimed_ = false;  // adopted memory: no timing events
};


}  // namespace hg
