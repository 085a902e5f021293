// Internal interface between the kernels (kernels.hip) and the host runtime
// (runtime.hip, api.hip, engine.hip).  Nothing here is part of the C ABI.
//
// Every kernel works on a batch: a table of holograms ("jobs") resident in
// device memory, and per launch a list of descriptors, each naming one job and
// the slice of the grid that works on it.  A single hologram is a batch of
// one.  The launch geometry of a job's pass depends only on that job, so a
// hologram computed alone or inside any batch gives bit-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
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

// Device arrays of the N spot coordinates (mm) and target amplitudes.
struct SpotPtrs {
  const double* x;
  const double* y;
  const double* z;
  const double* amp;
};

constexpr int kBlock = 256;          // threads per block of the pixel kernels
// Counters of the cross-block hand-off sit one 128-byte line apart, so that
// the arrivals of different groups do not contend for one line.
constexpr int kCounterStride = 32;
constexpr int kWaves = kBlock / 64;  // wave64s per block
constexpr int kTile = 64;            // pixels per tile of a pass
constexpr int kFeistelRoundsHost = 6;  // rounds of the pixel permutation

// Launch geometry of one pass over `count` pixels.
struct PassPlan {
  int32_t tiles;       // tiles of `sub` x kTile pixels
  int32_t sub;         // kTile-pixel sub-tiles per tile (tiles <= kMaxTiles)
  int32_t blocks;      // blocks of this pass (they take the tiles dynamically)
  int32_t group_size;  // tiles per first-level reduction group
  int32_t ngroups;
  int32_t shift;       // fixed-point scale 2^shift of the exact sums (|sum| <= pixels)
};
constexpr int32_t kMaxTiles = 8192;
// Words per spot in the rows of exact sums: the atomic additions of
// different spots go to different cache lines.
constexpr int kAccSpotWords = 2;
// Pass totals in the exact sums: kAccTotalRows sets of kAccReplicas rows.
// A compressed pass followed by another compressed pass of the same job
// (a deferring pass) adds each tile's sums straight into row
// tile mod kAccReplicas of set it mod 3 (it = iteration), with no counting:
// the next pass reads the set after this launch has ended and adds its rows
// (integer sums, so the total is the same whatever the split), and the pass
// after that clears it.  Other passes hand their sums over through group
// rows into the first row of their set (set 0 unless pending).
constexpr int kAccTotalRows = 3;
constexpr int kAccReplicas = 10;
constexpr int kAccGroupRow0 = kAccTotalRows * kAccReplicas;  // row of group 0
// Fixed-point scale of the exact sums of a pass over `pixels` pixels: every
// term has magnitude <= 1, so |sum| * 2^shift <= 2^62.
int sum_shift(int64_t pixels);
// Tiles of one kTile sub-tile while there are at most kMaxTiles of them;
// min(tiles, block_cap) blocks; groups of ceil(sqrt(tiles)) tiles.
PassPlan plan_pass(int32_t count, int32_t block_cap);
constexpr int32_t kDefaultBlockCap = 4096;

// Pupil of the setup (paper section 4): a round aperture of diameter D
// pixels and a Gaussian illumination.  With doubled offsets the aperture
// holds the pixels with Lx^2 + Ly^2 <= q, q = floor(D^2) (Lx, Ly, q
// integers), and in row j (Ly = 2j - (H-1)) these are the columns of one
// run: |Lx| <= s with s = floor(sqrt(q - Ly^2)).  Shared by the host (pupil
// size) and the setup kernel (row tables of the random order).
__host__ __device__ inline int64_t isqrt64(int64_t t) {
  int64_t s = (int64_t)sqrt((double)t);
  while (s * s > t) --s;
  while ((s + 1) * (s + 1) <= t) ++s;
  return s;
}
// Columns [*i0, *i1] of row j inside the aperture (q < 0: no aperture, the
// whole row); returns the count (0: none, and then *i0 > *i1).
__host__ __device__ inline int32_t pupil_run(int32_t W, int32_t H, int32_t q, int32_t j,
                                             int32_t* i0, int32_t* i1) {
  if (q < 0) {
    *i0 = 0;
    *i1 = W - 1;
    return W;
  }
  const int64_t ly = 2 * (int64_t)j - (H - 1);
  const int64_t t = (int64_t)q - ly * ly;
  if (t < 0) {
    *i0 = 1;
    *i1 = 0;
    return 0;
  }
  const int64_t s = isqrt64(t);
  // Lx = 2i - (W-1) in [-s, s]
  const int64_t lo = (W - 1) - s, hi = (W - 1) + s;
  const int64_t a = lo <= 0 ? 0 : (lo + 1) / 2;
  const int64_t b = hi / 2 < W - 1 ? hi / 2 : W - 1;
  *i0 = (int32_t)a;
  *i1 = (int32_t)b;
  return b >= a ? (int32_t)(b - a + 1) : 0;
}

// One hologram resident on the device.
struct JobDev {
  int32_t W, H, N, M;
  int32_t P;           // pixels of the pupil Omega (M without an aperture):
                       // the full pass's count and the random order's length
  int32_t ap_q;        // aperture: the pixels with Lx^2 + Ly^2 <= ap_q (-1: all)
  float ill_a;         // illumination A = exp(-Q ill_a), Q = Lx^2 + Ly^2 (0: A = 1)
  int32_t* rows;       // [2H + 1] (aperture and a random order): pupil pixels
                       // before row j (j <= H), then the first pupil column
                       // of each row
  int32_t iterations;
  int32_t m;           // pixels of a compressed pass (M if not compressed)
  int32_t compressed;  // 1: passes 1..I-1 use windows of the random order
  int32_t h;           // Feistel half width (compressed only)
  uint64_t seed;       // theta^0
  uint64_t order_key;  // key of the random order's Feistel tables
  int32_t order_shared;  // tab, perm and rows belong to an order shared by
                         // the holograms of this grid (built once): the
                         // setup leaves them alone and no permutation runs
  double pitch_mm, lambda_mm, focal_mm;
  SpotPtrs in;         // spot inputs (device)
  SpotRec* sp;         // [N] iteration state
  SpotRec* sp_alt;     // [N] second state buffer of deferred updates (FP32 jobs)
  int32_t defer_ok;    // deferred updates allowed: an FP32 job of one spot unit
                       // per wave (N <= 256), whose passes run in the one-unit
                       // launch of each round
  float2* coef;        // [N] C_n = A_n e^{i 2 pi th_n}, kept with the state
  uint32_t* tab;       // [6 << h] Feistel tables (compressed only)
  int32_t* perm;       // [P] random pixel order (compressed only)
  float* phi;          // [H][W] output hologram (or input of a forward test pass)
  float2* partial;     // [max pass tiles][N] (mixed-precision passes)
  double2* gpart;      // [max pass groups][N] (mixed-precision passes)
  // exact fixed-point sums of the FP32 passes: rows 0..kAccGroupRow0-1 the
  // sets of pass totals, row kAccGroupRow0 + g group g; per spot a (re, im) two's-
  // complement pair at the start of an entry of kAccSpotWords words; zero
  // between passes, except a total that a deferred update leaves for the
  // next pass
  unsigned long long* acc;  // [kAccGroupRow0 + max pass groups][N][kAccSpotWords]
  int64_t acc_len;
  unsigned* counters;  // [max pass groups + 1] group and pass counters, kCounterStride apart
  unsigned* grab;      // [iterations + 2] tile counters of the passes (PassDesc::grab_slot)
  int32_t counters_len;  // counters, grab and gen, zeroed by the setup
  unsigned* gen;       // [kGenCopies * kCounterStride] passes completed in a chained launch
  int32_t trace;       // V is [iterations][N] instead of [N]
  double2* V;
  int32_t* status;     // sticky status word of the caller's stream
  // factor tables of the full-grid passes in the lane order of the matrix-
  // core operands (see SepDesc and MxDesc); dimensions shared by both forms
  int32_t mixed;
  int32_t shared_e;    // compressed passes in the shared-exponential form
  int32_t mx_steps;    // Np / 16 with Np = N rounded up to 16
  int32_t mx_cblocks;  // Wp / 16 with Wp = W rounded up to 64
  int32_t mx_rblocks;  // Hp / 16
  // FP32 separable passes (FP32 jobs)
  float* sepFc;        // [Wp/16][Np/2][64]   back-propagation B operand
  float* sepFn;        // [Np/16][Wp/2][64]   forward B operand
  float2* sepGa;       // [Hp/16][Np/2][64]   G by row, per lane
  float4* sepGv;       // [Hp/16][Np/16][64] x 2 float4: G for the V sums
  // mixed-precision matrix-core passes: FP16 / FP32 tables
  uint4* mxFc;         // [Wp/16][Np/16][64] x 4 half2   (back-propagation operand)
  uint4* mxFn;         // [Np/16][Wp/16][64] x 4 half2   (forward operand)
  float4* mxGa;        // [Hp/16][Np/16][64] x 4 float2  (rows by lane)
  float4* mxGv;        // [Hp/16][Np/16][64] x 4 float2  (spots by lane)
  // SLM output: with a table, the final pass also writes the gray image
  const uint16_t* lut; // [lut_levels] gray value of each phase bin (or nullptr)
  int32_t lut_levels;
  int32_t gray_bits;   // 8 or 16: element type of gray
  void* gray;          // [H][W] gray image of the final hologram
};

// Pixel set of a pass: all pixels 0..count-1 (perm == idx == nullptr; with
// an aperture the pixels outside it are weighted 0, so the set is Omega),
// perm[(start + q) mod M] for q < count (M: the order's length), or
// explicit indices idx[q].
struct PixelSet {
  const int32_t* perm;
  const int32_t* idx;
  int64_t start;
  int32_t count;
  int32_t M;
};

// One pass of one job inside a batched launch.
struct PassDesc {
  int32_t block_begin;  // first block of the launch working on this pass
  int32_t job;
  PixelSet ps;
  PassPlan plan;
  int32_t update;       // apply eqs. (4)-(6) after the sums
  int32_t from_phi;     // forward of job.phi instead of back-propagation
  int32_t grab_slot;    // tile counter of this pass: job.grab[grab_slot]
  double inv_count;
  double2* V;           // spot fields of this pass, [N]
  // Deferred updates between consecutive compressed passes of a job
  // (N <= kPendMaxSpots).  A deferring pass stops once its tiles have
  // added into the rows of total set tot_row: the counts, the hand-off, the
  // read of the total and the update leave its critical path.  The next pass is pending:
  // every block applies that update to the state st_in at its start (the
  // same FP32 operations in the same order, so the same bits) and keeps the
  // result in LDS; its block 0 stores it to st_out when the pass defers in
  // turn, and clears total set clear_row.  A pending pass that does not
  // defer updates from its LDS state as usual and clears set prev_row at the end.
  int32_t defer = 0;
  int32_t pending = 0;
  int32_t tot_row = 0;     // total set of this pass's sums
  int32_t prev_row = 0;    // total set of the previous pass (pending)
  int32_t clear_row = -1;  // total set block 0 clears at its start (pending)
  double prev_inv = 0.0;   // 2^-shift / count of the previous pass (pending)
  const SpotRec* st_in = nullptr;  // state before the previous pass's update
  SpotRec* st_out = nullptr;       // updated state, for the next pass (pending and defer)
  double2* prev_V = nullptr;       // spot fields of the previous pass (traced jobs)
};
constexpr int kPendMaxSpots = 256;

// Final hologram of one job over a pixel set, written compactly to out[q].
struct BackDesc {
  int32_t block_begin;
  int32_t job;
  PixelSet ps;
  float* out;
};

// One job's share of a batched permutation launch.
struct JobSlice {
  int32_t block_begin;
  int32_t job;
};

// ---- prologue (FP64) ----
// One job's share of a prologue launch: blocks [block_begin, block_begin +
// setup_blocks) set up its spot records, theta^0, state, counters and exact
// sums (and the Feistel tables of a random order of its own); the next
// table_blocks build the factor tables of its full-grid passes (separable
// FP32 or mixed precision), which depend on the spot inputs alone.
struct PrologueSlice {
  int32_t block_begin;
  int32_t job;
  int32_t setup_blocks;
  int32_t table_blocks;
};
int prologue_setup_blocks(const JobDev& j);
int prologue_table_blocks(const JobDev& j);  // 0 without matrix-core passes
void launch_prologue(const JobDev* jobs, const PrologueSlice* slices, int nslices,
                     int total_blocks, hipStream_t s);
// Random pixel order of the compressed jobs; slices[] maps blocks to jobs.
int perm_blocks(int32_t M);
void launch_perm_batch(const JobDev* jobs, const JobSlice* slices, int nslices, int total_blocks,
                       bool lds, hipStream_t s);
void launch_theta0(uint64_t seed, int count, double* out, hipStream_t s);
void launch_set_state(int N, const double* wth, SpotRec* sp, float2* coef, hipStream_t s);
void launch_gather(const PixelSet& ps, int32_t* out, hipStream_t s);

// ---- iteration ----
// Units of phase-2 work per wave for N spots (selects the kernel variant).
int pass_units_per_wave(int N);
// Register width of the shared-exponential form for N spots (0: N too large
// for it; the two-phase form is used).
__host__ __device__ int pass_e_width(int N);
// Passes of jobs with pass_e_width(N) > 0 (and not from a stored Phi) use
// the shared-exponential form; e_width is the largest width they need,
// max_units the largest two-phase unit count of the others.
void launch_pass_batch(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                       int max_units, int e_width, hipStream_t s);
// Compressed passes of mixed-precision jobs (the per-pixel pass with FP16
// back-propagation products accumulated in FP32); descs and units as for
// launch_pass_batch.
void launch_pass_mx(const JobDev* jobs, const PassDesc* descs, int ndesc, int total_blocks,
                    int max_units, hipStream_t s);
void launch_backprop_batch(const JobDev* jobs, const BackDesc* descs, int ndesc,
                           int total_blocks, hipStream_t s);
int backprop_blocks(int32_t count);

// ---- chained compressed passes ----
// The compressed passes of one job in one cooperative launch (all blocks
// resident): the block that completes pass p applies the update, writes the
// spot state with device-scope stores and then sets the generation word to
// p + 1 (in kGenCopies copies, one per 128-byte line, so that the waiting
// blocks poll different lines); the others wait for it, then read the state
// with device-scope loads into LDS.  Waits are bounded: a wait that runs out
// sets the status word (HG_EDEVICE) and ends the launch.
constexpr int kChainMaxSpots = 256;
constexpr int kGenCopies = 16;
// Largest grid of k_pass_chain<units> that is resident at once (0: none).
int pass_chain_capacity(int max_units);
hipError_t launch_pass_chain(const JobDev* jobs, const PassDesc* descs, int npass, int blocks,
                             int max_units, hipStream_t s);

// ---- separable full-grid passes ----
// eq. (2) splits into a part in x' and a part in y': with doubled offsets,
//   phi_n / 2pi = fx_n(i) + fy_n(j),  fx_n = cx Lx + cz Lx^2,  fy_n = cy Ly + cz Ly^2,
// so e^{i phi_n(i,j)} = F_n(i) G_n(j).  A full-grid back-propagation is then
// the complex product S = B F (B_n(j) = C_n G_n(j), C_n = A_n e^{i th_n}) and the
// full-grid forward sum is V_n = (1/M) sum_j conj(G_n(j)) sum_i u(j,i) conj(F_n(i)).
constexpr int kSepTileH = 64;  // output tile of the separable passes: rows (16 per wave)
constexpr int kSepTileW = 32;  // and columns
struct SepDesc {
  int32_t block_begin;
  int32_t job;
  int32_t tiles_x;      // ceil(W / kSepTileW)
  int32_t tiles_y;      // ceil(H / kSepTileH)
  PassPlan plan;        // blocks = tiles_x * tiles_y, reduction groups
  int32_t update;       // weight update after the sums (fused passes)
  double inv_count;
  double2* V;
  float* out;           // final-phase variant: Phi output
  // Deferred updates, as in PassDesc: a pending pass (or final hologram)
  // applies the previous pass's update at its start, into LDS (records and
  // C_n); a deferring pass adds its tiles' sums into total set tot_row and
  // stops.
  int32_t defer = 0;
  int32_t pending = 0;
  int32_t tot_row = 0;
  int32_t prev_row = 0;
  int32_t clear_row = -1;
  double prev_inv = 0.0;
  const SpotRec* st_in = nullptr;
  SpotRec* st_out = nullptr;
  double2* prev_V = nullptr;
};
// (The factor tables are built by the prologue from FP64 phases: the spots
// do not move during the iterations.)

PassPlan plan_sep(int W, int H);
// Fused full-grid pass (back-propagation S = B F and forward T = U conj(F)^T
// on the FP32 matrix cores, exact sums, update) or, with final != 0, the
// full-grid hologram Phi = arg(B F).  max_steps: largest Np / 16.
void launch_sep_pass(const JobDev* jobs, const SepDesc* descs, int ndesc, int total_blocks,
                     bool final, int max_steps, hipStream_t s);

// ---- mixed-precision passes (FP16 matrix cores, FP32 sums) ----
// A pass is the separable recast above on the matrix cores: per output tile
// of kMxTile x kMxTileW pixels (wave w: rows 16w..16w+15), S = B F with FP16
// operands and FP32 accumulation (K = 2 Np: real and imaginary parts
// interleaved), u = S / |S| on every pixel of the pupil (else 0),
// T = u conj(F)^T the same way, and the tile's partial
// V_n = sum_j conj(G_n(j)) T[j][n].  These are the full-grid passes of the
// mixed form (its compressed passes run per pixel: launch_pass_mx).
// Partials are added across tiles with compensated FP32 sums.
constexpr int kMxTile = 64;   // table geometry: rows and columns padded to it
constexpr int kMxTileW = 32;  // columns of a pass tile (rows: kMxTile)
enum MxMode : int32_t { kMxIterate = 0, kMxFinal = 1, kMxFromPhi = 2 };
struct MxDesc {
  int32_t block_begin;
  int32_t job;
  int32_t tiles_x, tiles_y;
  PassPlan plan;
  int32_t update;       // weight update after the sums
  float inv_count;
  double2* V;           // [N] spot fields of the pass (FP32 values widened)
  float* out;           // final hologram (kMxFinal)
  // Deferred updates, as in PassDesc: a pending pass applies the previous
  // (compressed) pass's update at its start, into LDS (records and C_n).
  // These passes do not defer their own.
  int32_t defer = 0;
  int32_t pending = 0;
  int32_t tot_row = 0;
  int32_t prev_row = 0;
  int32_t clear_row = -1;
  double prev_inv = 0.0;
  const SpotRec* st_in = nullptr;
  SpotRec* st_out = nullptr;
  double2* prev_V = nullptr;
};
PassPlan plan_mx(int W, int H);
// (FP16 / FP32 tables built by the prologue from FP64 phases.)

// mode: MxMode; max_steps: largest Np / 16 among the descriptors.
void launch_mx_pass(const JobDev* jobs, const MxDesc* descs, int ndesc, int total_blocks,
                    int mode, int max_steps, hipStream_t s);

// ---- SLM output ----
// gray[p] = lut[bin(phi[p])] for p < count (see gray_level).
void launch_phase_to_gray(const float* phi, int64_t count, const uint16_t* lut, int levels,
                          int bits, void* gray, hipStream_t s);

// ---- metrics (FP64) ----
struct SetupArgs {
  int32_t N;
  int32_t W, H;
  double pitch_mm, lambda_mm, focal_mm;
};
void launch_metric_tables(const SetupArgs& a, const SpotPtrs& in, double2* Ex, double2* Ey,
                          hipStream_t s);
int metric_blocks(int H);
// ap_q, ill_a: the pupil (JobDev), ill_a here in FP64.
void launch_metric_rows(const double2* Ex, const double2* Ey, int N, int W, int H,
                        const float* phi, int32_t ap_q, double ill_a, double2* partial,
                        hipStream_t s);
void launch_metric_reduce(const double2* partial, int nblk, int N, double inv_count,
                          double2* V_out, hipStream_t s);

}  // namespace hg
