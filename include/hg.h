/*
 * hg.h - C ABI of libhg: phase-only holograms of 3-D spot clouds on AMD
 * MI355X (gfx950) by random superposition (RS), weighted Gerchberg-Saxton
 * (WGS) and compressed-sensing WGS (CS-WGS).
 *
 * Method: Pozzi & Mapelli, "Real time computer generation of
 * three-dimensional point cloud holograms through GPU implementation of
 * compressed sensing Gerchberg-Saxton algorithm" (arXiv 2003.05293),
 * section 2, eqs. (1)-(7).
 *
 * Conventions shared by every call
 * --------------------------------
 * Pixel grid (paper, GPU implementation section, fixed SLM parameters):
 *   W columns, H rows, square pixels of pitch `pitch_mm`; pixel (i, j) sits at
 *   x'_i = (i - (W-1)/2) * pitch, y'_j = (j - (H-1)/2) * pitch and has flat
 *   index p = j*W + i.  Every full-grid phase buffer is float32 [H][W]
 *   row-major, radians in (-pi, pi].
 * Spot phase phi_n (eq. 2), back-propagation (eq. 1), forward projection
 *   (eq. 3, read with the + sign and as a mean over the pixel set with
 *   uniform illumination), weight update (eqs. 4-6) and metrics (eq. 7)
 *   are as in the paper.
 * Random draws: theta_n^0 comes from the 64-bit `seed` through
 *   Philox4x64-10; the pixel subsets of the compressed iterations come from
 *   one keyed six-round Feistel permutation of [0, W*H) per grid and pupil
 *   (key HG_ORDER_KEY: one random pixel order of the SLM, as in the paper's
 *   compressed-sensing subsection; iteration j uses the window of
 *   m = ceil(c*W*H) consecutive entries starting at (j-1)*m, wrapping at
 *   W*H).
 *
 * Ownership: the caller owns every buffer.  Host arrays are read during the
 *   call only.  Device buffers (`*_dev`) are caller allocations on the
 *   current HIP device (for example torch tensors' data_ptr()).  `stream`
 *   is a hipStream_t (NULL = the default stream); work is enqueued on it in
 *   order.  The library keeps per-stream scratch memory that it allocates
 *   on first use and reuses; hg_release() frees it.  Two calls that overlap
 *   on different streams use different scratch and do not race.
 *
 * Errors: every call validates all arguments before launching anything.
 *   On failure it returns a non-zero hg_status, writes no output, and sets a
 *   thread-local message readable with hg_last_error().  No C++ exception
 *   crosses this interface.
 *
 * Limits: 1 <= W, H <= 8192; 1 <= N <= HG_MAX_SPOTS; 0 <= iterations <=
 *   HG_MAX_ITERATIONS; 0 < compression <= 1; pitch, wavelength, focal length
 *   positive and finite; coordinates finite; amplitudes positive and finite.
 */
#ifndef HG_H
#define HG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HG_MAX_SPOTS 4096
#define HG_MAX_ITERATIONS 100000
/* Key of the random pixel order of the compressed iterations.  As in the
 * paper's compressed-sensing subsection (one random order of the SLM's
 * pixels, made at start-up), every hologram of one grid and pupil uses the
 * same order: the algorithms key it with HG_ORDER_KEY, the library builds
 * it once per device, grid and pupil on first use (that call blocks until
 * it is complete) and keeps it until hg_release.  The hologram's seed
 * draws theta^0 only.  hg_subset takes the key as an argument. */
#define HG_ORDER_KEY 0ull

typedef enum hg_status {
  HG_OK = 0,
  HG_EINVAL = 1,   /* an argument is out of range, NULL or not finite        */
  HG_ENOMEM = 2,   /* device or pinned host allocation failed                */
  HG_EBUSY = 3,    /* engine: no slot or memory free for the request now     */
  HG_ENUMERIC = 4, /* a spot field came out zero or not finite               */
  HG_EDEVICE = 5   /* a HIP runtime call or kernel launch failed             */
} hg_status;

/* SLM pixel grid (paper: pixel coordinates x', y' uploaded once). */
typedef struct hg_grid {
  int32_t W;        /* columns (x')                                        */
  int32_t H;        /* rows (y')                                           */
  double pitch_mm;  /* pixel pitch                                         */
} hg_grid;

/* Optics of eq. (2): wavelength lambda and focal length f, in mm, and the
 * pupil of the experimental setup (section 4: a Gaussian beam on the SLM
 * behind the round aperture of the optics).  Both pupil fields are finite
 * and >= 0; 0 turns the part off.
 *   waist_mm:    the forward projection (eq. 3) weights each pixel by the
 *                illumination amplitude A = exp(-(x'^2 + y'^2) / waist^2);
 *                the metrics then divide the efficiency by the mean of A^2
 *                over the pupil (the power on the SLM), so e <= 1.
 *   aperture_px: diameter D in pixels of the round aperture: the pupil
 *                Omega is the set of pixels whose centre lies within D/2
 *                pixel pitches of the grid centre, i.e. with doubled offsets
 *                Lx = 2i - (W-1), Ly = 2j - (H-1), Lx^2 + Ly^2 <= D^2.  The
 *                forward sums of every iteration (the full set, and the
 *                random order of CS-WGS, taken over the |Omega| pupil pixels
 *                in index order) and the metrics run over Omega only; the
 *                hologram is still computed on every pixel.  HG_EINVAL if
 *                Omega is empty.
 * A zero-initialised pupil is the uniform full rectangle. */
typedef struct hg_optics {
  double lambda_mm;
  double focal_mm;
  double waist_mm;
  double aperture_px;
} hg_optics;

/* N target spots X_n = (x_n, y_n, z_n) in mm and target amplitudes a_n^0
 * (relative intensities |a_n^0|^2), section 2.  Four host arrays of n
 * doubles each. */
typedef struct hg_spots {
  int32_t n;
  const double *x_mm;
  const double *y_mm;
  const double *z_mm;
  const double *amp;
} hg_spots;

/* Arithmetic of the iteration kernels (low bits of hg_params.flags and of
 * the flags argument of the single-step calls). */
#define HG_PREC_FP32 0u   /* FP32 phases, sincos and sums                  */
#define HG_PREC_MIXED 1u  /* back-propagation as FP16 products
                             accumulated in FP32 (compressed passes: per
                             pixel, the cosines, sines and amplitudes of
                             two spots per FP16 dot product, exact sums;
                             full-grid passes: FP16 matrix cores,
                             compensated FP32 sums)                        */
#define HG_PREC_MASK 0xffu
/* hg_params.flags: the four hg_spots arrays are device pointers (already
 * in HBM) instead of host pointers.  Their values are then checked on the
 * device; a non-finite coordinate or a non-positive amplitude is reported
 * as HG_EINVAL by the next blocking call on the stream. */
#define HG_SPOTS_ON_DEVICE 0x100u
/* hg_params.flags, hg_job.flags and the single-step calls: compute full-grid
 * passes with the per-pixel kernels (phase and sincos per pixel and spot,
 * as in the paper's GPU section) instead of the default separable products
 * (eq. 2 factorises into an x' part and a y' part, so a full-grid
 * back-propagation is a complex matrix product over the spots and the
 * full-grid forward sum a product over the pixel columns).  Both compute
 * the same sums; the summation order differs. */
#define HG_FULL_DIRECT 0x200u

/* Extended parameters of hg_cswgs_ex. */
/* Launch parameters of the passes, 0 meaning the default.
 * Block caps: a pass runs on min(tiles, cap) blocks that take its tiles of
 * pixels dynamically (full-grid and compressed passes have separate caps).
 * Partial sums are kept per tile, whichever block computes it, so the caps
 * never change the results, only the speed.
 * pass_form (FP32 per-pixel passes): 0 = two sincos per (pixel, spot) pair,
 * one per propagation direction; 1 = one complex exponential per pair, kept
 * in registers between the directions (jobs with N <= 100; others use 0).
 * The form changes the rounding of the sums (both stay within the same
 * accuracy bars).
 * chain_passes: 1 = the compressed passes of a single FP32 hologram
 * (hg_cswgs, hg_cswgs_ex; two-sincos form, N <= 256) run in one cooperative
 * launch, each pass handing the updated spot state to the next through
 * device memory, when all its blocks fit on the device at once; 0 = one
 * launch per pass.  Both give bit-identical results.
 * Chosen per shape by the package's autotuner. */
typedef struct hg_tune {
  int32_t full_block_cap;
  int32_t subset_block_cap;
  int32_t pass_form;
  int32_t chain_passes;
} hg_tune;

/* Phase-to-gray lookup table of the SLM (GPU implementation section: a
 * fixed parameter of the SLM, uploaded to the device once at start-up and
 * used for every hologram).  levels gray values g[0..levels-1] cover one
 * phase period: bin k holds the phases Phi (radians, any real) with
 * k/levels <= frac(Phi / 2 pi) < (k+1)/levels.  The bin is decided in FP32:
 * t = fl(Phi * fl(1/(2 pi))), t = fl(t - floor(t)), k = min(floor(fl(t *
 * levels)), levels - 1).  bits: 8 (gray images of uint8) or 16 (uint16).
 * The table lives on the device that is current at creation. */
typedef struct hg_lut hg_lut;

typedef struct hg_params {
  int32_t iterations;    /* I >= 0                                          */
  double compression;    /* c in (0, 1]; 1 gives WGS                        */
  uint64_t seed;         /* theta^0 and subsets                             */
  uint32_t flags;        /* HG_PREC_*                                       */
  double *trace_V;       /* NULL, or host [iterations][N][2] doubles: the
                            spot field V^j (re, im) of every iteration j    */
  hg_tune tune;          /* launch geometry (zeros: defaults)               */
  const hg_lut *lut;     /* NULL, or the SLM table: the final pass also
                            writes the gray image of Phi^I to gray_dev      */
  void *gray_dev;        /* device [H][W] uint8 or uint16 (the table's
                            bits); NULL exactly when lut is NULL            */
} hg_params;

/* ---------------------------------------------------------------------- */
/* Algorithms                                                             */
/* ---------------------------------------------------------------------- */

/* RS (section 2, eq. 1 with random theta_n^0 and w_n = 1).  Writes the
 * hologram Phi^0 to phi_dev (float32 [H][W], radians).  Asynchronous. */
hg_status hg_rs(const hg_grid *grid, const hg_optics *optics,
                const hg_spots *spots, uint64_t seed, float *phi_dev,
                void *stream);

/* WGS (section 2, eqs. 1-6): RS, then `iterations` iterations of forward
 * projection over all pixels, weight update and back-propagation.
 * iterations = 0 gives RS.  Writes Phi^I to phi_dev.  Asynchronous. */
hg_status hg_wgs(const hg_grid *grid, const hg_optics *optics,
                 const hg_spots *spots, int32_t iterations, uint64_t seed,
                 float *phi_dev, void *stream);

/* CS-WGS (section 2, compressed variant; GPU section, compressed sensing):
 * as WGS, but the forward sum of iteration j < I runs over the random subset
 * Omega^j of m = ceil(c*W*H) pixels, and the phase is computed only where
 * the next forward step reads it; iteration I and the output Phi^I use all
 * pixels.  compression = 1 gives WGS (same sets, other summation order).
 * Asynchronous. */
hg_status hg_cswgs(const hg_grid *grid, const hg_optics *optics,
                   const hg_spots *spots, int32_t iterations,
                   double compression, uint64_t seed, float *phi_dev,
                   void *stream);

/* CS-WGS with the precision flag and an optional per-iteration trace of the
 * spot fields.  With trace_V != NULL the call blocks until the trace is on
 * the host; otherwise it is asynchronous. */
hg_status hg_cswgs_ex(const hg_grid *grid, const hg_optics *optics,
                      const hg_spots *spots, const hg_params *params,
                      float *phi_dev, void *stream);

/* Size of the static device scratch of hg_cswgs_static, per GPU. */
#define HG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* hg_cswgs_ex for callers that cannot allocate memory: tight serving loops
 * and harnesses that forbid hipMalloc after start-up.  (It stages launch
 * descriptors through host memory and waits for the previous upload, so it
 * is not meant to be recorded into a HIP graph; hg_batch_create is.)
 * Computes the same hologram as hg_cswgs_ex with the same arguments (the
 * same kernels, bit-identical results) without allocating: no hipMalloc,
 * hipHostMalloc or hipFree and no torch allocation.  Its device scratch
 * (spot state, random order, factor tables, sums and counters, launch
 * descriptors) is a file-scope static array of HG_STATIC_SCRATCH_BYTES,
 * of which each GPU the library runs on holds its own copy until the
 * process ends; the descriptors are staged through a static host area of
 * 1 MiB.  The first call on a device sets that device up (looks up its
 * copy of the array and creates one event).  Host-side planning still uses
 * ordinary C++ containers.
 * Arguments: as hg_cswgs_ex, with these restrictions, each rejected with
 * HG_EINVAL before anything runs: params->flags must have
 * HG_SPOTS_ON_DEVICE (spot arrays in HBM) and params->trace_V must be NULL.
 * A hologram whose scratch or descriptors do not fit is rejected with
 * HG_ENOMEM and a message giving the bytes it needs.  The 64 MiB hold, for
 * example, an FP32 CS-WGS hologram of 1152 x 1152 pixels with N <= 1200 or
 * of 1920 x 1152 with N <= 900 (mixed precision: N <= 1600 and 1100), and
 * the descriptors of up to 4000 iterations.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind; the kernels clear what must start at zero.  Calls that overlap on
 * one GPU (two streams, or two host threads) race on the array and give
 * undefined results: serialise them.  Device-side numeric flags are not
 * reported by this call.  Asynchronous. */
hg_status hg_cswgs_static(const hg_grid *grid, const hg_optics *optics,
                          const hg_spots *spots, const hg_params *params,
                          float *phi_dev, void *stream);

/* Efficiency and uniformity of a hologram (section 2, last paragraph, and
 * eq. 7), in FP64: V*_n = mean over the pupil Omega of
 * A(p) e^{i(Phi - phi_n)}, I_n = |V*_n|^2, e = sum_n I_n / mean_Omega(A^2),
 * u = 1 - (max I - min I)/(max I + min I).  Without a pupil, Omega is every
 * pixel and A = 1.  phi_dev: float32 [H][W].  intensities: NULL or host
 * array of N doubles.  Blocks until the results are on the host. */
hg_status hg_metrics(const hg_grid *grid, const hg_optics *optics,
                     const hg_spots *spots, const float *phi_dev, double *e,
                     double *u, double *intensities, void *stream);

/* ---------------------------------------------------------------------- */
/* Batches: many holograms per launch                                     */
/* ---------------------------------------------------------------------- */

/* One hologram of a batch.  The schedule is that of hg_cswgs (compression
 * in (0, 1]; iterations = 0 gives RS).  spots are host arrays, or device
 * arrays when flags has HG_SPOTS_ON_DEVICE.  phi_dev receives Phi^I,
 * float32 [H][W].  trace_V: NULL or host [iterations][N][2] doubles. */
typedef struct hg_job {
  hg_grid grid;
  hg_optics optics;
  hg_spots spots;
  int32_t iterations;
  double compression;
  uint64_t seed;
  uint32_t flags;
  float *phi_dev;
  double *trace_V;
  const hg_lut *lut;  /* as in hg_params: NULL, or the gray image of Phi^I */
  void *gray_dev;     /* to gray_dev                                      */
} hg_job;

/* Runs `count` holograms together (paper section 2 for each; the paper
 * computes one hologram at a time): one launch per iteration round covers
 * every hologram still iterating, so the per-iteration reductions of one
 * hologram overlap the work of the others.  Each hologram's result is
 * bit-identical to computing it alone.  tune may be
 * NULL.  Asynchronous unless a job asks for a trace. */
hg_status hg_cswgs_batch(int32_t count, const hg_job *jobs, const hg_tune *tune,
                         void *stream);

/* A reusable batch: planned and allocated once, then run any number of
 * times.  Every job must have HG_SPOTS_ON_DEVICE (each run reads the spot
 * arrays' current contents) and no trace.  With use_graph != 0 the first
 * run on a stream captures the whole schedule (setup, random orders, all
 * iteration rounds, final phases) as a HIP graph and later runs replay it;
 * the stream must then not be the NULL stream.  The batch owns its scratch
 * and releases it in hg_batch_destroy; runs of one batch share that scratch,
 * so they must not overlap (issue them on one stream).  Errors found on the
 * device (non-finite spot values) are not reported by the runs. */
typedef struct hg_batch hg_batch;
hg_status hg_batch_create(int32_t count, const hg_job *jobs, const hg_tune *tune,
                          int32_t use_graph, hg_batch **out);
hg_status hg_batch_run(hg_batch *batch, void *stream);
hg_status hg_batch_destroy(hg_batch *batch);

/* ---------------------------------------------------------------------- */
/* Serving: continuous batching of hologram requests                      */
/* ---------------------------------------------------------------------- */

/* An engine that admits hologram requests as device memory and slots free
 * up and advances every admitted hologram by one iteration per step, in one
 * batched launch, so that requests arriving while others run join the
 * running batch at the next step (continuous batching).  Each hologram's
 * launch geometry depends only on that hologram: a result is bit-identical
 * to computing the same request alone (hg_cswgs_batch of one, same tune). */
typedef struct hg_engine hg_engine;

typedef struct hg_engine_config {
  size_t mem_budget_bytes;  /* device scratch for admitted requests (one
                               pool allocated at creation)                   */
  int32_t max_slots;        /* holograms in flight at most (1 .. 4096)      */
  hg_tune tune;             /* launch geometry, 0 = default                 */
} hg_engine_config;

/* Creates the engine on the current device. */
hg_status hg_engine_create(const hg_engine_config *config, hg_engine **out);

/* Queues a request (one hologram, as in hg_job; no trace).  Host spot
 * arrays are copied; device spot arrays (HG_SPOTS_ON_DEVICE) and phi_dev
 * must stay valid until the request is done.  Returns a ticket.  A request
 * whose scratch can never fit the budget is rejected with HG_ENOMEM. */
hg_status hg_engine_submit(hg_engine *engine, const hg_job *job, uint64_t *ticket);

/* One engine step on `stream`: retires finished requests (their scratch
 * returns to the pool once the device is done with it), admits queued
 * requests in arrival order while a slot and room in the pool are free
 * (HG_EBUSY-style waiting: a request that does not fit yet stays queued),
 * sets them up, then launches one pass that advances every admitted
 * hologram by one iteration and the final phase of those that completed
 * their last iteration.  At most two steps are in flight on the device: a
 * step waits for the one before the previous.  pending_out (may be NULL)
 * receives the number of requests admitted or queued and not yet done. */
hg_status hg_engine_step(hg_engine *engine, void *stream, int32_t *pending_out);

/* done = 1 once the hologram of `ticket` is complete in its phi_dev buffer
 * (the device has finished it); 0 otherwise.  Unknown tickets: HG_EINVAL. */
hg_status hg_engine_poll(hg_engine *engine, uint64_t ticket, int32_t *done);

/* Waits for the device, frees the pool and the engine. */
hg_status hg_engine_destroy(hg_engine *engine);

/* ---------------------------------------------------------------------- */
/* Single steps, for testing each kernel against the oracle               */
/* ---------------------------------------------------------------------- */

/* theta_n^0 (radians, FP64) for n < count, computed on the device.  Blocks. */
hg_status hg_theta0(uint64_t seed, int32_t count, double *out_host);

/* Pixel indices of Omega^j (j >= 1) for compression c in the random order
 * keyed by `seed` (the algorithms' order is the one of seed = HG_ORDER_KEY):
 * writes m = ceil(c*|Omega|) int32 indices, in order, to idx_dev (capacity
 * >= m) and m to *m_out.  optics: NULL or its aperture_px alone is read (the
 * random order runs over the pupil pixels; |Omega| = W*H without an
 * aperture).  Blocks until *m_out is set. */
hg_status hg_subset(const hg_grid *grid, const hg_optics *optics, uint64_t seed,
                    int32_t j, double compression, int32_t *idx_dev,
                    int32_t *m_out, void *stream);

/* Forward projection (eq. 3) of a given hologram: V_n = mean over the pixel
 * set of A(p) e^{i(Phi(p) - phi_n(p))}, A the illumination amplitude of the
 * optics (1 without a waist).  phi_dev: float32 [H][W].  idx_dev: NULL for
 * the pupil Omega (all pixels without an aperture), else m device int32
 * pixel indices.  V_out: host, 2N doubles (re, im).  flags: HG_PREC_*.
 * Blocks. */
hg_status hg_forward(const hg_grid *grid, const hg_optics *optics,
                     const hg_spots *spots, const float *phi_dev,
                     const int32_t *idx_dev, int32_t m, uint32_t flags,
                     double *V_out, void *stream);

/* Back-propagation (eq. 1) with given weights w_n and phases theta_n (host,
 * N doubles each; a_n = w_n a_n^0): writes Phi at the pixel set to phi_dev,
 * compact: phi_dev[q] = Phi(idx[q]) for q < m, or phi_dev[p] for all p when
 * idx_dev is NULL.  flags: HG_PREC_*.  Asynchronous. */
hg_status hg_backward(const hg_grid *grid, const hg_optics *optics,
                      const hg_spots *spots, const double *w,
                      const double *theta, const int32_t *idx_dev, int32_t m,
                      uint32_t flags, float *phi_dev, void *stream);

/* One fused iteration body: back-propagation with (w, theta) on the pixel
 * set immediately followed by the forward projection over the same set
 * (eqs. 1 and 3, the pixel set and A as in hg_forward), returning V (host,
 * 2N doubles).  This is the kernel the iteration loop runs.  Blocks. */
hg_status hg_step(const hg_grid *grid, const hg_optics *optics,
                  const hg_spots *spots, const double *w, const double *theta,
                  const int32_t *idx_dev, int32_t m, uint32_t flags,
                  double *V_out, void *stream);

/* ---------------------------------------------------------------------- */
/* SLM output                                                             */
/* ---------------------------------------------------------------------- */

/* Uploads a phase-to-gray table (host, levels uint16 values; each <= 255
 * when bits is 8) to the current device.  levels in [1, 65536], bits 8 or
 * 16.  Blocks until the copy is done.  *out is owned by the caller. */
hg_status hg_lut_create(const uint16_t *gray, int32_t levels, int32_t bits,
                        hg_lut **out);

/* Frees a table.  Calls still running on the device may read it: the
 * caller synchronises the streams that used it first. */
hg_status hg_lut_destroy(hg_lut *lut);

/* Gray image of a hologram: gray_dev[p] = g[k(phi_dev[p])] for p < count
 * (device arrays; gray_dev of uint8 or uint16 by the table's bits), the
 * same conversion the final pass applies when hg_params.lut is set.
 * Asynchronous. */
hg_status hg_phase_to_gray(const hg_lut *lut, const float *phi_dev, int64_t count,
                           void *gray_dev, void *stream);

/* ---------------------------------------------------------------------- */
/* Library state                                                          */
/* ---------------------------------------------------------------------- */

/* Message of the last failed call on this thread ("" if none). */
const char *hg_last_error(void);

/* Frees all scratch memory after synchronising the streams that used it. */
hg_status hg_release(void);

/* Kernel timing for benchmarks.  While enabled, every launch of the
 * iteration kernels is bracketed by two HIP events recorded on the stream it
 * runs on.  hg_timing_read synchronises those events and returns, for the
 * kernel family `name` ("k_pass_subset": compressed iterations, "k_pass_full":
 * full-grid iterations, "k_backprop_phi": the final hologram), the summed
 * duration in ms and the number of launches since the last reset. */
hg_status hg_timing_enable(int on);
hg_status hg_timing_reset(void);
hg_status hg_timing_read(const char *name, double *total_ms, int64_t *launches);

/* Library version string. */
const char *hg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HG_H */
