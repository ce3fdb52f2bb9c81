/*
 * epic.h - C ABI of the MI355X (gfx950) MOFF direct imager.
 *
 * The library images channelised antenna E-fields the way the paper's EPIC
 * imager does (Kent et al. 2019, "A Real-Time, All-Sky, High Time Resolution,
 * Direct Imager for the Long Wavelength Array"):
 *   - Sec. 3.2: 4+4-bit complex samples ordered [Time][Channel][Pol][Antenna]
 *     are unpacked and multiplied by a per-antenna complex calibration factor
 *     (cable delays appear as a phase of that factor);
 *   - Sec. 2.1, Eq. (4)-(5): the calibrated point measurements are convolved
 *     with an illumination kernel W and gridded on a regular aperture grid whose
 *     spacing is a fixed fraction of the channel wavelength (half, Sec. 4.2);
 *   - Sec. 2.1, Eq. (5) and Sec. 3.2: each gridded aperture is transformed with
 *     an unnormalised 2-D DFT of positive exponent sign;
 *   - Sec. 2.1 and Sec. 3.2: the instantaneous images are squared or cross
 *     multiplied between polarisations (XX, XY, YX, YY) and summed over time.
 *
 * Conventions shared by every call
 *   - Every pointer documented as "device" is memory on the context's GPU that
 *     the caller owns; the library never frees or retains it after a call.
 *     "host" pointers are read during the call only.
 *   - complex64 = two interleaved float32 (re, im); complex128 = two
 *     interleaved float64.
 *   - Sample byte: high nibble = real part, low nibble = imaginary part, both
 *     two's complement in [-8, 7] (0x7F = 7 - 1i, 0x80 = -8 + 0i).
 *   - Grid: antenna a of channel c sits at cell coordinates
 *     X = x_a / (lambda_c * cell_wavelengths) + N/2, same for Y with y_a;
 *     lambda_c = 299792458 / freq_hz[c].  Its kernel taps are the K x K cells
 *     centred on (floor(X + 1/2), floor(Y + 1/2)); the weight of tap (i, j) is
 *     exp(-((i - X)^2 + (j - Y)^2) / (2 sigma^2)) (peak 1, not renormalised).
 *   - Image: F[km][kl] = sum_{j,i} A[j][i] exp(+2 pi i (i kl + j km) / N),
 *     A the gridded aperture (row j <-> y, column i <-> x).  Images are stored
 *     fftshifted: pixel (row q_m, col q_l) holds k = (q - N/2) mod N, i.e.
 *     direction l = (q_l - N/2) / (N * cell_wavelengths), same for m.
 *   - Products: n_pol = 2 -> 4 products in the order XX, XY, YX, YY with
 *     XY = F_X conj(F_Y), YX = F_Y conj(F_X); n_pol = 1 -> XX only.
 *   - Calls are enqueued on the context's stream and return before the GPU has
 *     finished; device faults surface at the caller's next synchronisation.
 *     Arguments are validated before anything is enqueued: on any error the
 *     outputs are untouched.  No call takes a lock; use one context per
 *     stream or host thread.
 *   - Results are deterministic: every reduction has a fixed order and no
 *     floating-point atomics are used, so identical calls give identical bits.
 */
#ifndef EPIC_H
#define EPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum epic_status {
  EPIC_OK = 0,
  EPIC_E_INVALID = 1,     /* null pointer, size out of range, non-finite geometry */
  EPIC_E_DEVICE = 2,      /* the device is not gfx950, or a HIP runtime call failed */
  EPIC_E_NOMEM = 3,       /* a device or host allocation failed */
  EPIC_E_OFFGRID = 4,     /* a kernel tap of some antenna leaves the grid */
  EPIC_E_STATE = 5,       /* antennas not set before an imaging call */
  EPIC_E_LAUNCH = 6,      /* a kernel launch was rejected */
  EPIC_E_UNSUPPORTED = 7  /* valid request outside what the library implements */
} epic_status;

/* epic_config.precision */
enum { EPIC_FP32 = 0, EPIC_SPLIT_FP16 = 1, EPIC_SPLIT_BF16 = 2 };

/* epic_config.flags */
enum {
  EPIC_FLAG_STAGED = 1,   /* one kernel per stage with FP32 intermediates in HBM
                             (the plain comparator); default is the fused kernel */
  EPIC_FLAG_TIMING = 2,   /* record HIP events around the main kernel of each call */
  EPIC_FLAG_REMOVE_AUTOS = 4  /* subtract the antenna autocorrelations from the image
                                 (see epic_image_accumulate) */
};

typedef struct epic_config {
  int32_t grid_n;              /* N: grid side; 32, 64 or 128 */
  int32_t n_chan;              /* C >= 1 */
  int32_t n_pol;               /* P: 1 or 2 */
  int32_t n_ant;               /* A: 1 .. 4096 */
  int32_t kernel_support;      /* K: odd, 1 .. 15 (EPIC_FLAG_REMOVE_AUTOS: 1 .. 7) */
  double kernel_sigma_cells;   /* Gaussian kernel width in cells, > 0 */
  double cell_wavelengths;     /* grid spacing in wavelengths, > 0 (0.5 = lambda/2) */
  int32_t precision;           /* EPIC_FP32, EPIC_SPLIT_FP16 or EPIC_SPLIT_BF16 */
  int32_t flags;               /* EPIC_FLAG_* */
} epic_config;

typedef struct epic_ctx epic_ctx;

/* Create a context on `device` (a HIP device ordinal).  Not an operation of
 * the paper: it holds the imager's configuration -- the grid side, channel,
 * polarisation and antenna counts and the gridding kernel of Sec. 2.1 and
 * Sec. 3.2 -- and the workspace every later call reuses, so that no imaging
 * call allocates.  All later work of the
 * context is enqueued on `hip_stream` (a hipStream_t; NULL = the null stream).
 * The config is copied.  Allocates the library-owned tables and workspace.
 * Errors: EPIC_E_INVALID (bad config or out == NULL), EPIC_E_DEVICE (not a
 * gfx950 device), EPIC_E_NOMEM.  On error *out is set to NULL. */
epic_status epic_init(const epic_config *cfg, int device, void *hip_stream,
                      epic_ctx **out);

/* Rebind the context to another stream (hipStream_t). */
epic_status epic_set_stream(epic_ctx *ctx, void *hip_stream);

/* Set the array geometry (Sec. 3.2 and Sec. 4.2: gridding at a fixed fraction
 * of each channel's wavelength).  xy_m: host float64 [n_ant][2] (east, north)
 * in metres; freq_hz: host float64 [n_chan].  Builds the per-channel kernel
 * weights (in float64, rounded once to float32) and the gridding tables and
 * uploads them before returning (synchronous).  May be called again.
 * Errors: EPIC_E_INVALID (null, non-finite position, frequency not finite and
 * positive), EPIC_E_OFFGRID (a tap outside [0, N) for some channel; the
 * previous geometry, if any, stays in force), EPIC_E_NOMEM. */
epic_status epic_set_antennas(epic_ctx *ctx, const double *xy_m, const double *freq_hz);

/* epic_set_antennas with the caller's own gridding kernels in place of the
 * Gaussian (Sec. 3.3: the gridding convolution takes any kernel per antenna,
 * e.g. its illumination pattern for A-projection).  kernels: host complex64
 * [n_chan][n_ant][K][K] (K = kernel_support, up to 15; row dj outer, column
 * di inner), the weight of antenna a at cell (i0 + di - K/2, j0 + dj - K/2)
 * of channel c, where (i0, j0) is the cell nearest to the antenna (as for
 * the Gaussian).  Copied; kernels == NULL is epic_set_antennas.  Works on
 * every path (fused, staged, split), in epic_image_backward and with
 * EPIC_FLAG_REMOVE_AUTOS (kernel_support <= 7 there).
 * Errors: as epic_set_antennas; EPIC_E_INVALID (a non-finite kernel value). */
epic_status epic_set_antennas_kernels(epic_ctx *ctx, const double *xy_m, const double *freq_hz,
                                      const float *kernels);

/* Host-side view of the gridding programs the fused kernels run for a
 * configuration and geometry (Sec. 2.1 Eq. (4): the kernel taps of every
 * antenna, gathered per grid cell).  No device work: usable without a GPU, for
 * verification tools.  cfg must select the fused float32 path (EPIC_FP32, no
 * EPIC_FLAG_STAGED).  out receives, as epic_set_antennas uploads it,
 *   uint32 [n_chan][1 + L][NT][2]:
 *     row 0, word 0: the line thread t transforms in the row pass, p << 16 | j
 *                    (int32 -1: none); word 1: bits 0-23 the line of the
 *                    second row pass of the wide block (below; 0xFFFFFF:
 *                    none), bits 24-31 the steps thread t's wave runs (1..255;
 *                    its later steps are padding; 0: all L);
 *     rows 1..L:     steps {LDS byte offset of the cell, relative to the grid
 *                    base, << 15 | LDS byte offset of E'[p = 0][a] (a multiple
 *                    of 8), bit 0 set on a cell's last entry; float32 weight}.
 * words: in, the capacity of out in uint32 (0 to query); out, the words needed.
 * layout: out, int32 [10] = {NT, L, row stride, polarisation stride, grid
 * base, E' polarisation stride, row order, transposed, block rows, block
 * columns}, strides and base in float2 units; row order 1: aperture row j is
 * stored at physical row 8 (j >> 3) + 2 (j & 3) + ((j >> 2) & 1) (headers and
 * cell offsets use physical rows), 0: at row j.  The aperture block is
 * N/2 x N/2 cells, or at N = 64, when some channel's taps do not fit that,
 * the wide block of 32, 40 or 48 rows by 48 columns: the narrower of the
 * taps' two extents (over all channels) lies along its rows, so with
 * transposed = 1 the programs grid each tap at (column, row) swapped and the
 * kernels image the transposed aperture (their results are transposed back).
 * Its rows fill one row pass of the 8 waves or more: at P = 2 the waves
 * 0-3 (48 rows) or 0 and 1 (40 rows) run two row passes and the others one;
 * at P = 1 the first rows / 8 waves run one and the others none.  The image
 * and its gradient run the wide kernels.
 * Errors: EPIC_E_INVALID (null pointer, bad configuration or geometry),
 * EPIC_E_OFFGRID, EPIC_E_UNSUPPORTED (no fused kernel for cfg, or a channel's
 * taps do not fit the block), EPIC_E_NOMEM (capacity too small;
 * *words holds the size).  Messages: epic_last_error(NULL). */
epic_status epic_gridding_program(const epic_config *cfg, const double *xy_m,
                                  const double *freq_hz, uint32_t *out, int64_t *words,
                                  int32_t *layout);

/* Accumulate polarised images over n_time samples (Sec. 2.1 Eq. (5), Sec. 3.2).
 *   efield: device uint8 [n_time][n_chan][n_pol][n_ant] (4+4-bit samples);
 *   gains:  device complex64 [n_chan][n_pol][n_ant], e' = gain * e;
 *   image:  device complex128 [n_chan][n_prod][N][N] (n_prod = 4 or 1),
 *           fftshifted; reset != 0 overwrites it, reset == 0 adds to it, so an
 *           integration can be split over several calls.
 * XX and YY are written with a zero imaginary part (reset != 0) or have their
 * imaginary part left unchanged (reset == 0).  Accumulation is float64;
 * the per-sample transform is float32 (EPIC_FP32) or split float16 / bfloat16
 * matrix products with float32 accumulation (EPIC_SPLIT_*).  Allocates nothing.
 * With EPIC_FLAG_REMOVE_AUTOS (Sec. 3.2 and Fig. 2: the optional removal of
 * the zero-spacing power, done after squaring and accumulation) the call then
 * subtracts the a = b terms of the visibility form of the image,
 *   sum_a V_PQ[a] |b_a(k)|^2,  V_PQ[a] = g_P conj(g_Q) sum_t e_P[t,a] conj(e_Q[t,a]),
 * b_a(k) the transform of antenna a's kernel taps: the integer sums are exact
 * and the rest is float64.  It adds two passes: one more read of efield and a
 * read-modify-write of image.  Only the samples of this call are removed, so
 * split integrations stay consistent; a call takes at most 2^24 - 1 samples
 * with the flag (more: EPIC_E_UNSUPPORTED).
 * Errors: EPIC_E_STATE (no antennas), EPIC_E_INVALID (null pointer,
 * n_time <= 0), EPIC_E_UNSUPPORTED, EPIC_E_LAUNCH. */
epic_status epic_image_accumulate(epic_ctx *ctx, const uint8_t *efield, int64_t n_time,
                                  const float *gains, double *image, int32_t reset);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * imaging call as epic_image_accumulate, with the same arguments, ownership,
 * product order and result, but its partial-image slots live in a static
 * device array of the library (96 MiB, held by each device the library runs
 * on until the process ends) instead of the context's workspace.  The call
 * allocates nothing and runs the fused float32 kernels only (grid_n 32, 64
 * and 128 with the taps inside an N/2 x N/2 block, or 3N/4 x 3N/4 at N = 64).
 * The slots need (W + C - 1) * n_prod * N * N * 8 bytes, W the persistent
 * grid (at N = 128: (W + 2C - 1) * n_prod * N * N * 4); larger calls are
 * refused before anything is enqueued.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (any contexts,
 * any streams) race, so serialise them.  Nothing needs clearing between
 * calls (each call writes its slots before it reads them).
 * Errors: as epic_image_accumulate; EPIC_E_UNSUPPORTED for the staged and
 * split paths and for calls whose slots exceed the array; EPIC_E_DEVICE when
 * the array has no address on this device. */
epic_status epic_image_accumulate_noalloc(epic_ctx *ctx, const uint8_t *efield, int64_t n_time,
                                          const float *gains, double *image, int32_t reset);

/* Gradient of a real loss L with respect to the gains, given the gradient of
 * L with respect to the image accumulated by epic_image_accumulate(reset=1)
 * over the same efield and gains.  The paper does not compute this: it leaves
 * calibration of the per-antenna gains as future work (Sec. 6, "EPICal").
 * The call is the exact adjoint (chain rule) of the forward path above:
 * products, the transform of Sec. 2.1 Eq. (5) with the opposite sign, and the
 * gridding of Eq. (4) read back at each antenna's kernel taps.
 *   grad_image: device complex128 like image, holding dL/dRe(I) + i dL/dIm(I);
 *               the imaginary parts for XX and YY are ignored (those products
 *               are real);
 *   grad_gains: device complex64 [n_chan][n_pol][n_ant], overwritten with
 *               dL/dRe(g) + i dL/dIm(g).
 * The per-sample transforms are recomputed, not stored; the reduction over
 * time is float64.  With EPIC_FLAG_REMOVE_AUTOS the loss is that of the image
 * without the autocorrelation terms.  Runs wherever the float32 image runs:
 * the fused kernels (grid_n 32, 64 and 128) or the staged ones
 * (EPIC_FLAG_STAGED, or a channel's taps outside an N/2 x N/2 block).
 * Allocates nothing.  Errors as epic_image_accumulate; EPIC_E_UNSUPPORTED for
 * the split precisions. */
epic_status epic_image_backward(epic_ctx *ctx, const uint8_t *efield, int64_t n_time,
                                const float *gains, const double *grad_image,
                                float *grad_gains);

/* Post-processing of an accumulated image (Sec. 3.2: the imprint of the
 * gridding kernels is known in advance and removed after the fact; Sec. 4.3:
 * pseudo-Stokes images, linear combinations of the linear-polarisation
 * products without leakage correction).
 *   image: device complex128 [n_chan][n_prod][N][N] from epic_image_accumulate;
 *   out:   device float64 [n_chan][4][N][N] = I = XX + YY, Q = XX - YY,
 *          U = XY + YX, V = -i (XY - YX) for n_pol = 2; [n_chan][1][N][N] = XX
 *          for n_pol = 1;
 *   taper_floor < 0: no correction; 0 <= taper_floor <= 1: each plane is
 *          divided by the kernel taper T (epic_kernel_taper) at pixels where T is
 *          at least taper_floor times the channel's maximum, and set to 0 elsewhere.
 * Exact when all antennas share one kernel up to a whole-cell shift (then
 * every product is the point-kernel image times T); otherwise it divides by
 * the antennas' mean kernel power pattern.  Allocates nothing; enqueued on the
 * context's stream.  Errors: EPIC_E_STATE (no antennas), EPIC_E_INVALID (null,
 * taper_floor NaN or above 1), EPIC_E_LAUNCH. */
epic_status epic_postprocess(epic_ctx *ctx, const double *image, double taper_floor, double *out);

/* The kernel taper of the current geometry, T_c(k) = mean over antennas of
 * |b_a(k)|^2 (b_a the transform of antenna a's kernel taps, positive exponent),
 * fftshifted like the image, float64 computed from the kernel weights the
 * imager uses; built by epic_set_antennas.  taper: device float64
 * [n_chan][N][N], overwritten (asynchronously, on the context's stream).
 * Errors: EPIC_E_STATE, EPIC_E_INVALID, EPIC_E_LAUNCH. */
epic_status epic_kernel_taper(epic_ctx *ctx, double *taper);

/* With EPIC_FLAG_TIMING: wait for the last imaging call and report the
 * duration of its main kernel and of the whole call, in milliseconds, measured
 * with HIP events on the context's stream.  Errors: EPIC_E_STATE (no timed
 * call yet or flag not set). */
epic_status epic_last_timing(epic_ctx *ctx, float *main_kernel_ms, float *call_ms);

/* With EPIC_FLAG_TIMING: the main-kernel durations, in milliseconds, of the
 * last n timed calls (imaging and gradient calls alike), oldest first, from
 * HIP events recorded on the context's stream around each call's main kernel
 * (kept for the last 256 calls).  Waits for the last of them only, so a caller
 * can time a run of calls without waiting after each.  Not an operation of
 * the paper (measurement).  main_ms: host float [n].  Errors: EPIC_E_STATE
 * (flag not set, or fewer than n timed calls), EPIC_E_INVALID (n outside
 * 1 .. 256, null pointer). */
epic_status epic_timing_history(epic_ctx *ctx, int32_t n, float *main_ms);

/* With EPIC_FLAG_TIMING and EPIC_FLAG_REMOVE_AUTOS: wait for the last imaging
 * call and report the duration of its autocorrelation-sum kernel (the pass
 * over efield) and of the whole removal (sums, table and subtraction), in
 * milliseconds.  Errors: EPIC_E_STATE (no such call yet). */
epic_status epic_last_autos_timing(epic_ctx *ctx, float *sum_kernel_ms, float *removal_ms);

/* Name of the main kernel the last imaging call launched (static string). */
const char *epic_last_kernel_name(const epic_ctx *ctx);

/* ------------------------------------------------------------------------
 * Front end and streaming ingest (Sec. 3.2 and Fig. 2: the channelised
 * samples are decimated in frequency, then transposed from [Time, Channel,
 * Antenna, Polarisation] to [Time, Channel, Polarisation, Antenna]; Sec. 5.1:
 * a gulp must be processed within about 90 % of the time it spans).
 * ------------------------------------------------------------------------ */

/* Decimate and transpose one gulp on the context's stream (bytes moved, not
 * changed):
 *   raw:    device uint8 [n_time][c_in][n_ant][n_pol], as it arrives;
 *   efield: device uint8 [n_time][n_chan][n_pol][n_ant] (the layout of
 *           epic_image_accumulate), overwritten;
 *   output channel i = input channel c0 + i * c_step, i < n_chan (the
 *   context's channel count).
 * Allocates nothing.  Errors: EPIC_E_INVALID (null pointer, n_time <= 0, a
 * selected channel outside [0, c_in)), EPIC_E_LAUNCH. */
epic_status epic_frontend(epic_ctx *ctx, const uint8_t *raw, int64_t n_time, int32_t c_in,
                          int32_t c0, int32_t c_step, uint8_t *efield);

typedef struct epic_pipeline epic_pipeline;

/* Statistics of the gulps a pipeline has completed (all times in ms). */
typedef struct epic_pipeline_stats {
  int64_t gulps;            /* gulps completed and measured */
  int64_t over_budget;      /* gulps whose processing time exceeded 0.9 * gulp_ms */
  double gulp_ms;           /* time one gulp spans: n_time * sample_s */
  double mean_ms, max_ms;   /* processing time per gulp: from the later of its copy
                               start and the previous gulp's end, to its end */
  double mean_copy_ms;      /* host-to-device copy of one gulp */
  double mean_compute_ms;   /* front end + imaging of one gulp (incl. waiting for
                               the previous gulp) */
} epic_pipeline_stats;

/* Create a double-buffered ingest for ctx: gulps of n_time samples with c_in
 * channels in arrival order, channels c0 + i * c_step imaged (i < n_chan).
 * Allocates two device gulp buffers and one transposed buffer, a copy stream
 * (default priority) and events; sample_s is the duration of one sample in
 * seconds (40e-6 for 25 kHz channels).  With c_step == 1 only the selected
 * sub-band is copied from the host.  The pipeline uses ctx (its stream,
 * tables, flags): destroy the pipeline before the context.
 * Errors: EPIC_E_INVALID (null, n_time <= 0, sample_s not positive, a channel
 * outside [0, c_in)), EPIC_E_NOMEM, EPIC_E_DEVICE; *out is NULL on error and
 * epic_pipeline_last_error(NULL) says why. */
epic_status epic_pipeline_create(epic_ctx *ctx, int64_t n_time, int32_t c_in, int32_t c0,
                                 int32_t c_step, double sample_s, epic_pipeline **out);

/* Enqueue one gulp and return: the copy of host_raw (host uint8
 * [n_time][c_in][n_ant][n_pol]; pinned memory, e.g. from hipHostMalloc, lets
 * the copy overlap the imaging of the previous gulp) starts once the buffer it
 * fills is free, then the front end and epic_image_accumulate(gains, image,
 * reset) run on the context's stream.  host_raw must stay valid and unchanged
 * until the gulp's copy has finished (at the latest when epic_pipeline_report
 * or epic_pipeline_destroy returns).  After kRing = 64 gulps a push waits for
 * the gulp 63 places earlier to finish (bounded run-ahead).
 * Errors: EPIC_E_INVALID, EPIC_E_STATE (no antennas), EPIC_E_UNSUPPORTED /
 * EPIC_E_LAUNCH from the imaging call, EPIC_E_DEVICE. */
epic_status epic_pipeline_push(epic_pipeline *p, const uint8_t *host_raw, const float *gains,
                               double *image, int32_t reset);

/* Wait for every pushed gulp and report the statistics. */
epic_status epic_pipeline_report(epic_pipeline *p, epic_pipeline_stats *out);

/* Wait for the pipeline's work and free it (not the context). */
void epic_pipeline_destroy(epic_pipeline *p);

/* Message of the last failed call on p (NULL: of the last failed create). */
const char *epic_pipeline_last_error(const epic_pipeline *p);

/* ------------------------------------------------------------------------
 * Heterogeneous batch: n_blocks independent configurations (different grid
 * sizes, antenna and channel counts) imaged together.  The paper sizes its
 * gulp, channel count and grid by measurement for its GPUs (Sec. 5.1) and
 * leaves optimisation as future work (Sec. 6); the batch makes that sizing a
 * tuning step.  Every block gets its own context.  Blocks that run the fused
 * float32 kernels (no autocorrelation removal) and share the grid side,
 * polarisation count, sample bytes per thread and aperture class are imaged
 * by one persistent launch that walks all their channels as one (channel,
 * time) list -- one launch per such group (at most 8 blocks each), plus one
 * reduction writing the group's images; any other block runs through its own
 * context.  A batch call forks from hip_stream to one stream per launch and
 * joins back.  All pointer-array arguments are host arrays of n_blocks device
 * pointers, laid out per block exactly as for epic_image_accumulate; n_time
 * is common to all blocks.
 * ------------------------------------------------------------------------ */
typedef struct epic_batch epic_batch;

/* Create the batch and one context per block (configs copied).  Errors as
 * epic_init; on error *out is NULL and epic_batch_last_error(NULL) says which
 * block failed. */
epic_status epic_batch_create(const epic_config *cfgs, int32_t n_blocks, int device,
                              void *hip_stream, epic_batch **out);

/* epic_set_antennas for one block.  Once every block has its antennas the
 * batch cuts its launches and allocates the grouped launches' workspace (a
 * later call rebuilds them, and drops a captured graph). */
epic_status epic_batch_set_antennas(epic_batch *b, int32_t block, const double *xy_m,
                                    const double *freq_hz);

/* The images of every block, as epic_image_accumulate would give them
 * (the same tolerance; grouped blocks sum in another order), ordered after
 * earlier work on hip_stream; later work on hip_stream waits for all blocks.
 * Allocates nothing.  Errors: EPIC_E_STATE (a block has no antennas), as
 * epic_image_accumulate otherwise. */
epic_status epic_batch_accumulate(epic_batch *b, const uint8_t *const *efields, int64_t n_time,
                                  const float *const *gains, double *const *images,
                                  int32_t reset);

/* Capture the same fork-join sequence into a HIP graph (replacing any earlier
 * one).  Nothing runs until epic_batch_replay; every replay reads and writes
 * the buffers given here.  The library's kernels clear their own workspace,
 * so the graph contains kernel nodes only. */
epic_status epic_batch_capture(epic_batch *b, const uint8_t *const *efields, int64_t n_time,
                               const float *const *gains, double *const *images,
                               int32_t reset);

/* Launch the captured graph on hip_stream.  Errors: EPIC_E_STATE (none). */
epic_status epic_batch_replay(epic_batch *b);

/* Autotune the launch shapes on these inputs -- for a grouped launch its
 * persistent grid size (samples per workgroup), its team size (time chunk:
 * the workgroups that share each channel's samples), the float32 block
 * length before a float64 flush (128 or 64 samples) and whether a team's
 * workgroups are dealt to one XCD; for a single block its context's
 * grid or staged sample batch -- and whether the launches run concurrently
 * or one after another: runs and times each launch alone and the whole
 * batch (overwriting images), or, when
 * cache_path names a file holding a plan for the same device, block shapes
 * and n_time, loads it.  A measured plan is appended to cache_path (if not
 * NULL).  *measured = 1 when timings were taken, 0 when the cache was used.
 * Synchronises hip_stream.  Call it before epic_batch_capture. */
epic_status epic_batch_tune(epic_batch *b, const uint8_t *const *efields, int64_t n_time,
                            const float *const *gains, double *const *images,
                            const char *cache_path, int32_t *measured);

/* The launch shape in force for a block: grid = persistent workgroups of the
 * fused kernel (0 if the block runs the staged kernels), staged_batch =
 * samples per staged pass (0 if fused). */
epic_status epic_batch_plan(const epic_batch *b, int32_t block, int32_t *grid,
                            int32_t *staged_batch);

/* Which launch images a block and its tuned shape: launch = index of the
 * launch, n_blocks = blocks that launch walks (0: the block runs alone
 * through its context), team = workgroups that share each channel's samples
 * (each taking T / team of them; 0: chosen from T), kblock = samples summed
 * in float32 before a float64 flush, xcd = 1 if a team's workgroups share an
 * XCD.  Errors: EPIC_E_INVALID (no such block), EPIC_E_STATE (launches not
 * cut yet). */
epic_status epic_batch_launch_plan(const epic_batch *b, int32_t block, int32_t *launch,
                                   int32_t *n_blocks, int32_t *team, int32_t *kblock,
                                   int32_t *xcd);

/* Set a grouped launch's shape by hand (as epic_batch_tune would): grid =
 * persistent workgroups (0: as many as stay resident; larger values are
 * capped there, and rounded down to whole teams), team = 0 (from T), 1, 2, 4
 * or 8, kblock = float32 block length in samples (1 .. 128), xcd != 0: a
 * team's workgroups on one XCD.  Applies to later accumulate and capture
 * calls.  Errors: EPIC_E_INVALID (no such launch, bad values),
 * EPIC_E_UNSUPPORTED (a block running alone). */
epic_status epic_batch_set_launch(epic_batch *b, int32_t launch, int32_t grid, int32_t team,
                                  int32_t kblock, int32_t xcd);

/* 1 if the launches of b run one after another (each persistent launch with
 * the whole GPU), 0 if they run concurrently on their own streams; set by
 * epic_batch_tune (default 0) and applied to accumulate and capture. */
int32_t epic_batch_serial(const epic_batch *b);

/* Choose the mode by hand (serial != 0: one after another); applies to later
 * accumulate and capture calls.  Errors: EPIC_E_INVALID (b NULL). */
epic_status epic_batch_set_serial(epic_batch *b, int32_t serial);

/* Free the batch, its graph, streams and contexts. */
void epic_batch_destroy(epic_batch *b);

/* Message of the last failed batch call (NULL: the last failed create). */
const char *epic_batch_last_error(const epic_batch *b);

/* Free the context and its library-owned memory (waits for its stream).
 * Resource management only; no operation of the paper. */
void epic_destroy(epic_ctx *ctx);

/* Message of the last failed call on ctx, valid until the next call on ctx.
 * With ctx == NULL: the message of the last failed epic_init in this thread.
 * Error reporting only; no operation of the paper.  Never NULL ("" before
 * any failure). */
const char *epic_last_error(const epic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* EPIC_H */
