/*
 * pdc.h -- C ABI of libpdc: pixel-detector correction and photon finding on
 * one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Blaj, Chang and Kenney, "Ultrafast Processing of Pixel
 * Detector Data with Machine Learning Frameworks" (AIP Conf. Proc. 2054,
 * 060077, 2019; arXiv:1903.06838):
 *   - a minibatch of N raw frames is an N x H x W tensor of 14-bit ADC values
 *     (Novel Tensorflow Models, Dark and Gain; Fig. b "Raw");
 *   - Frames1 = (Raw - Dark) / Gain per pixel (Fig. b);
 *   - common mode: a per-bank offset is estimated and subtracted, giving
 *     Frames2 (Common Mode section, Fig. c; the section allows row, column or
 *     block common modes; here a bank is one row of bank_cols contiguous
 *     columns of a tile and the estimate is the bank's lower median);
 *   - photon finding: a photon's charge is summed from its cloud and placed on
 *     the cloud's highest pixel (Photon Charge Summing section, Fig. e), with
 *     pixels within noise zeroed (Photon Subpixel Resolution section);
 *   - photon counting: charge / single-photon signal, rounded to the nearest
 *     integer (Photon Charge Summing section);
 *   - summarization into sparse photon lists (Summarization section).
 *
 * Exact contract, per frame f, tile t, row r, column c, pixel
 * p = (t*rows + r)*cols + c, all arithmetic IEEE binary32 round-to-nearest-even
 * with every operation rounded on its own:
 *   adc = raw & 0x3FFF;  u = ((float)adc - pedestal[p]) * k[p],  k[p] = 1.0f / gain[p]
 *   m   = element of rank (B-1)/2 (0-based, ascending) of the bank's B values u
 *   v   = u - m                                                  (Frames2)
 *   hit at p iff v[p] > T_seed and, for every neighbour q of the 3x3 window
 *   inside the same tile, v[p] > v[q] or (v[p] == v[q] and p < q)
 *   charge = sum over the in-tile 3x3 window, rows top to bottom, columns left
 *            to right, from +0.0f, of (v[j] > T_nb ? v[j] : 0.0f)
 *   nphot  = rint(charge / photon_adu) (ties to even), saturating at 2^32-1
 *   T_seed = n_seed * sigma,  T_nb = n_nb * sigma  (formed in binary32)
 *
 * Threading: a context is used by one host thread at a time.  All functions
 * return a pdc_status; no C++ exception crosses this boundary; on a negative
 * status the output parameters are left untouched.
 */
#ifndef PDC_H
#define PDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pdc_status;

#define PDC_OK 0
#define PDC_WARN_TRUNCATED 1 /* soft: more hits than the destination holds */
#define PDC_EINVAL (-1)      /* invalid argument, geometry, plane value or parameter */
#define PDC_ENOMEM (-2)      /* device or host memory exhausted */
#define PDC_EDEVICE (-3)     /* HIP runtime error, no device, or a kernel-reported fault */
#define PDC_ESTATE (-4)      /* unknown or released detector / batch, wrong call order */

/* Keep Frames2 (float32 [N][T][H][W]) of a batch for pdc_get_corrected. */
#define PDC_KEEP_CORRECTED 1u
/* Keep each frame's common-mode values of a batch (the bank medians, or the
 * thresholded mean's stage values): pdc_capture_patches then forms patches
 * from the frames without Frames2.  They take
 * n_frames * n_tiles * rows * (cols / bank_cols) floats of device memory. */
#define PDC_KEEP_MEDIANS 2u

typedef struct pdc_ctx pdc_ctx;
typedef struct pdc_graph pdc_graph;

/* Detector geometry.  A frame is n_tiles tiles of rows x cols pixels (tiles are
 * separate sensors: 3x3 windows stop at tile edges).  Common-mode banks are
 * one row of bank_cols contiguous columns; cols % bank_cols == 0.
 * Limits: 1 <= n_tiles, rows; 1 <= bank_cols <= cols <= 2048; bank_cols <= 1024;
 * n_tiles*rows*cols < 2^31.  gain_mode is a PDC_GAIN_* value. */
typedef struct {
    int32_t n_tiles;
    int32_t rows;
    int32_t cols;
    int32_t bank_cols;
    int32_t gain_mode;
} pdc_geometry;

/* Gain ranges (Dark and Gain section, Fig. b: several darks and gains for
 * auto-ranging detectors).  PDC_GAIN_SINGLE: one range, bits 14-15 of a raw
 * word ignored.  Otherwise bits 14-15 report the pixel's range and the
 * calibration holds one pedestal and one gain plane per range (3 ranges):
 *   PDC_GAIN_EPIX10K:  codes 0, 1, 2 -> ranges 0, 1, 2; code 3 invalid
 *   PDC_GAIN_JUNGFRAU: codes 0, 1, 3 -> ranges 0, 1, 2; code 2 invalid
 * u = ((float)adc - pedestal[r][p]) * k[r][p] with r the reported range.  A
 * pixel with an invalid code has no u: it takes no part in the common mode
 * (the median is then the element of rank (n-1)/2 of the bank's n valid
 * values, m = 0 when n = 0; the thresholded mean does not count it as noise,
 * its guard still uses the region's size), its Frames2 value is +0.0 (it
 * never seeds and adds nothing to a charge), and it is counted per frame
 * (pdc_get_invalid_counts).  One threshold pair applies to every range. */
#define PDC_GAIN_SINGLE 0
#define PDC_GAIN_EPIX10K 1
#define PDC_GAIN_JUNGFRAU 2

/* Common-mode estimator (cm_mode of pdc_params).
 * PDC_CM_MEDIAN: m = the bank's lower median, v = u - m (the contract above).
 * PDC_CM_BANK_MEAN, PDC_CM_TILE_MEAN: the thresholded mean of Fig. c over
 *   each bank or each tile (for a one-tile detector, the frame), applied
 *   cm_stages times in sequence (the stacked stages of the performance
 *   model).  Stage s, on the current values v of a region of P pixels:
 *     noise pixels: v < T_cm = n_cm * sigma;  N0 = their number;
 *     S = their binary32 sum: pixel i of the region (raster order within the
 *       region) is added to partial sum i mod Q (Q = 64 for a bank, 256 for
 *       a tile), partials start at +0.0 and take their pixels in increasing
 *       i, and the Q partials are added in a balanced binary tree (pairs
 *       (0,1), (2,3), ... first);
 *     CM_s = S / max((float)N0, sqrtf((float)P));  v = v - CM_s.
 *   Frames2 is v after the last stage; hit finding is unchanged.  Each
 *   operation is one binary32 operation rounded to nearest even. */
#define PDC_CM_MEDIAN 0
#define PDC_CM_BANK_MEAN 1
#define PDC_CM_TILE_MEAN 2

/* Thresholds and photon scale (Results, Accuracy: the two noise thresholds,
 * typically 3 to 5 sigma).  sigma > 0, n_seed >= 0, n_nb >= 0 finite, with
 * T_nb <= T_seed; photon_adu in [2^-24, 2^24]; flags is 0 or PDC_KEEP_CORRECTED.
 * cm_mode is a PDC_CM_* value; with a mean mode, 1 <= cm_stages <= 3 and
 * n_cm >= 0 finite (the segmentation threshold of Fig. c, typically 3);
 * both are ignored by PDC_CM_MEDIAN. */
typedef struct {
    float sigma;
    float n_seed;
    float n_nb;
    float photon_adu;
    uint32_t flags;
    int32_t cm_mode;
    int32_t cm_stages;
    float n_cm;
} pdc_params;

/* One photon hit (16 bytes).  frame is relative to the batch. */
typedef struct {
    uint32_t frame;
    uint32_t pixel;  /* (tile*rows + row)*cols + col */
    float charge;    /* masked 3x3 charge sum, ADU after gain correction */
    uint32_t nphot;  /* rint(charge / photon_adu) */
} pdc_hit;

/* Static text for a status code. */
const char *pdc_strerror(pdc_status status);

/* Message of the last failing call on ctx (empty string if none). */
const char *pdc_last_error(const pdc_ctx *ctx);

/* Open a context on HIP device `device`.  The library owns every device buffer
 * it allocates; they are freed by pdc_destroy.  EDEVICE if the device does not
 * exist or is not gfx950.  Test hooks read from the environment here:
 * PDC_FORCE_GENERAL=1 runs every batch on the general kernel;
 * PDC_DEBUG_TIGHT_POOL=1 sizes a batch's first hit staging to hit_capacity
 * alone (no per-workgroup slack), so a small capacity forces the staging
 * overflow and its exact recomputation. */
pdc_status pdc_create(int32_t device, pdc_ctx **out);

/* Wait for outstanding work, free everything.  NULL is accepted. */
pdc_status pdc_destroy(pdc_ctx *ctx);

/* Host-only validation of what pdc_calibrate would accept (no device use).
 * pedestal and gain are host arrays float32 [n_ranges][n_tiles][rows][cols]
 * (n_ranges = 1 for PDC_GAIN_SINGLE, else 3).  Each
 * pedestal must be finite with |x| <= 2^24 and (x == 0 or |x| >= 2^-64); each
 * gain finite in [2^-24, 2^24].  These bounds keep every intermediate finite,
 * normal or +0 (no -0, no subnormal, no NaN).  EINVAL names the first
 * offending value in the status text of the context-free check. */
pdc_status pdc_check_calibration(const pdc_geometry *geom, const float *pedestal,
                                 const float *gain, const pdc_params *params);

/* Dark and gain calibration (Fig. b weights "Dark" and "Gain", 1 x H x W).
 * Copies the host planes into resident device memory (the caller keeps its
 * arrays), forms k = 1.0f / gain on the host, T_seed and T_nb, and returns a
 * detector id in *det_out.  EINVAL on invalid geometry, planes or params. */
pdc_status pdc_calibrate(pdc_ctx *ctx, const pdc_geometry *geom, const float *pedestal,
                         const float *gain, const pdc_params *params, int32_t *det_out);

/* Free a detector's planes after its pending batches complete. */
pdc_status pdc_release_detector(pdc_ctx *ctx, int32_t det);

/* Enqueue the whole pipeline on a batch of frames: the raw minibatch
 * N x H x W x 1 of the Dark and Gain section goes through dark and gain
 * (Fig. b), common mode (Fig. c) and photon finding, charge summing and
 * counting (Fig. e, Photon Charge Summing section), and ends in the sparse
 * photon lists of the Summarization section.
 * frames_dev: DEVICE pointer to uint16 [n_frames][n_tiles][rows][cols], raw
 *   ADC words (bits 14-15 ignored); borrowed, it must stay valid and unchanged
 *   until pdc_get_hits or pdc_release_batch of this batch returns.
 * hit_capacity: expected upper bound on hits in the batch; buffers are sized
 *   from it.  If the batch holds more, pdc_get_hits recomputes it with exact
 *   sizes, so the result is always complete.
 * hip_stream: a hipStream_t of the context's device, or NULL for the
 *   context's own stream.  That stream is non-blocking: it is not ordered
 *   with other streams (the HIP null stream included), so frames written on
 *   another stream must be complete before the call (synchronize, or pass
 *   the producing stream).  The call returns once the work is enqueued.
 * *batch_out: id for pdc_get_hits / pdc_get_corrected / pdc_release_batch.
 * n_frames may be 0.  Results of a frame do not depend on the other frames of
 * the batch.  EINVAL on a bad pointer or size, ESTATE on an unknown detector,
 * ENOMEM if device buffers cannot be allocated. */
pdc_status pdc_process_frames(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev,
                              uint64_t n_frames, uint64_t hit_capacity, void *hip_stream,
                              uint64_t *batch_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * results of pdc_process_frames + pdc_get_hits (device destination) +
 * pdc_release_batch in one synchronous call that allocates nothing.  Every
 * intermediate buffer (batch state, per-unit and per-frame arrays, the
 * common-mode values of the mean modes, the hit staging pool) lies in a
 * static device array of PDC_STATIC_SCRATCH_BYTES that each GPU the library
 * runs on holds until the process ends; its address is taken per device by
 * pdc_create.  All calls on one GPU share that array and it keeps the last
 * call's contents: calls that overlap on one GPU (from several threads or
 * contexts, on any streams) race, so the caller serializes them.
 * frames_dev: DEVICE uint16 [n_frames][n_tiles][rows][cols] as for
 *   pdc_process_frames.
 * hits_dev: DEVICE records, room for hits_capacity (the first
 *   min(total, hits_capacity) hits in (frame, pixel) order are written).
 * frame_hits_dev (uint32 [n_frames]) and frame_photons_dev (uint64
 *   [n_frames]): DEVICE per-frame counts and photon totals.
 * *n_hits_total (may be NULL): the true total.
 * Work is enqueued on hip_stream (NULL: the context's stream) and the call
 * returns when it has finished.  PDC_WARN_TRUNCATED when the total exceeds
 * hits_capacity.  EINVAL when n_frames needs more per-unit arrays and
 * staging room than the scratch holds (an ePix100 or CSPAD detector fits
 * several hundred frames per call), or for a PDC_KEEP_CORRECTED detector
 * (Frames2 needs a buffer of its own); ENOMEM when the batch's hits
 * overflow the scratch's staging pool (the outputs are then unspecified);
 * ESTATE for an unknown detector. */
#define PDC_STATIC_SCRATCH_BYTES (64ull << 20)
pdc_status pdc_process_frames_static(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                                     pdc_hit *hits_dev, uint64_t hits_capacity, uint32_t *frame_hits_dev,
                                     uint64_t *frame_photons_dev, void *hip_stream, uint64_t *n_hits_total);

/* Batches of several detectors (mixed geometries, gain modes and
 * common-mode settings) enqueued at once: item i becomes batch batch_out[i]
 * exactly as pdc_process_frames would make it, on one of up to 8 internal
 * streams forked from hip_stream (NULL: the context's stream) and joined back
 * into it, so the detectors' kernels may overlap and work enqueued later on
 * hip_stream waits for all of them.  When there are 2 to 8 items and every
 * one takes the persistent kernel with the median common mode, keeping
 * neither Frames2 nor common-mode values, their frame kernels are one launch
 * over the (detector, strip, frame group) work items of all of them, each
 * workgroup running the body compiled for its detector's lane layout and gain
 * mode (the Dark and Gain section's several darks and gains in one pass);
 * the work before and after it stays on the batches' streams.  Otherwise, or
 * with PDC_MIX_FORKED=1 in the environment at pdc_create, each batch has
 * launches of its own.  Each batch's share of the launch is the whole chip's
 * worth of frame groups (PDC_MIX_SHARE=1 at pdc_create sizes each for the
 * share of the chip its pixels are of the whole instead).  1 <= n_items <= 64.
 * On an error no batch is left outstanding. */
typedef struct {
    int32_t det;
    const uint16_t *frames_dev;  /* DEVICE [n_frames][n_tiles][rows][cols], borrowed as above */
    uint64_t n_frames;
    uint64_t hit_capacity;
} pdc_mixed_item;

pdc_status pdc_process_mixed(pdc_ctx *ctx, const pdc_mixed_item *items, int32_t n_items, void *hip_stream,
                             uint64_t *batch_out);

/* Tile-shape autotuner: times the persistent kernel on n_frames of the
 * caller's frames (DEVICE, as for pdc_process_frames) with its frame-group
 * count at 1, 2 and 4 times the smallest count that fills whole rounds of the
 * chip, and keeps the fastest for the detector's later batches (results do not
 * depend on it).  *mult_out (may be NULL) receives the multiplier, ms_out
 * (host float[3], may be NULL) the frame-kernel times.  Synchronous; runs 9
 * batches. */
pdc_status pdc_autotune(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                        uint64_t hit_capacity, void *hip_stream, int32_t *mult_out, float *ms_out);

/* Strip-height autotuner: the persistent kernel with at most R own rows per
 * strip, R the most its lane layout holds and 4 and 8 fewer (those of at
 * least 4 rows), each timed with pdc_autotune's three frame-group counts on
 * the caller's frames; the detector keeps the fastest (strip rows, frame
 * groups) for its later batches (results do not depend on them).  *rows_out
 * and *mult_out (may be NULL) receive the choice, ms_out (host float[9], may
 * be NULL) the frame-kernel times, row r of 3 for the r-th strip height,
 * *n_tried (may be NULL) the strip heights timed.  ESTATE while the detector
 * has outstanding batches or graphs (they hold its strip plan) or does not
 * take the persistent kernel.  Synchronous; runs 9 batches per height. */
pdc_status pdc_autotune_strips(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                               uint64_t hit_capacity, void *hip_stream, int32_t *rows_out, int32_t *mult_out,
                               float *ms_out, int32_t *n_tried);

/* Wait for the batch and copy its results (Summarization section: lists of
 * sparse photons, each with its position, energy and photon count; per-frame
 * photon-counting totals), hits in (frame, pixel) order.
 * dst: room for dst_capacity records, in host memory (dst_is_device = 0) or
 *   device memory of the context's device (dst_is_device = 1); may be NULL
 *   when dst_capacity is 0.  The first min(total, dst_capacity) hits are
 *   written; *n_hits_total (may be NULL) receives the true total.
 * per_frame_hits (uint32 [n_frames]) and per_frame_photons (uint64
 *   [n_frames]): host arrays or NULL.
 * Returns PDC_WARN_TRUNCATED when total > dst_capacity, else PDC_OK.  A
 * batch whose hits outgrew the buffers sized from hit_capacity is recomputed
 * here with exact sizes first, so the total and the lists are always
 * complete.  The batch stays alive until pdc_release_batch (it can be read
 * again, with other destinations).  ESTATE for an unknown batch. */
pdc_status pdc_get_hits(pdc_ctx *ctx, uint64_t batch, pdc_hit *dst, uint64_t dst_capacity,
                        int32_t dst_is_device, uint64_t *n_hits_total, uint32_t *per_frame_hits,
                        uint64_t *per_frame_photons);

/* Frames2 of a batch processed with PDC_KEEP_CORRECTED: float32
 * [n_frames][n_tiles][rows][cols] into host or device memory.  ESTATE if the
 * flag was not set. */
pdc_status pdc_get_corrected(pdc_ctx *ctx, uint64_t batch, float *dst, int32_t dst_is_device);

/* Per-frame number of pixels with an invalid gain code (uint32 [n_frames],
 * host), zeros for a single-range detector.  Waits for the batch. */
pdc_status pdc_get_invalid_counts(pdc_ctx *ctx, uint64_t batch, uint32_t *per_frame_invalid);

/* Wait for the batch and return its buffers to the context for reuse. */
pdc_status pdc_release_batch(pdc_ctx *ctx, uint64_t batch);

/* Device memory, in bytes, of the buffers pdc_process_frames uses for a batch
 * of n_frames frames with this hit_capacity on detector det (staging pool,
 * hit list, per-unit and per-frame records, and Frames2 or the kept
 * common-mode values when the detector's flags ask for them).  Buffers are
 * reused from batch to batch, so this is what a batch needs, not what a call
 * allocates.  Admission control of a serving loop charges it.  ESTATE for an
 * unknown detector; EINVAL for n_frames > 2^31 or a NULL pointer. */
pdc_status pdc_batch_bytes(pdc_ctx *ctx, int32_t det, uint64_t n_frames, uint64_t hit_capacity,
                           uint64_t *bytes);

/* Timing of a finished batch from HIP events recorded on its stream:
 * *main_ms = the fused frame kernel alone, *total_ms = every kernel of the
 * batch (common-mode pass of the mean modes, frame kernel, scans, hit
 * scatter).  Either pointer may be NULL. */
pdc_status pdc_batch_timing(pdc_ctx *ctx, uint64_t batch, float *main_ms, float *total_ms);

/* Measurement aid: a plain streaming read of bytes (a nonzero multiple of 16)
 * at the DEVICE pointer src_dev (16-byte aligned), each byte once, on
 * hip_stream (NULL: the context's stream); *ms_out (may be NULL) receives its
 * duration from HIP events around the kernel on that stream.  bytes / ms is
 * the HBM read bandwidth a kernel can reach on this device, the reference
 * beside the frame kernel's fraction of the published peak.  Synchronous;
 * allocates 4 bytes and two events for the call.  EINVAL on a bad pointer or
 * size. */
pdc_status pdc_stream_read(pdc_ctx *ctx, const void *src_dev, uint64_t bytes, void *hip_stream, float *ms_out);

/* HIP graph of one batch (the pipeline of the Fig. a chain, as
 * pdc_process_frames enqueues it), for loops that process the same number of
 * frames from the same device buffer over and over: the kernels are captured
 * once and each launch replays them with one call.
 * pdc_graph_create captures a batch of n_frames (>= 1) frames at frames_dev
 * for detector det, with buffers sized from hit_capacity, and returns the graph
 * in *out.  The graph owns its device buffers and holds the detector (which
 * pdc_release_detector frees only after pdc_graph_destroy).  The captured
 * nodes are kernels only (no memset or copy nodes).
 * pdc_graph_launch enqueues the graph on hip_stream (NULL: the context's
 * stream) and returns a batch id in *batch_out (one per item for a mixed
 * graph, below) that the batch calls
 * (pdc_get_hits, pdc_get_corrected, summaries, pdc_release_batch, ...) take
 * as for pdc_process_frames.  The frames are read from frames_dev when the
 * graph runs: write the next frames there, ordered before the launch on
 * hip_stream, and leave them unchanged until the batch is released.  One batch
 * per graph at a time: ESTATE until the previous one is released.  A batch that
 * needs recomputing from the start (staging overflow beyond hit_capacity, or
 * no general-kernel plan for overflowing seed lists) is moved to buffers of its
 * own, so results stay exact and the graph stays valid.  Batch timing reports
 * the whole graph as main_ms.
 * pdc_graph_destroy frees the graph; ESTATE while its batch is outstanding.
 * pdc_destroy frees graphs still alive.  A graph is used from its context's
 * thread, as the context is. */
pdc_status pdc_graph_create(pdc_ctx *ctx, int32_t det, const uint16_t *frames_dev, uint64_t n_frames,
                            uint64_t hit_capacity, pdc_graph **out);
pdc_status pdc_graph_launch(pdc_graph *graph, void *hip_stream, uint64_t *batch_out);
pdc_status pdc_graph_destroy(pdc_graph *graph);

/* One graph over batches of several detectors (mixed geometries, gain modes
 * and common-mode settings), captured as pdc_process_mixed enqueues them:
 * item i's kernels run on one of up to 8 internal streams forked inside the
 * graph and joined back, so one pdc_graph_launch replays all of them and
 * returns n_items batch ids in batch_out[0..n_items) (item order).  Each
 * item's frames_dev is read at replay time as for pdc_graph_create.  All of
 * the graph's batches must be released before the next launch.  1 <= n_items
 * <= 64; pdc_graph_items returns a graph's item count (0 for NULL). */
pdc_status pdc_graph_create_mixed(pdc_ctx *ctx, const pdc_mixed_item *items, int32_t n_items, pdc_graph **out);
int32_t pdc_graph_items(const pdc_graph *graph);

/* ------------------------------------------------------------------------
 * Subpixel position of hits (Photon Subpixel Resolution section and its
 * figure comparing centroid and learned positions).
 *
 * A patch is the 5x5 block of Frames2 values centred on a hit, float32
 * [5][5] row-major (rows top to bottom), zero outside the hit's tile.  A
 * position is (dy, dx) in pixel pitches relative to the centre of the hit
 * pixel.  Patch, position and table arguments named *_dev are DEVICE pointers
 * of the context's device; hip_stream is a hipStream_t of that device or NULL
 * for the context's (non-blocking) stream, which is not ordered with other
 * streams: inputs and outputs touched on another stream must be complete
 * first.  The calls return once the work is enqueued unless stated otherwise.  EINVAL for a NULL pointer with n > 0 or an out-of-range
 * scalar.
 * ------------------------------------------------------------------------ */

/* Patches of the first min(total, capacity) hits of a batch, in hit-list
 * order, into patches_dev float32 [capacity][25]; *n_out (may be NULL)
 * receives the number written.  The batch was processed with
 * PDC_KEEP_CORRECTED (the patch is copied from Frames2) or with
 * PDC_KEEP_MEDIANS, and then the frames given to pdc_process_frames must
 * still hold the batch's frames: each patch value is formed from the raw
 * word, the calibration and the kept common-mode values by the operations
 * of Frames2, so it is the same binary32 value.  Synchronous.  ESTATE for an
 * unknown batch or one with neither flag. */
pdc_status pdc_capture_patches(pdc_ctx *ctx, uint64_t batch, float *patches_dev, uint64_t capacity,
                               uint64_t *n_out);

/* The learned estimator's inputs of the same hits, 64 bytes per hit instead
 * of 100: inputs_dev uint16 [capacity][PDC_MLP_INPUT_WORDS], word j < 25 of a
 * hit the bfloat16 (round to nearest even) of fl(v_j * fl(1 / photon_adu)) for
 * patch value v_j, words 25..31 zero.  These are the values pdc_mlp_infer
 * forms from a float32 patch, so pdc_mlp_infer_inputs on them gives the same
 * positions.  photon_adu in [2^-24, 2^24]; otherwise as pdc_capture_patches. */
#define PDC_MLP_INPUT_WORDS 32
pdc_status pdc_capture_inputs(pdc_ctx *ctx, uint64_t batch, float photon_adu, uint16_t *inputs_dev,
                              uint64_t capacity, uint64_t *n_out);

/* Classical positions of the same hits without patches: the masked 3x3
 * centroid below (eta-corrected when eta_dev is not NULL) of each of the first
 * min(total, capacity) hits, computed from the hit's Frames2 values as
 * pdc_capture_patches forms them, into positions_dev float32 [capacity][2]; the
 * same values as pdc_centroid on the captured patches.  only_implausible != 0:
 * positions_dev already holds positions of these hits (the learned
 * estimator's) and only those that are not finite or outside [-1, 1] in a
 * coordinate are replaced by the classical ones: the runtime fallback.
 * t_nb finite; 1 <= nbins <= 65536 when eta_dev is used.  Synchronous;
 * ESTATE as for pdc_capture_patches. */
pdc_status pdc_capture_centroids(pdc_ctx *ctx, uint64_t batch, float t_nb, const float *eta_dev, int32_t nbins,
                                 float *positions_dev, uint64_t capacity, int32_t only_implausible, uint64_t *n_out);

/* Masked 3x3 centroid of each patch: s = (v > t_nb ? v : 0) over the central
 * 3x3 pixels; dy = sum(s*dr) / sum(s), dx = sum(s*dc) / sum(s), the sums in
 * row-major order from +0.0f, IEEE binary32, (0, 0) when sum(s) == 0.
 * If eta_dev is not NULL (float32 [2][nbins + 1] from pdc_eta_table) each
 * coordinate c is then mapped to CDF(c) - 1/2, linear between the table's
 * edges (eta correction: the linearization of centroids into positions).
 * out_dev: float32 [n][2].  t_nb finite; 1 <= nbins <= 65536 when eta_dev is
 * used. */
pdc_status pdc_centroid(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float t_nb,
                        const float *eta_dev, int32_t nbins, float *out_dev, void *hip_stream);

/* Eta table from n patches of hits with impact points uniform over the pixel:
 * per axis, the empirical CDF of the centroid coordinate at the nbins + 1
 * edges of nbins equal bins over [-1, 1] (coordinates are clamped to the
 * range).  table_dev: float32 [2][nbins + 1]; workspace_dev: uint32
 * [2 * nbins], scratch of this call.  1 <= nbins <= 65536. */
pdc_status pdc_eta_table(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float t_nb, int32_t nbins,
                         uint32_t *workspace_dev, float *table_dev, void *hip_stream);

/* Learned estimator: a 25-64-64-2 ReLU network on the patch divided by
 * photon_adu, y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3.  Its products
 * take bfloat16 operands (round to nearest even: inputs, activations,
 * back-propagated gradients and a bf16 copy of the weights) with float32
 * accumulation (MFMA); parameters, biases and Adam state are float32.
 * theta layout, float32 [PDC_MLP_PARAMS]: W1[25][64], b1[64], W2[64][64],
 * b2[64], W3[64][2], b3[2] (row-major, W[in][out]).
 * Calls on one network are ordered: use one stream, or synchronize.  The
 * synchronous calls below wait for the network's own last enqueued work (on
 * whatever stream it went), not for the whole device. */
#define PDC_MLP_PARAMS 5954
typedef struct pdc_mlp pdc_mlp;

/* Create a network on ctx's device with parameters theta_host (host, finite)
 * and zero Adam state.  It holds about 25 MB of device memory. */
pdc_status pdc_mlp_create(pdc_ctx *ctx, const float *theta_host, pdc_mlp **out);
pdc_status pdc_mlp_destroy(pdc_mlp *net);
/* Replace the parameters and reset the Adam state (synchronous). */
pdc_status pdc_mlp_set_params(pdc_mlp *net, const float *theta_host);
/* Copy the parameters to theta_host (synchronous). */
pdc_status pdc_mlp_get_params(pdc_mlp *net, float *theta_host);

/* Positions of n hits: out_dev float32 [n][2].  photon_adu in [2^-24, 2^24]. */
pdc_status pdc_mlp_infer(pdc_mlp *net, const float *patches_dev, uint64_t n, float photon_adu,
                         float *out_dev, void *hip_stream);

/* Network inputs (layout of pdc_capture_inputs) of n float32 patches:
 * inputs_dev uint16 [n][PDC_MLP_INPUT_WORDS].  photon_adu in [2^-24, 2^24]. */
pdc_status pdc_mlp_make_inputs(pdc_ctx *ctx, const float *patches_dev, uint64_t n, float photon_adu,
                               uint16_t *inputs_dev, void *hip_stream);

/* Positions of n hits from their network inputs (inputs_dev uint16
 * [n][PDC_MLP_INPUT_WORDS]; the padding words are ignored): the same values as
 * pdc_mlp_infer on the patches the inputs were made from, with 36 % fewer
 * bytes read. */
pdc_status pdc_mlp_infer_inputs(pdc_mlp *net, const uint16_t *inputs_dev, uint64_t n, float *out_dev,
                                void *hip_stream);

/* Gradient of L = sum((y - target)^2) / (2 n) over n >= 1 hits (target_dev
 * float32 [n][2]) into grad_host float32 [PDC_MLP_PARAMS] and L into
 * *loss_host (either may be NULL).  Deterministic.  Synchronous. */
pdc_status pdc_mlp_gradient(pdc_mlp *net, const float *patches_dev, const float *target_dev, uint64_t n,
                            float photon_adu, float *grad_host, double *loss_host, void *hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step count
 * kept by the network) on the gradient of L over the n >= 1 hits given.
 * lr finite and >= 0. */
pdc_status pdc_mlp_train_step(pdc_mlp *net, const float *patches_dev, const float *target_dev, uint64_t n,
                              float photon_adu, float lr, void *hip_stream);

/* L of the last pdc_mlp_train_step, at the parameters before its update
 * (synchronous).  ESTATE before the first step. */
pdc_status pdc_mlp_last_loss(pdc_mlp *net, double *loss);

/* ------------------------------------------------------------------------
 * Serving loop: several detectors' frame streams, each frame arriving at its
 * own time, processed on one GPU with continuous batching.  Each stream gets
 * its own HIP stream, so batches of different detectors overlap on the
 * device; a stream launches whatever has arrived (up to max_batch frames,
 * contiguous in its pool) whenever it has fewer than max_inflight batches in
 * flight and the device-memory budget admits the batch; arrivals beyond
 * max_queue waiting frames are dropped.  Results of a frame never depend on
 * the batch it was processed in (the per-frame contract above).  The run
 * ends when every frame is done or dropped; it blocks the calling thread
 * (a polling loop on the host clock).
 * ------------------------------------------------------------------------ */
#define PDC_SERVE_PENDING 0
#define PDC_SERVE_DONE 1
#define PDC_SERVE_DROPPED 2

typedef struct {
    uint64_t arrival_ns, launch_ns, done_ns;  /* host steady clock, from the start of the run */
    uint32_t hits;                            /* hits of the frame */
    uint32_t batch_frames;                    /* frames in the batch it was processed in */
    uint64_t photons;                         /* photons of the frame */
    int32_t status;                           /* PDC_SERVE_* */
    int32_t reserved;
} pdc_serve_frame;

/* Subpixel stage of a served stream (Photon Subpixel Resolution section):
 * positions of every hit, from the batch's patches (the detector must keep
 * PDC_KEEP_CORRECTED or PDC_KEEP_MEDIANS). */
#define PDC_SERVE_SUBPIXEL_NONE 0
#define PDC_SERVE_SUBPIXEL_MLP 1       /* the config's network on each hit's inputs (pdc_capture_inputs,
                                          pdc_mlp_infer_inputs) */
#define PDC_SERVE_SUBPIXEL_CENTROID 2  /* pdc_capture_centroids, eta-corrected when the config has a table */
#define PDC_SERVE_SUBPIXEL_MLP_FALLBACK 3  /* the network, then the centroid (eta-corrected when the config
                                              has a table) in place of every position that is not finite
                                              or outside [-1, 1] (pdc_capture_centroids' fallback) */

typedef struct {
    int32_t det;                 /* detector id from pdc_calibrate */
    uint32_t pool_frames;        /* frames in pool_dev (>= 1 when n_frames > 0) */
    const uint16_t *pool_dev;    /* DEVICE frames [pool_frames][pixels_per_frame]; frame i of the
                                    stream is pool frame i % pool_frames; borrowed for the run */
    uint64_t pixels_per_frame;   /* n_tiles * rows * cols of the detector */
    uint64_t n_frames;           /* frames of the stream */
    const uint64_t *arrival_ns;  /* host [n_frames], non-decreasing, from the start of the run */
    double hit_fraction;         /* hits per pixel to size batch buffers (exceeding it only costs
                                    a recomputation) */
    pdc_serve_frame *results;    /* host [n_frames], written by the run */
    pdc_hit *hits;               /* host hit records of the stream in (frame, pixel) order with
                                    frame = stream frame index, or NULL */
    uint64_t hits_capacity;      /* records the hits array holds (excess hits are not kept) */
    uint64_t hits_kept;          /* out: records written */
    int32_t subpixel;            /* PDC_SERVE_SUBPIXEL_* */
    float photon_adu;            /* the detector's single-photon signal (the network's input scale) */
    float t_nb;                  /* the detector's neighbour threshold n_nb * sigma (centroid mask) */
    float *positions;            /* host [hits_capacity][2] (dy, dx) of the kept hits, or NULL */
} pdc_serve_stream;

typedef struct {
    uint32_t max_batch;          /* frames per launch, >= 1 */
    uint32_t max_inflight;       /* batches in flight per stream, 1..64 */
    uint64_t max_queue;          /* waiting frames per stream before arrivals are dropped (0: none) */
    uint64_t hbm_budget;         /* bytes of in-flight batches over all streams (0: none), each
                                    charged pdc_batch_bytes plus its patches and positions;
                                    a stream with nothing in flight may always launch */
    pdc_mlp *net;                /* network of PDC_SERVE_SUBPIXEL_MLP(_FALLBACK) streams, or NULL */
    const float *eta_dev;        /* eta table of the centroid of PDC_SERVE_SUBPIXEL_CENTROID and
                                    _MLP_FALLBACK streams (float32 [2][eta_bins + 1] from
                                    pdc_eta_table), or NULL: plain centroid */
    int32_t eta_bins;
} pdc_serve_config;

typedef struct {
    uint64_t frames_done, frames_dropped, batches, peak_bytes, wall_ns;
} pdc_serve_summary;

/* Run the serving loop over n_streams (1..64) streams.  A frame is done once
 * its hits, counts and (with a subpixel stage) positions are on the host; a
 * subpixel stage runs when its batch completes, before the frame's done
 * time.  EINVAL on a bad argument (NULL arrays, decreasing arrival times,
 * zero sizes, an MLP stage without a network); errors of the calls it makes
 * are returned as they are.  summary may be NULL. */
pdc_status pdc_serve_run(pdc_ctx *ctx, pdc_serve_stream *streams, int32_t n_streams,
                         const pdc_serve_config *cfg, pdc_serve_summary *summary);

/* Test hook of the serving loop's batching (host only, no device work): the
 * number of frames the loop launches next for a queue holding the stream
 * frame indices pending[0..n_pending) (strictly increasing; gaps are frames
 * that were dropped), i.e. the run of consecutive indices at the front, at
 * most max_batch and not past the end of the device pool (pool frame
 * pending[0] % pool_frames onwards).  0 when the queue is empty.  EINVAL on
 * a NULL pointer or indices that do not increase. */
pdc_status pdc_debug_serve_batch_len(const uint64_t *pending, uint64_t n_pending, uint64_t max_batch,
                                     uint64_t pool_frames, uint64_t *n_out);

/* ------------------------------------------------------------------------
 * Summaries (Summarization section: photon-counting maps and histograms
 * accumulated over frames; Fig. g: spectra of Frames2 and of the summed
 * charges, split by the number of pixels summed; Dark and Gain section and
 * the noise thresholds of the Results section: pedestal and noise from dark
 * frames).
 *
 * Histograms have nbins + 2 uint32 counters: bin 0 counts values below lo
 * (and NaN), bins 1..nbins the range, bin nbins + 1 the values at or above
 * its end.  With s = nbins / (hi - lo) formed in binary32, a value x >= lo
 * goes to bin 1 + floor(t), t = fl(fl(x - lo) * s), when t < nbins, else to
 * bin nbins + 1.  1 <= nbins <= 2^24, lo < hi finite, and s must be a finite
 * positive binary32 value (EINVAL otherwise).
 *
 * Counts are ADDED to the caller's device arrays (clear them first, e.g. with
 * a fill kernel), with integer atomics: results do not depend on thread order,
 * and a counter wraps modulo 2^32.  The work is enqueued on hip_stream (a
 * hipStream_t of the context's device, or NULL for the context's
 * non-blocking stream) after the batch's kernels; the call returns once it is
 * enqueued, and pdc_release_batch waits for it.
 * ------------------------------------------------------------------------ */

/* Accumulate a batch's hits.  Each array may be NULL (then skipped):
 *   count_map_dev uint32 [n_tiles*rows*cols]: += nphot at the hit's pixel
 *     (photon-counting image summed over the batch's frames);
 *   spectrum_dev uint32 [nbins + 2]: += 1 at the bin of the hit's charge;
 *   size_spectra_dev uint32 [9][nbins + 2]: += 1 at [size - 1][bin(charge)],
 *     size = number of pixels of the hit's in-tile 3x3 window with Frames2
 *     above T_nb (1..9); needs PDC_KEEP_CORRECTED (ESTATE otherwise).
 * lo, hi and nbins are checked only when a histogram is requested. */
pdc_status pdc_accumulate_hits(pdc_ctx *ctx, uint64_t batch, uint32_t *count_map_dev, uint32_t *spectrum_dev,
                               uint32_t *size_spectra_dev, float lo, float hi, int32_t nbins, void *hip_stream);

/* Accumulate the histogram of every Frames2 value of a batch processed with
 * PDC_KEEP_CORRECTED (ESTATE otherwise) into hist_dev uint32 [nbins + 2]. */
pdc_status pdc_histogram_corrected(pdc_ctx *ctx, uint64_t batch, uint32_t *hist_dev, float lo, float hi,
                                   int32_t nbins, void *hip_stream);

/* Pedestal and noise per pixel from n_frames dark frames (DEVICE uint16
 * [n_frames][n_tiles][rows][cols], bits 14-15 ignored), 2 <= n_frames < 2^32.
 * With the exact integer sums S1 = sum adc and S2 = sum adc^2 over the frames
 * (adc = raw & 0x3FFF): pedestal = S1 / n and noise (the sample standard
 * deviation) = sqrt((n S2 - S1^2) / (n (n - 1))), each quotient and the root
 * in IEEE double from the exact integers, then rounded to binary32.
 * pedestal_host and noise_host (may be NULL) are host float32
 * [n_tiles*rows*cols].  Synchronous; device scratch of 16 bytes per pixel is
 * allocated for the call. */
pdc_status pdc_dark_stats(pdc_ctx *ctx, const pdc_geometry *geom, const uint16_t *darks_dev, uint64_t n_frames,
                          float *pedestal_host, float *noise_host, void *hip_stream);

/* pdc_dark_stats followed by pdc_calibrate with that pedestal and the host
 * gain plane: a detector calibrated from its dark frames.  noise_host may be
 * NULL.  Single-range detectors only (EINVAL otherwise). */
pdc_status pdc_calibrate_darks(pdc_ctx *ctx, const pdc_geometry *geom, const uint16_t *darks_dev, uint64_t n_frames,
                               const float *gain, const pdc_params *params, float *noise_host, int32_t *det_out);

/* Test hook: D = A B for one 16x32 by 32x16 bfloat16 tile through the MFMA
 * operand loads the network kernels use.  A (uint16 bf16 bits [16][32]),
 * B ([32][16]) and D (float32 [16][16]) are host arrays, row-major.
 * Synchronous. */
pdc_status pdc_debug_mfma_probe(pdc_ctx *ctx, const uint16_t *A, const uint16_t *B, float *D);

/* Test hook: the kernel that produced a batch's results, 1 for the general
 * kernel, 2 for the persistent one, 3 for the persistent one with the units
 * whose seed lists overflowed redone by the general kernel (after any
 * recomputation); 4 and 5 for 2 and 3 when the persistent kernel ran in the
 * one launch of a mixed call.  Waits for the batch. */
pdc_status pdc_debug_batch_path(pdc_ctx *ctx, uint64_t batch, int32_t *path);

#ifdef __cplusplus
}
#endif

#endif /* PDC_H */
