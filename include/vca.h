/*
 * vca.h -- C ABI of the MI355X (gfx950) Video Complexity Analyzer library.
 *
 * The library computes, per video frame, the seven block-DCT features of
 * Menon et al., "Green Video Complexity Analysis for Efficient Encoding in
 * Adaptive Video Streaming" (GMSys 2023), Section 2:
 *   E_Y  luma texture energy          h    gradient (frame-to-frame change) of E_Y
 *   L_Y  luma brightness              E_U, E_V  chroma texture energies
 *   L_U, L_V  chroma brightness
 * including the low-pass DCT option of Section 2 (optimisation (3)), read as
 * computing only the top-left K x K coefficients of each w x w block.
 *
 * Definitions (the cited VCA paper, which Section 2 defers to for formulas,
 * is not reproduced here; these are the readings this library implements):
 *   - Each plane (Y: W x H, U and V: W/2 x H/2, 4:2:0) is tiled with complete
 *     w x w blocks anchored at (0,0); rows/columns past the last complete
 *     block are ignored.  C_P = number of blocks of plane P.
 *   - Per block X (raw samples, bit depth B), the H.265 integer core transform
 *     C_w (entries in [-90, 90]) in two rounded passes, horizontal first:
 *       T = floor((X C_w^T + 2^(s1-1)) / 2^s1),  s1 = log2 w + B - 9
 *       Y = floor((C_w T   + 2^(s2-1)) / 2^s2),  s2 = log2 w + 6
 *     Y[i][k]: i = vertical, k = horizontal frequency; DC = Y[0][0].
 *   - Block energy H = sum_{(i,k) != (0,0), i,k < K} W_ik |Y[i][k]| with
 *     W_ik = exp(|((i+1)(k+1)/w^2)^2 - 1|).
 *   - E_P = sum H / (C_P w^2); L_P = sum sqrt(DC) / (C_P w^2);
 *     h = sum over luma blocks |H_p - H_{p-1}| / (C_Y w^2), h = 0 for the
 *     first frame after vca_open or vca_reset.
 * DCT coefficients and DC are exact integers (bit-exact); E, h and L are
 * accumulated in FP64 on the device and returned as FP32.
 *
 * Conventions: every function returns vca_status (except where noted); no
 * exception crosses the ABI.  A context is not thread-safe: use one per host
 * thread.  All device work of a context runs on the HIP stream given to
 * vca_open, in submission order.
 */
#ifndef VCA_H
#define VCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vca_ctx vca_ctx; /* opaque; owned by the library */

typedef enum {
  VCA_OK = 0,
  VCA_ERR_INVALID_ARG = 1, /* null pointer, out-of-range field, misaligned buffer      */
  VCA_ERR_UNSUPPORTED = 2, /* valid but not implemented (e.g. host frames to vca_tune)   */
  VCA_ERR_OOM = 3,         /* device or host allocation failed                          */
  VCA_ERR_DEVICE = 4,      /* a HIP call failed; vca_last_error() holds its message     */
  VCA_ERR_STATE = 5        /* request inconsistent with the context's history           */
} vca_status;

/* vca_config.flags */
#define VCA_F_KEEP_COEFFS 0x1u /* keep the K x K int16 coefficients of the last call (tests) */
#define VCA_F_VALIDATE 0x2u    /* 10-bit: mark each frame holding a sample above 1023;        \
                                  vca_features fails for a range that includes such a frame */
#define VCA_F_TIMING 0x4u      /* record HIP events around every kernel launch (vca_timing)  */
#define VCA_F_DOWNSAMPLE 0x8u  /* the paper's own low-pass option (Section 2, (3)): every     \
                                  plane is downsampled by two -- each sample the mean of a    \
                                  2 x 2 block, rounded half up -- and the features are those  \
                                  of the half-size video with the full w x w transform.       \
                                  Needs width and height divisible by 4, width/4 and          \
                                  height/4 >= block_size, lowpass_k 0 or w; not with          \
                                  VCA_F_KEEP_COEFFS or the batched form (VCA_ERR_UNSUPPORTED). \
                                  Frames are passed at full size; vca_block_counts and the    \
                                  per-block exports refer to the half-size planes.            */

typedef struct {
  uint32_t struct_size;  /* = sizeof(vca_config); guards ABI evolution                    */
  int32_t width;         /* luma width in samples; even; width/2  >= block_size            */
  int32_t height;        /* luma height in samples; even; height/2 >= block_size           */
  int32_t bit_depth;     /* 8 (uint8 samples) or 10 (uint16 little-endian, 0..1023)       */
  int32_t chroma_format; /* 420 (the only supported layout)                              */
  int32_t block_size;    /* w: 8, 16 or 32                                                 */
  int32_t lowpass_k;     /* 0 or w: full transform; else K in {w/2, w/4}                   */
  int32_t device;        /* HIP device ordinal                                             */
  uint32_t flags;        /* VCA_F_*                                                        */
  int32_t max_batch;     /* frames per internal launch (scratch sizing); 0 = 256           */
  int32_t feature_capacity; /* frames of features kept in the ring; 0 = 65536; must be    \
                               >= max_batch (after defaults), else VCA_ERR_INVALID_ARG    */
} vca_config;

/* A run of consecutive frames of one video.
 * Device frames (on_device = 1): y/u/v, pitches and frame strides must be
 * multiples of 16 bytes.  Host frames (on_device = 0, vca_analyze_frames
 * only): any alignment; the library copies them through pinned staging
 * buffers before vca_analyze_frames returns. */
typedef struct {
  const void* y;       /* first sample of frame 0 of each plane                        */
  const void* u;
  const void* v;
  int64_t pitch_y;     /* bytes between rows of Y (>= width * bytes per sample)        */
  int64_t pitch_uv;    /* bytes between rows of U and of V (>= width/2 * bytes/sample) */
  int64_t fstride_y;   /* bytes between consecutive frames of Y                        */
  int64_t fstride_uv;  /* bytes between consecutive frames of U and of V               */
  int32_t on_device;   /* 1: device pointers; 0: host pointers (staged by the library) */
} vca_frames;

/* Per-frame feature record, in the order Section 2 lists the features. */
typedef struct {
  float E_Y, h, L_Y, E_U, E_V, L_U, L_V;
} vca_frame_features;

/* Device time spent in the library's kernels (needs VCA_F_TIMING), summed
 * over launches since vca_open or the last reset of the counters. */
typedef struct {
  double forward_ms;        /* block transform + energy kernels                   */
  double reduce_ms;         /* per-frame feature reduction kernels                */
  int64_t forward_launches;
  int64_t reduce_launches;
  int64_t frames;           /* frames covered by the timed launches                */
} vca_timing;

/* Number of complete blocks of the Y, U and V planes for a configuration.
 * Host only; touches no device. */
vca_status vca_block_counts(const vca_config* cfg, int32_t counts[3]);

/* Creates a context: validates cfg, builds the transform and weight tables,
 * allocates device state on cfg->device.  hip_stream is a hipStream_t (NULL:
 * the context creates and owns a stream of default priority).  On success
 * *out receives the context; on failure *out is NULL. */
vca_status vca_open(const vca_config* cfg, void* hip_stream, vca_ctx** out);

/* Enqueues the analysis of n_frames frames (n_frames >= 0) on the context's
 * stream and returns without waiting.  Frames are numbered after those of
 * earlier calls, and h chains across calls.  Device frames: the caller keeps
 * the buffers valid until the stream has finished the work (vca_features of
 * the call's last frame waits for it).  Host frames (frames->on_device = 0):
 * the library copies them, batch by batch, into one of two pinned staging
 * buffers (in parallel over host threads) and from there to the device on a
 * second stream, each batch's copy overlapping the analysis of the one
 * before; the caller may reuse its buffers as soon as the call returns.  Host frames are not
 * accepted with VCA_F_KEEP_COEFFS (VCA_ERR_UNSUPPORTED).
 * With VCA_F_KEEP_COEFFS, n_frames must not exceed max_batch. */
vca_status vca_analyze_frames(vca_ctx* ctx, const vca_frames* frames, int32_t n_frames);

/* Analyses frames [first_frame, first_frame + n_frames) of a raw planar
 * 4:2:0 .yuv file (I420: per frame the Y rows, then U, then V, no row
 * padding; 10-bit samples as little-endian uint16) of the context's
 * resolution and bit depth, read with pread straight into the pinned staging
 * buffers and otherwise handled like host frames.  Returns when every
 * frame has been read; the analysis is enqueued.  VCA_ERR_INVALID_ARG if the
 * file cannot be opened or holds fewer frames. */
vca_status vca_analyze_yuv_file(vca_ctx* ctx, const char* path, int64_t first_frame,
                                int32_t n_frames);

/* Host only (no device): reads frames [first_frame, first_frame + n_frames)
 * of a raw .yuv file laid out as above into tight planes y [n][height][width],
 * u and v [n][height/2][width/2] (samples of 1 or 2 bytes).
 * VCA_ERR_INVALID_ARG on a bad argument, a missing file or too few frames. */
vca_status vca_read_yuv(const char* path, int32_t width, int32_t height, int32_t bit_depth,
                        int64_t first_frame, int32_t n_frames, void* y, void* u, void* v);

/* Waits for the launch that produced frame first_frame + count - 1 (not for
 * work queued after it, so the next call may already be enqueued), then
 * copies the features of frames [first_frame, first_frame + count) into
 * out_host (count records).
 * VCA_ERR_STATE if a frame was not yet submitted or has left the ring, or if
 * VCA_F_VALIDATE found a sample above 1023 in one of the requested frames
 * (each frame carries its own mark, so frames of other calls do not
 * matter). */
vca_status vca_features(vca_ctx* ctx, int64_t first_frame, int32_t count,
                        vca_frame_features* out_host);

/* Test/debug export (needs VCA_F_KEEP_COEFFS): waits for the stream, then
 * copies the coefficients of frame `frame` of the most recent
 * vca_analyze_frames call: blocks of Y, then U, then V, each in raster order;
 * per block K x K int16, row-major (row = vertical frequency), DC included.
 * All three planes of the frame come in one call (the frame's block list is
 * one array, as for vca_block_stats; vca_block_counts gives the plane
 * boundaries), so there is no plane argument.
 * capacity is the number of int16 elements out_host can hold. */
vca_status vca_block_coeffs(vca_ctx* ctx, int64_t frame, int16_t* out_host, size_t capacity);

/* Per-block export of frame `frame` of the most recent call: block energies
 * H (FP64) and DC (int32), blocks ordered as in vca_block_coeffs.  Waits for
 * the stream.  capacity is the number of blocks each array can hold. */
vca_status vca_block_stats(vca_ctx* ctx, int64_t frame, double* h_host, int32_t* dc_host,
                           size_t capacity);

/* Per-block feature maps (the summands of the features of Section 2 of the
 * paper, for encoder decisions per block) of frames [first_frame,
 * first_frame + count) of the most recent launch -- the frames of the last
 * max_batch-sized chunk of the most recent vca_analyze_frames call --
 * written to caller-owned DEVICE memory on the context's stream (enqueued,
 * no wait; the caller orders later use after the stream):
 *   h_dev [i * P + b]   block energy H_b of frame first_frame + i (FP64),
 *                       P = vca_block_counts total, blocks ordered as in
 *                       vca_block_coeffs (Y, then U, then V, raster order);
 *   dc_dev[i * P + b]   block DC (int32, the integer transform's (0,0));
 *   dh_dev[i * C_Y + b] |H_b(t) - H_b(t-1)| of luma block b (FP64), the
 *                       summand of h; 0 where frame t has no previous frame
 *                       (the first frame after vca_open or vca_reset).
 * Any of the three output pointers may be NULL (that map is skipped); each
 * non-NULL one must be 8-byte aligned and hold count maps.
 * VCA_ERR_INVALID_ARG for a NULL context, count <= 0 or all outputs NULL;
 * VCA_ERR_STATE if the range is not inside the most recent launch. */
vca_status vca_block_maps(vca_ctx* ctx, int64_t first_frame, int32_t count, double* h_dev,
                          int32_t* dc_dev, double* dh_dev);

/* Waits for the context's stream and returns the kernel times measured with
 * HIP events on that stream (VCA_F_TIMING); reset != 0 clears the counters
 * afterwards.  VCA_ERR_STATE if the context was opened without the flag. */
vca_status vca_get_timing(vca_ctx* ctx, vca_timing* out, int32_t reset);

/* Autotuner of the launch shape: times the forward kernel on the given
 * frames (at most max_batch of them) for every candidate -- tiles in flight
 * per wavefront 1, 2 or 4 times workgroups per compute unit 1..(as many as
 * fit) --
 * with `reps` timed launches each, and keeps the fastest for this context.
 * The choice is also cached for the process (and in the text file named by
 * the environment variable VCA_TUNE_CACHE, if set) under the key (device,
 * bit depth, w, K, resolution); later vca_open calls with the same key use
 * it.  Features, h state and frame numbering are unchanged; the per-block
 * results of the previous call are overwritten, so vca_block_stats and
 * vca_block_maps return VCA_ERR_STATE until the next analysis.  The tuning
 * launches do not validate samples.  Not available with
 * VCA_F_KEEP_COEFFS (VCA_ERR_STATE).  Launches too small to fill the device
 * (about two 2160p frames or fewer) take runs of one strip at the untuned
 * depth instead; the tuned shape applies to all others. */
vca_status vca_tune(vca_ctx* ctx, const vca_frames* frames, int32_t n_frames, int32_t reps);

/* Launch shape in use: tiles in flight per wavefront (0: untuned default),
 * workgroups per compute unit (0: as many as fit), and the tuned kernel time
 * in ms.  Any output pointer may be NULL. */
vca_status vca_tuned_launch(const vca_ctx* ctx, int32_t* depth, int32_t* groups_per_cu, double* ms);

/* Forgets the previous frame: the next analysed frame gets h = 0.  Frame
 * numbering continues. */
vca_status vca_reset(vca_ctx* ctx);

/* Number of frames submitted so far (returns -1 for a NULL context). */
int64_t vca_frames_submitted(const vca_ctx* ctx);

/* Waits for outstanding work and frees the context.  NULL-safe. */
void vca_close(vca_ctx* ctx);

/* Allocation-free analysis, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Analyses n_frames device-resident frames (frames->on_device
 * = 1, the alignment rules above) of a video with configuration cfg as one
 * fresh sequence -- h = 0 for its first frame, chained over the rest -- and
 * enqueues the plain path's kernels on hip_stream (a hipStream_t; NULL = the
 * null stream) without waiting.  The features (7 floats per frame, in
 * vca_frame_features order) are written to features_dev, caller-owned DEVICE
 * memory of n_frames records, 4-byte aligned; they are identical to those of
 * a freshly opened context fed the same frames.  No context, no allocation:
 * every intermediate (tables, per-block energies and DC, the previous
 * frame's luma energies) lives in one fixed 32 MiB device array of the
 * library, which every device the call runs on holds until the process ends.
 * The call cuts the frames into launches of as many frames as fit there.
 *   - The first call on each device finds the array's address and uploads
 *     the transform tables with synchronous copies; make that call outside
 *     stream capture.
 *   - Calls share their device's array: two calls that may run at the same
 *     time on one device (different streams) race and corrupt each other's
 *     results.  Calls on one stream are ordered and safe.
 *   - cfg->max_batch and feature_capacity are ignored; VCA_F_KEEP_COEFFS,
 *     VCA_F_VALIDATE and VCA_F_TIMING give VCA_ERR_UNSUPPORTED, as does a
 *     frame too large for the array: one frame needs 12 bytes per block (all
 *     planes) plus 16 bytes per luma block, and the array leaves
 *     32 MiB - 144 KiB for that (every size up to 8192 x 4096 at w = 8).
 *   - VCA_ERR_INVALID_ARG for a bad cfg, frames or output pointer;
 *     VCA_ERR_DEVICE if a HIP call fails.  No error detail is kept. */
vca_status vca_analyze_noalloc(const vca_config* cfg, const vca_frames* frames, int32_t n_frames,
                               float* features_dev, void* hip_stream);

/* ------------------------------------------------------------ batched form
 * Many independent streams -- each with its own resolution, block size,
 * low-pass size, bit depth and frame count -- analysed in one round of
 * launches: per class of streams (bit depth, w, K) ONE persistent kernel
 * launch over all their tiles (its wavefronts draw work from a device counter
 * of the class; one small kernel zeroes the counters first), each followed by
 * the class's reduction launch, the classes one after another or side by
 * side on parallel branches (the tuned arrangement); the round is captured
 * into a hipGraph on the first call with a given signature (frames per
 * stream, class shapes, arrangement) and replayed afterwards (only the
 * per-stream descriptor tables are uploaded per call).  A batch keeps up to
 * 16 such graphs until it is closed; a round with a further signature runs
 * its launches in line on the batch's stream.  Per stream the results are
 * identical to a vca_ctx opened with the same configuration and fed the
 * same frames. */
typedef struct vca_batch vca_batch; /* opaque; owned by the library */

/* Opens a batch of n_streams streams (cfgs[s] configures stream s; all on
 * the same device; VCA_F_KEEP_COEFFS is not supported).  max_batch = 0 means
 * 300 frames per stream and launch, feature_capacity = 0 means 4096. */
vca_status vca_open_batch(const vca_config* cfgs, int32_t n_streams, void* hip_stream,
                          vca_batch** out);

/* Enqueues frames[s] (n_frames[s] >= 0 frames) for every stream s; returns
 * without waiting.  Streams whose count exceeds their max_batch are
 * processed in several rounds.  Frame buffers must stay valid until the
 * round that reads them is done (vca_batch_features of a stream's last
 * submitted frame waits for it). */
vca_status vca_analyze_batch(vca_batch* b, const vca_frames* frames, const int32_t* n_frames);

/* Features of frames [first, first + count) of stream `stream`; waits for
 * the round that produced frame first + count - 1 (not for later rounds).
 * VCA_ERR_STATE if that stream was opened with VCA_F_VALIDATE and one of
 * the requested frames holds a 10-bit sample above 1023 (other frames and
 * streams are unaffected).  The stream's feature_capacity must be at least
 * its max_batch (vca_open_batch returns VCA_ERR_INVALID_ARG otherwise). */
vca_status vca_batch_features(vca_batch* b, int32_t stream, int64_t first, int32_t count,
                              vca_frame_features* out_host);

/* Several feature reads in one call: request r is frames [first[r],
 * first[r] + count[r]) of stream streams[r] (host arrays of n_requests
 * entries); their records go to out_host one request after another
 * (sum of count[r] records, caller-owned).  Waits once, for the latest round
 * any request needs.  Every request is checked before anything is copied
 * (VCA_ERR_INVALID_ARG for a bad stream or range, VCA_ERR_STATE for frames
 * not submitted or out of the ring); a stream with a validation mark on a requested frame
 * gives VCA_ERR_STATE (a requested frame of it holds a 10-bit sample above
 * 1023) after the records of the requests before it are written. */
vca_status vca_batch_features_many(vca_batch* b, int32_t n_requests, const int32_t* streams,
                                   const int64_t* first, const int32_t* count,
                                   vca_frame_features* out_host);

/* Autotuner of the batched launch shapes: over the first round of the given
 * frames of every stream, times each class's forward launch alone for every
 * ring depth (1, 2, 4), wavefronts per workgroup (4, 8) and count of
 * workgroups per compute unit that fits, then every chunk size (8, 16, 32,
 * 64 strips) at the fastest of those, and keeps the fastest per class; then
 * times whole rounds of the tuned classes (reductions included) one after
 * another and side by side, max(reps, 4) of each in turn, and keeps the
 * faster arrangement
 * (vca_batch_arrangement).  Cached under the batch's stream list for the
 * process (and in the file named by VCA_TUNE_CACHE).  Allocates a scratch
 * area of 32 bytes per feature-ring slot of the largest ring while it runs
 * (VCA_ERR_OOM if that fails).  Features and h state are unchanged. */
vca_status vca_tune_batch(vca_batch* b, const vca_frames* frames, const int32_t* n_frames,
                          int32_t reps);

/* Launch shape of the batch (see vca_tuned_launch): the shape of its most
 * expensive class, and the sum of the classes' tuned forward times. */
vca_status vca_batch_tuned_launch(const vca_batch* b, int32_t* depth, int32_t* groups_per_cu,
                                  double* ms);

/* Per class of streams, the tuned forward launch: ms[k] its device time alone
 * (0 for a class not tuned), depth[k] its ring depth, groups_per_cu[k] its
 * workgroups per compute unit, waves[k] its wavefronts per workgroup (4 or
 * 8) and chunk_strips[k] the strips a wavefront draws at a time (8 to 64),
 * all 0 when untuned.  Each output may be NULL, else an array of 18 entries
 * indexed by class k = (B == 10 ? 9 : 0) + 3 * (w == 32 ? 0 : w == 16 ? 1 :
 * 2) + (K == w ? 0 : K == w / 2 ? 1 : 2).  Host only. */
vca_status vca_batch_class_times(const vca_batch* b, double* ms, int32_t* depth,
                                 int32_t* groups_per_cu, int32_t* waves, int32_t* chunk_strips);

/* Arrangement of the classes in a round: *serial = 1 when the classes'
 * forward launches run one after another (each class's reduction overlapping
 * the next class), 0 when they run side by side on parallel branches.
 * Serial unless vca_tune_batch (here or earlier in the process, or through
 * VCA_TUNE_CACHE) measured side by side faster; *serial_ms and *parallel_ms
 * are those tuned round times, reductions included (0 when not measured).
 * Each output may be NULL.  Host only. */
vca_status vca_batch_arrangement(const vca_batch* b, int32_t* serial, double* serial_ms,
                                 double* parallel_ms);

/* Sets class cls's launch shape for the later rounds in place of the tuned
 * one (until the next vca_tune_batch): ring depth 1, 2 or 4, workgroups per
 * compute unit (0: as many as fit), wavefronts per workgroup 4 or 8, and
 * strips per chunk 8, 16, 32 or 64; cls numbered as in
 * vca_batch_class_times.  VCA_ERR_INVALID_ARG for any other value; its
 * ms in vca_batch_class_times reads 0.  Host only. */
vca_status vca_batch_set_class_shape(vca_batch* b, int32_t cls, int32_t depth, int32_t groups_per_cu,
                                     int32_t waves, int32_t chunk_strips);

/* Sets the arrangement of the later rounds (serial = 1: one class after
 * another, 0: side by side) in place of the tuned one, until the next
 * vca_tune_batch.  VCA_ERR_INVALID_ARG for another value.  Host only. */
vca_status vca_batch_set_arrangement(vca_batch* b, int32_t serial);

/* Device time of the batch's launches (both kernels), measured with HIP
 * events on its stream when any stream was opened with VCA_F_TIMING. */
vca_status vca_batch_timing(vca_batch* b, double* total_ms, int64_t* launches, int64_t* frames,
                            int32_t reset);

/* Forgets the previous frame of one stream (stream >= 0) or of all (-1). */
vca_status vca_reset_batch(vca_batch* b, int32_t stream);

/* Frames submitted so far to a stream (-1 for a bad argument). */
int64_t vca_batch_submitted(const vca_batch* b, int32_t stream);

/* Message of the batch's last failure (owned by the batch). */
const char* vca_batch_last_error(const vca_batch* b);

/* Waits for outstanding work and frees the batch.  NULL-safe. */
void vca_close_batch(vca_batch* b);

/* ---------------------------------------------------------- backward form
 * Differentiable luma texture energy E_Y and its gradient h (Section 2
 * names both features) for training pre-processing filters toward a target
 * complexity.  The rounding of the two transform passes is dropped so that
 * the features are piecewise linear in the samples: per w x w block X of a
 * float luma plane,
 *   Y = C_w X C_w^T * 2^-(2 log2 w + B - 3)  (the unrounded composition of
 *       the two integer passes above; B = bit_depth fixes only the scale),
 *   H = sum W_ik |Y[i][k]| over (i,k) != (0,0), i,k < K,
 *   E_t = sum_blocks H_t / (C_Y w^2),
 *   h_t = sum_blocks |H_t - H_{t-1}| / (C_Y w^2), h = 0 at a sequence start,
 * and dH/dX = 2^-(2 log2 w + B - 3) C_w^T (W o sign(Y)) C_w, sign(0) = 0.
 * The transforms run on fp16 matrix cores with FP32 accumulation over
 * operands split into fp16 integers, so every accumulation is exact: each
 * sample is taken as a + 2^-11 b + 2^-22 c (three integer digits), which is
 * the sample itself for |x| in [2, 2^11) and for every sample on the 2^-22
 * grid, and within 2^-23 of it for |x| < 2; the coefficients Y are then
 * exact (assembled in FP64), so E and h carry only FP64 rounding.  Samples
 * of magnitude 2^11 or more are outside this domain (results approximate).
 * Block energies and the per-frame sums are FP64.  Input: n_seq sequences of
 * seq_len consecutive float32 frames. */
typedef struct {
  uint32_t struct_size; /* = sizeof(vca_grad_config)                                   */
  int32_t width;        /* luma width; >= block_size                                   */
  int32_t height;       /* luma height; >= block_size                                  */
  int32_t block_size;   /* w: 8, 16 or 32                                              */
  int32_t lowpass_k;    /* 0 or w: full; else K in {w/2, w/4}                          */
  int32_t bit_depth;    /* 8 or 10: B of the scale above                               */
  int32_t n_seq;        /* sequences (h restarts at each); n_seq * seq_len <= 65535    */
  int32_t seq_len;      /* frames per sequence                                         */
  int32_t device;       /* HIP device ordinal                                          */
  int64_t pitch;        /* floats between rows (>= width, multiple of 4)               */
  int64_t fstride;      /* floats between consecutive frames (multiple of 4)           */
} vca_grad_config;

/* Bytes of device workspace the two calls below need (the FP64 block
 * energies of every frame and the signs of every tile's coefficients, 256
 * bytes per 32 x 32 tile), or -1 for an invalid configuration.  Host only. */
int64_t vca_grad_workspace(const vca_grad_config* cfg);

/* Forward: reads x (device, 16-byte aligned, cfg's layout), writes E[f] and
 * h[f] (device, n_seq * seq_len floats each, frame f = s * seq_len + t) and
 * the workspace (device, vca_grad_workspace bytes, 256-byte aligned; keep it
 * unchanged for vca_energy_backward).  Within the domain above, the signs
 * of all coefficients, zeros included, are exact.  Enqueued on
 * hip_stream (NULL: the default stream); returns without waiting. */
vca_status vca_energy_forward(const vca_grad_config* cfg, const float* x, float* E, float* h,
                              void* workspace, void* hip_stream);

/* Backward: given dL/dE and dL/dh per frame (device, n_seq * seq_len floats)
 * and the workspace of the forward call, writes dL/dx to grad_x (device,
 * 16-byte aligned, the layout of the forward's x); every sample within
 * width x height of every frame is written (0 outside the block grid), the
 * pitch padding is not touched.  The samples themselves are not read again.
 * Enqueued on hip_stream; returns without waiting. */
vca_status vca_energy_backward(const vca_grad_config* cfg, const void* workspace,
                               const float* grad_E, const float* grad_h, float* grad_x,
                               void* hip_stream);

/* Static string naming a status code. */
const char* vca_status_str(vca_status s);

/* Message of the last failure of ctx (owned by ctx; "" if none). */
const char* vca_last_error(const vca_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* VCA_H */
