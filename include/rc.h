/*
 * rc.h - real-time FMCW SAR back-projection on AMD Instinct MI355X (gfx950).
 *
 * C ABI of librc.so.  The library forms SAR images from FMCW radar frames with
 * the optimised back-projection of Hoffmann et al., "Implementation of
 * Real-Time Automotive SAR Imaging" (arXiv 2306.09784), Alg. 2, and runs a
 * cell-averaging CFAR detector on each image.  Per frame it executes, on one
 * HIP stream:
 *
 *   1. range compression: windowed, zero-padded DFT of every chirp/channel
 *      beat signal, cropped to the kept bins (the equidistant beat spectrum s
 *      that Alg. 1 and Alg. 2 interpolate, Sec. III-C);
 *   2. per-frame tables: the per-pixel Doppler shift from the average
 *      velocity (Sec. III-D);
 *   3. back-projection (Alg. 2): per pixel, chirp and channel the two-way
 *      path d_hyp, index f_ind = a1 d_hyp + f_doppler(p), phase
 *      exp(a2 d_hyp), linear interpolation of s at f_ind, weight w_sar[m]
 *      (Sec. III-B) and the coherent sum;
 *   4. 2-D CA-CFAR on |P|^2 over the pixel lattice (a detection stage layered
 *      on the image; not part of the paper) and ordered compaction of the
 *      detections.
 *
 * Conventions
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  Complex numbers are interleaved
 *     float pairs (re, im), i.e. complex64.
 *   - Every function returns an rc_status.  No exception crosses the ABI.  On
 *     an error the thread-local message of rc_last_error() describes it.
 *   - A plan is used by one host thread at a time.  Streams are hipStream_t
 *     passed as void*; NULL means the default stream.
 *   - Distances are metres, frequencies Hz, times seconds.  Positions are
 *     planar (x, y); distances are the paper's 2-D ones unless a frame gives
 *     the antennas a height above the pixels' plane.
 */
#ifndef RC_H_
#define RC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RC_ABI_VERSION 5

typedef enum rc_status {
  RC_OK = 0,
  RC_EINVAL = 1,     /* bad argument or descriptor; nothing was launched          */
  RC_ENOMEM = 2,     /* device or pinned memory exhausted, or over the HBM budget */
  RC_ETRUNC = 3,     /* output buffer too small; *n_out holds the needed count    */
  RC_EHIP = 4,       /* a HIP runtime call failed; see rc_last_error()            */
  RC_ENOTREADY = 5,  /* no free frame slot / frame still in flight                */
  RC_ENOTFOUND = 6   /* unknown frame id                                          */
} rc_status;

typedef enum rc_window_kind {
  RC_WIN_RECT = 0,
  RC_WIN_HANN = 1,   /* symmetric Hann, 0.5 - 0.5 cos(2 pi t / (n - 1))           */
  RC_WIN_KAISER = 2  /* I0(beta sqrt(1 - (2t/(n-1) - 1)^2)) / I0(beta)            */
} rc_window_kind;

typedef enum rc_precision {
  /* Alg. 2 in single precision, as the paper runs it (Sec. III-A). */
  RC_PREC_FP32 = 0,
  /* Single precision with the phase split into a per-pixel reference path
   * (evaluated in double) plus a small single-precision difference; keeps the
   * carrier phase accurate to ~1e-5 of a turn.  Its detection lists match the
   * FP64 oracle's outside the CFAR band; the plain form's carry its ~1e-4
   * turns of phase rounding at weak cells beside strong scatterers. */
  RC_PREC_FP32_SPLIT = 1,
  /* Reduced-precision spectrum: range compression (the beat spectrum s of
   * Sec. III-C) on the matrix cores, its two DFT stages as complex matrix
   * products with FP16 (RC_PREC_FP16) or BF16 (RC_PREC_BF16) operands, FP32
   * accumulation and twiddles split into high and low parts; back-projection
   * as RC_PREC_FP32_SPLIT.  DFT lengths 256 .. 4096 with n_samples at most
   * n_fft / 2 (RC_EINVAL otherwise). */
  RC_PREC_FP16 = 2,
  RC_PREC_BF16 = 3
} rc_precision;

typedef enum rc_doppler_mode {
  /* Alg. 2: the Doppler shift of each pixel is evaluated once, at the
   * aperture centre with the mean velocity (Sec. III-D). */
  RC_DOPPLER_AVERAGE = 0,
  /* Alg. 1: the radial velocity of every pixel, chirp and channel from that
   * chirp's velocity (the paper's reference before the simplification).
   * Single precision only (not with RC_PREC_FP32_SPLIT). */
  RC_DOPPLER_EXACT = 1,
  /* Alg. 1 as the paper states it, before its constants are folded
   * (Sec. III-C, Tab. II "Opt."): metres and seconds, tau = (d_tx + d_rx) / c,
   * f_hyp = mu tau + f0 v / c in Hz, the interpolation index f_hyp / df and
   * the phase f0 tau, each a division or product per term; the radial speeds
   * <p - q, v> / d divided out per leg.  The same values as RC_DOPPLER_EXACT
   * to single-precision rounding (its phase holds ~2e-3 turns of it at 30 m),
   * slower: the reference row of the ablation.  Single precision only, no
   * continuous SAR. */
  RC_DOPPLER_EXACT_DIRECT = 2
} rc_doppler_mode;

/* Continuous SAR (the paper's conclusion, Sec. V: a continuous measurement
 * imaged as it arrives).  A sensor's chirp stream is cut into sub-apertures
 * of S chirps, one rc_frame each; the image of sub-aperture b is the aperture
 * of the last K sub-apertures (N = K S chirps, b - K + 1 .. b), weighted by
 * the plan's chirp window over N positions (Sec. III-B); sub-apertures before
 * the stream started hold no chirps.  With the averaged Doppler (Alg. 2) each
 * sub-aperture's terms use that sub-aperture's own Doppler table (its mean
 * positions and velocity, Sec. III-D).  Every chirp is back-projected once:
 * the plan keeps, per sensor, the last sub-apertures' partial images (for the
 * Hann window three of them: the plain sum and the sums weighted by the
 * cosine and sine of the chirp's window phase, from which any window offset
 * is one linear combination), and forms each aperture from them. */
typedef enum rc_sliding {
  RC_SLIDE_OFF = 0,    /* an independent aperture (default)                       */
  RC_SLIDE_NEXT = 1,   /* the next sub-aperture of sensor_id's stream             */
  RC_SLIDE_START = 2   /* the first sub-aperture of a new stream of sensor_id     */
} rc_sliding;

typedef enum rc_input_kind {
  RC_INPUT_RAW = 0,      /* data = beat signal complex64 [n_chirps][n_channels][n_samples] */
  RC_INPUT_SPECTRUM = 1  /* data = beat spectrum complex64 [n_chirps][n_channels][n_bins]  */
} rc_input_kind;

/* How a plan holds the device memory of the frames in flight. */
typedef enum rc_frame_memory {
  /* Every frame slot sized for the plan's limits and allocated at creation
   * (hbm_budget_bytes, if set, bounds their total). */
  RC_MEMORY_SLOTS = 0,
  /* One device arena of hbm_budget_bytes allocated at creation.  A frame takes
   * from it the bytes its own sizes need (rc_frame_bytes) when it is admitted
   * and gives them back when it is released, so frames of uneven sizes share
   * the budget by what they use: rc_process_batch returns RC_ENOTREADY
   * (enqueuing nothing) while the batch does not fit what is free, and
   * RC_ENOMEM for a frame larger than the whole arena (it would never fit);
   * max_frames_in_flight still bounds the count.  A frame may then hand over
   * its input in pinned host memory (rc_frame.data_host): the plan copies it
   * into the frame's share of the arena on a copy stream of its own, and the
   * frame's kernels wait for the copy (the paper's pinned-memory Load,
   * Sec. IV).  A batch of one frame whose back-projection splits its chirps
   * into blocks is copied in those blocks' pieces, and each block's range
   * compression and back-projection wait only for their own piece, so the
   * later pieces' copies overlap the frame's own compute (same results). */
  RC_MEMORY_BUDGET = 1
} rc_frame_memory;

/* Radar constants (Tab. I of the paper for its sensor). */
typedef struct rc_radar {
  double f0;         /* carrier frequency, Hz (76.6e9)              */
  double bandwidth;  /* RF bandwidth B, Hz (931e6)                  */
  double t_chirp;    /* chirp duration T_P, s (102.4e-6)            */
  double c;          /* propagation speed, m/s; 0 -> 299792458      */
} rc_radar;

/* Plan descriptor: limits size the per-frame slots allocated at creation. */
typedef struct rc_plan_desc {
  int32_t abi_version;          /* must be RC_ABI_VERSION                         */
  rc_radar radar;
  int32_t n_samples_max;        /* fast-time samples per chirp                    */
  int32_t n_fft_max;            /* zero-padded DFT length, power of two <= 4096   */
  int32_t n_bins_max;           /* kept spectrum bins                             */
  int32_t n_chirps_max;
  int32_t n_channels_max;
  int64_t n_pix_max;
  int32_t max_frames_in_flight; /* frame slots                                    */
  int32_t max_detections;       /* detection capacity per frame                   */
  rc_window_kind range_window;  double range_kaiser_beta;
  rc_window_kind sar_window;    double sar_kaiser_beta;   /* w_sar over chirps   */
  rc_precision precision;
  rc_doppler_mode doppler;
  int32_t cfar_guard;           /* guard cells each side (2)                      */
  int32_t cfar_train;           /* training cells each side beyond guard (8)      */
  double cfar_pfa;              /* design false-alarm probability (1e-4)          */
  double cfar_margin_rel;       /* near-threshold band: |power - thr| <= margin * thr */
  int32_t max_rechecks;         /* near-threshold cells per frame whose decision is
                                   re-evaluated in double precision (their pixel and
                                   training pixels formed again by back-projection in
                                   double); 0 disables the recheck.  Cells of the band
                                   not rechecked are flagged RC_DET_NEAR_THRESHOLD.  */
  int64_t hbm_budget_bytes;     /* 0 = unlimited                                  */
  int32_t stage_timing;         /* nonzero: bracket every stage with timing events
                                   (read with rc_stage_times)                      */
  /* continuous SAR (rc_sliding); sliding_sensors = 0 disables it.  The plan
   * holds (K + depth - 1) partial images of n_pix_max pixels per sensor (three
   * planes each with the Hann window, one with the rectangular one; the
   * Kaiser window has no such decomposition and is refused) */
  int32_t sliding_sensors;      /* sensors 0 .. sliding_sensors - 1                */
  int32_t sliding_subapertures; /* K, sub-apertures per aperture, 1 .. 64          */
  int32_t sliding_depth;        /* sub-apertures of one sensor in flight at once   */
  rc_frame_memory frame_memory; /* RC_MEMORY_SLOTS (default) or RC_MEMORY_BUDGET     */
} rc_plan_desc;

/* One radar frame (one synthetic aperture -> one image + detection list).
 * The caller owns every buffer and keeps it alive until the frame completes
 * (rc_poll() == RC_OK or rc_detections() returned). */
typedef struct rc_frame {
  int64_t frame_id;             /* caller-chosen, unique among frames in flight   */
  int32_t sensor_id;
  int32_t n_samples;            /* fast-time samples per chirp (RAW)              */
  int32_t n_fft;                /* DFT length, power of two >= n_samples (RAW)    */
  int32_t n_bins;               /* spectrum bins kept and interpolated            */
  int32_t n_chirps;             /* chirps m (per-TX cycles for TDM-MIMO)          */
  int32_t n_channels;           /* channels ch per chirp                          */
  double fs;                    /* IQ sample rate, Hz                             */
  rc_input_kind input_kind;
  const void* data;             /* device, see rc_input_kind                      */
  const float* q_tx;            /* host [n_chirps][n_channels][2] TX positions   */
  const float* q_rx;            /* host [n_chirps][n_channels][2] RX positions   */
  const float* vel;             /* host [n_chirps][2] vehicle velocity            */
  const float* pixels;          /* device [n_rows * n_cols][2] pixel positions p,
                                   row-major lattice (Cartesian or polar grid)    */
  int32_t n_rows;
  int32_t n_cols;
  void* image_out;              /* device complex64 [n_rows * n_cols] or NULL     */
  float* doppler_out;           /* device float [n_rows * n_cols] (bins) or NULL  */
  void* spectrum_out;           /* device complex64 [n_chirps][n_channels][n_bins]
                                   beat spectrum before w_sar, or NULL            */
  double height;                /* antennas above the plane of the pixels, metres:
                                   distances become sqrt(|p - q|^2 + height^2);
                                   0 is the paper's planar geometry               */
  rc_sliding sliding;           /* RC_SLIDE_NEXT / _START: this frame is the next
                                   sub-aperture (n_chirps = S) of sensor_id's
                                   stream; image_out and the detections are of the
                                   aperture it completes.  Every sub-aperture of a
                                   stream has the same n_chirps, n_channels,
                                   lattice (n_rows, n_cols and the same pixels
                                   pointer) and height; its doppler_out and
                                   spectrum_out are the sub-aperture's own.  No
                                   double-precision recheck (near-threshold cells
                                   are flagged RC_DET_NEAR_THRESHOLD).            */
  const float* w_sar;           /* host [n_chirps]: the chirp window w_sar[m] of
                                   Alg. 2 (Sec. III-B), finite; NULL: the plan's
                                   window.  Not with sub-apertures (their window
                                   spans the aperture).                           */
  const float* f_doppler;       /* device [n_rows * n_cols]: the Doppler index
                                   f_doppler(p) of Alg. 2 in bins, e.g. from a
                                   caller's own velocity estimate; NULL: the plan
                                   computes it from the mean velocity at the
                                   aperture centre (Sec. III-D).  Not with
                                   RC_DOPPLER_EXACT (Alg. 1 has no such table). */
  const void* data_host;        /* RC_MEMORY_BUDGET only: the input of `data`, in
                                   pinned host memory, with data = NULL; the plan
                                   copies it to the device.  NULL otherwise.      */
} rc_frame;

#define RC_DET_NEAR_THRESHOLD 1u  /* in the band, decided in single precision */
#define RC_DET_RECHECKED 2u       /* in the band, decided by the double-precision recheck */

typedef struct rc_detection {
  int32_t pixel;                /* flat lattice index row * n_cols + col          */
  float power;                  /* |P|^2                                          */
  float threshold;              /* alpha * mean(training cells)                   */
  uint32_t flags;               /* RC_DET_*                                       */
} rc_detection;

/* Create a plan.  Validates the descriptor (RC_EINVAL), sizes every frame slot
 * from its limits and allocates device and pinned host memory for all slots
 * up front (RC_ENOMEM if the total exceeds hbm_budget_bytes or an allocation
 * fails).  *out receives the plan; the caller destroys it with
 * rc_plan_destroy().  Uses the current HIP device. */
rc_status rc_plan_create(const rc_plan_desc* desc, void** out);

/* Bytes of device memory one frame slot of this descriptor needs. */
rc_status rc_plan_slot_bytes(const rc_plan_desc* desc, int64_t* bytes);

/* Bytes of device memory one frame (host descriptor, checked as by
 * rc_frame_validate) takes from the arena of a RC_MEMORY_BUDGET plan with this
 * descriptor: its interpolation table, geometry, pixel tables, partial images,
 * image (if image_out is NULL), CFAR buffers, detection list, recheck buffers
 * and, with data_host, its input.  Host only, no GPU.  The partial images
 * are counted for the default chirp split (rc_plan_tune below); a plan whose
 * tuning table gives the frame's class more blocks takes n_rows x n_cols x 8
 * bytes more per extra block from its arena. */
rc_status rc_frame_bytes(const rc_plan_desc* desc, const rc_frame* frame, int64_t* bytes);

/* Checks one frame (host) against a plan descriptor (host) exactly as
 * rc_process_batch() checks it before enqueuing anything, without a plan or a
 * GPU (no device pointer is dereferenced; q_tx, q_rx, vel and w_sar are
 * read).  RC_OK or RC_EINVAL with the reason in rc_last_error().  Besides the
 * limits and sizes this includes the phase range of the single-precision
 * forms (Alg. 2's exp(a2 d_hyp) takes the whole two-way path in wavelengths):
 * with RC_PREC_FP32, paths that can contribute - those whose index
 * a1 d_hyp + f_doppler can lie in [0, n_bins - 1] - must stay within 2^16
 * wavelengths, taking |f_doppler| <= 2 kd max|v| for the plan's own Doppler
 * table and for Alg. 1, and |f_doppler| <= n_bins - 1 for a caller's table
 * (which callers must respect); longer frames need RC_PREC_FP32_SPLIT. */
rc_status rc_frame_validate(const rc_plan_desc* desc, const rc_frame* frame);

/* Enqueue n_frames frames on stream (Alg. 2 pipeline, steps 1-4 above).
 * Each frame takes a free slot.  Sub-apertures of one stream are processed
 * in the order given (within the batch and across calls, on any streams:
 * the plan orders them with events); more than sliding_depth of one sensor
 * in flight (unreleased) gives RC_ENOTREADY, RC_SLIDE_NEXT without a started
 * stream or with sizes, lattice or height unlike the stream's RC_EINVAL.  Geometry is copied from the host arrays
 * before the call returns (through pinned staging), so they may be reused
 * at once; device inputs must stay valid until the frame completes.
 * Returns RC_ENOTREADY without enqueuing anything when fewer than n_frames
 * slots are free (or, under RC_MEMORY_BUDGET, fewer bytes of the arena than
 * the batch needs), RC_EINVAL on a frame outside the plan's limits or with
 * inconsistent sizes.  Kernel contributions whose interpolation index lies
 * outside [0, n_bins - 1] are zero, not an error. */
rc_status rc_process_batch(void* plan, const rc_frame* frames, int32_t n_frames,
                           void* stream);

/* Plan-time tuning of back-projection's chirp split, per size class.
 * Back-projection divides a frame's chirps into blocks (work items of one
 * launch) whose partial images are summed in block order.  By default the
 * block count follows a rule of the frame's size: about ten generations of
 * the GPU's waves, at least 512 chirp x channel rows a block, at most 16
 * blocks.  A size class is a frame's (n_rows, n_cols, n_chirps, n_channels).
 * The block count changes only the order in which a pixel's terms are
 * summed: a tuned class's images differ from the rule's by rounding, and
 * stay bitwise reproducible within the plan (and in any plan given the same
 * table), whatever batch a frame arrives in.  Sub-apertures of a continuous
 * stream always take the rule. */
typedef struct rc_tuning_entry {
  int32_t n_rows, n_cols;         /* the size class: lattice, ...                 */
  int32_t n_chirps, n_channels;   /* ... chirps and channels                      */
  int32_t chirp_blocks;           /* blocks the class takes, 1 .. min(16, n_chirps)*/
  int32_t default_blocks;         /* the rule's count (rc_plan_tune writes it)    */
  float ms_default;               /* rc_plan_tune: median frame time, rule's split */
  float ms_chosen;                /* rc_plan_tune: median frame time, chosen split */
} rc_tuning_entry;

/* Measures, for each size class among frames (host array; sub-apertures
 * refused), the device time per frame on stream of a batch of min(4, free
 * slots) copies of the class's first frame (fewer when an HBM-budget arena
 * holds fewer; rc_process_batch; one untimed
 * batch, then the median of three), so that the split suits frames that
 * share the GPU, with the rule's block count and with a quarter, half,
 * twice and four times as many (within 1 .. min(16, n_chirps) and the slots'
 * partial-image capacity); installs the fastest in the plan when it beats
 * the rule's by more than 2 % (else the rule's), and writes one entry per
 * class to out (host, cap entries), *n_out = number of classes.  The first
 * copy writes the frame's image_out, doppler_out and spectrum_out, the others
 * their slots' buffers; inputs must stay valid until the call returns.  The
 * copies take frame ids that no frame in flight has; the plan needs a free
 * slot and the call synchronizes stream.  RC_EINVAL on a frame the plan refuses, RC_ETRUNC
 * (nothing measured) when cap is below the number of classes, RC_ENOTREADY
 * when no slot is free.  Frames already in flight keep their split. */
rc_status rc_plan_tune(void* plan, const rc_frame* frames, int32_t n_frames, void* stream,
                       rc_tuning_entry* out, int32_t cap, int32_t* n_out);

/* Installs a tuning table (host; for instance the entries rc_plan_tune wrote
 * for another plan of the same descriptor): each entry's size class takes
 * its chirp_blocks; the other fields are ignored.  The table replaces the
 * plan's; n = 0 clears it.  RC_EINVAL, with the table unchanged, on a class
 * outside the plan's limits or a block count outside 1 .. min(16, n_chirps)
 * or beyond the slots' partial-image capacity.  Frames already in flight
 * keep their split. */
rc_status rc_plan_set_tuning(void* plan, const rc_tuning_entry* entries, int32_t n);

/* RC_OK if the frame's work is complete, RC_ENOTREADY if not, RC_ENOTFOUND. */
rc_status rc_poll(void* plan, int64_t frame_id);

/* Blocks until the frame completes, then copies its detections, in ascending
 * pixel order, to dst (host).  *n_out = number of detections.  If more than
 * cap exist, the first cap are copied and RC_ETRUNC is returned; if more than
 * the plan's max_detections exist, RC_ETRUNC is returned with *n_out = the
 * true count and max_detections entries are available. */
rc_status rc_detections(void* plan, int64_t frame_id, rc_detection* dst,
                        int64_t cap, int64_t* n_out);

/* Copies the frame's complex64 image (n_rows * n_cols) to dst (device) on
 * stream, after the frame's work.  RC_ETRUNC if cap_pixels is too small. */
rc_status rc_image(void* plan, int64_t frame_id, void* dst, int64_t cap_pixels,
                   void* stream);

/* Blocks until the frame completes; ms4 (host, float[4]) receives the device
 * time in milliseconds of range compression, the per-frame tables,
 * back-projection and detection (CFAR + compaction), measured with HIP events
 * recorded on the frame's stream around each stage.  A lone frame copied from
 * pinned memory in chirp-block pieces (RC_MEMORY_BUDGET) runs range
 * compression block by block inside back-projection: its range time reads 0
 * and its back-projection time includes range compression and the waits for
 * its pieces.  RC_EINVAL if the plan was created with stage_timing = 0. */
rc_status rc_stage_times(void* plan, int64_t frame_id, float* ms4);

/* Waits for the frame and returns its slot to the free pool. */
rc_status rc_frame_release(void* plan, int64_t frame_id);

/* Synchronises outstanding work and frees every resource of the plan. */
rc_status rc_plan_destroy(void* plan);

/* ---------------------------------------------------------------------------
 * One frame with no allocation.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Runs the
 * pipeline of rc_process_batch() (range compression, tables, back-projection,
 * CA-CFAR and ordered compaction) for one frame without a plan.  Every
 * intermediate lives in one scratch array the library holds on each GPU from
 * its load to the end of the process (RC_STATIC_SCRATCH_BYTES); the call makes
 * no hipMalloc, hipFree or pinned allocation.  The geometry is copied from the
 * host arrays with hipMemcpyAsync from pageable memory (read before the call
 * returns).
 *   desc        the settings of a plan (radar, windows, precision, Doppler
 *               mode, CFAR); its limits bound the frame as in rc_process_batch;
 *               max_rechecks and sliding_sensors must be 0;
 *   frame       as for rc_process_batch; image_out (device) is required;
 *               sliding must be RC_SLIDE_OFF;
 *   detections  device rc_detection[det_cap]: the first det_cap detections in
 *               ascending pixel order; n_det (device int64): their true count;
 *   stream      the HIP stream (NULL = default) every step is enqueued on.
 * Returns after enqueuing; the outputs are valid once the stream reaches the
 * end of the call.  RC_EINVAL for a frame that needs more than
 * RC_STATIC_SCRATCH_BYTES of scratch (interpolation table 16 B per chirp,
 * channel and bin; about 40 B per pixel plus 8 B per pixel and chirp block of
 * partial images), or more than 16384 chirp x channel rows, and for the
 * arguments rc_process_batch refuses.  All calls on one GPU share its scratch:
 * calls whose work overlaps on that GPU (other streams, other threads without
 * a stream order) race and give wrong results; nothing in the scratch needs to
 * start cleared, so calls in stream order are independent of each other. */
#define RC_STATIC_SCRATCH_BYTES (32 << 20)
rc_status rc_process_frame_static(const rc_plan_desc* desc, const rc_frame* frame,
                                  rc_detection* detections, int64_t det_cap, int64_t* n_det,
                                  void* stream);

/* Thread-local description of the last error ("" if none). */
const char* rc_last_error(void);

/* ---------------------------------------------------------------------------
 * Reconstruction grids (host functions, no GPU work).
 * ------------------------------------------------------------------------- */

/* Cartesian lattice (Sec. II reference grid): pixel (iy, ix) at
 * (x0 + ix dx, y0 + iy dy), row-major with y slow, written to xy (host,
 * float [ny * nx][2]); coordinates are evaluated in double, rounded once. */
rc_status rc_grid_cartesian(double x0, double dx, int32_t nx, double y0, double dy,
                            int32_t ny, float* xy);

/* Polar lattice parameters (Sec. III-E): the grid originates at the
 * synthetic-aperture centre (ox, oy); range step c / (2 B) / factor and
 * azimuth step lam / (2 L) / factor (L = aperture length, lam = c / f0);
 * theta is measured from +y towards +x; the lattice spans the range and
 * angle extent of the box [x0, x1] x [y0, y1] (which must lie at y > oy).
 * out6 receives {r0, dr, th0, dth, nr, nth}. */
rc_status rc_grid_polar_params(const rc_radar* radar, double x0, double x1, double y0,
                               double y1, double ox, double oy, double aperture_len,
                               double factor, double* out6);

/* Polar lattice points (ith, ir) -> (ox + r sin th, oy + r cos th) with
 * r = r0 + ir dr, th = th0 + ith dth, row-major with theta slow, written to
 * xy (host, float [nth * nr][2]). */
rc_status rc_grid_polar(double ox, double oy, double r0, double dr, int32_t nr,
                        double th0, double dth, int32_t nth, float* xy);

/* Magnitude of a polar-grid image at arbitrary points (Sec. III-E: the image
 * is formed on the polar lattice; showing it on the Cartesian reference grid,
 * as the comparison of Fig. 3 does, needs its magnitude at Cartesian points).
 *   polar_image  device, complex64 [nth][nr] (the layout rc_grid_polar gives
 *                the pixels: theta slow), e.g. a frame's image_out;
 *   ox, oy, r0, dr, th0, dth  the lattice (as from rc_grid_polar_params);
 *   points       device, float [n_points][2], metres;
 *   out          device, float [n_points].
 * For a point at range r and azimuth theta (from +y towards +x) around
 * (ox, oy), u = (r - r0) / dr and v = (theta - th0) / dth index the lattice;
 * |P| is interpolated bilinearly in (v, u), an index equal to the last one
 * takes that sample, and a point outside [0, nth - 1] x [0, nr - 1] gets 0.
 * Enqueued on `stream` (hipStream_t, NULL = default); the caller keeps the
 * buffers alive until it completes.  RC_EINVAL for null buffers, nth or
 * nr < 1, dr or dth not positive and finite, or n_points < 0. */
rc_status rc_resample_polar(const void* polar_image, int32_t nth, int32_t nr, double ox, double oy,
                            double r0, double dr, double th0, double dth, const void* points,
                            int64_t n_points, void* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RC_H_ */
