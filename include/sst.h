/*
 * sst.h -- C ABI of the shift-and-stack search for moving sources
 * ("synthetic tracking", Burdanov, Hasler & de Wit, MNRAS 2023,
 * arXiv:2303.07293), implemented with HIP kernels for AMD gfx950.
 *
 * The search (paper Sec. 1 and Sec. 2.1): stationary sources are removed
 * (here: each frame's mean is subtracted), linear motion is assumed with no
 * prior on position angle, each frame is shifted along a trial motion and the
 * frames are summed; tracks come back with their velocity, pixel coordinates
 * and S/N (Sec. 2.1).  Concretely, for a trial velocity v = (vx[a], vy[b]) in
 * px per time unit, frame i is sampled at integer offset
 *     d_i = llround(v * (t[i] - t_ref))      (round half away from zero)
 * and, for every pixel p of the w x h grid at t_ref,
 *     S'(p) = sum over in-frame samples, in ascending i, of F_i(p + d_i) - b_i
 *     c(p)  = number of in-frame samples     V(p) = sum of s2_i over them
 *     SN(p) = S'(p) / sqrt(V(p))   (-inf where c = 0, 0 where V = 0)
 * with b_i, s2_i the mean and population variance of frame i.  A candidate is
 * a pixel with c >= min_coverage, SN > threshold, whose key (SN, -raster
 * index) beats all in-grid 8-neighbours.  Where the paper is silent these
 * are readings: t_ref is an argument, shifts round half away from zero,
 * out-of-frame samples add nothing, the background is the frame mean and the
 * S/N is per pixel with no matched filter.
 *
 * Conventions for every entry point:
 *  - Memory: "dev" pointers are device memory of the current HIP device,
 *    "host" pointers are host memory.  The caller owns every buffer; the
 *    library keeps no per-call state and allocates no device memory (all
 *    scratch space is the caller's workspace `ws`).  The one-shot
 *    sst_stack and sst_detect copy their host-built shift tables into `ws`
 *    through one process-wide pinned host buffer (allocated on first use,
 *    grown when needed, kept until the process ends), so they return
 *    without waiting for that copy; they are not for graph capture (use a
 *    plan).
 *  - Layout: frames are C-contiguous [n][h][w]; velocity index k = b*nvx + a
 *    (vy major); stacks are [nvy][nvx][h][w].
 *  - Streams: work is enqueued on `stream` (a hipStream_t; NULL = the null
 *    stream) and the call returns after enqueueing, except where noted.
 *  - Errors: a negative SST_E_* code is returned and sst_last_error() gives
 *    a message.  All argument checks happen on the host before any device
 *    work is enqueued; a failed check enqueues nothing.
 *  - Time and velocity units are the caller's (hours and px/h in the
 *    examples); t must be strictly increasing and finite.
 */
#ifndef SST_H
#define SST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SST_OK 0
#define SST_E_ARG (-1)         /* null pointer, bad size, bad enum, NaN */
#define SST_E_UNSORTED (-2)    /* timestamps not strictly increasing */
#define SST_E_RANGE (-3)       /* a shift or size beyond the supported range */
#define SST_E_WORKSPACE (-4)   /* workspace missing or too small */
#define SST_E_DEVICE (-5)      /* a HIP runtime call failed */
#define SST_E_UNSUPPORTED (-6) /* valid request the library does not handle */

/* frame storage types.  16-bit frames carry a per-frame float32 scale s_i:
 * the frame value is the float32 product s_i * (stored value), and every
 * later step (statistics, stacking, S/N) works on those float32 values
 * exactly as on float32 frames; sums stay float32.  Storage only: the
 * search itself is not computed in 16 bits (with sst_set_half_search on,
 * staged searches of SST_F16 frames read the 16-bit samples and scale each
 * in a mixed-precision FMA into float32 sums). */
#define SST_F32 0
#define SST_BF16 1
#define SST_F16 2

/* operations (for sst_workspace_bytes) */
#define SST_OP_STACK 0
#define SST_OP_DETECT 1
#define SST_OP_STATS 2
#define SST_OP_QUANT 3
#define SST_OP_REFINE 4

/* plain-stack modes */
#define SST_SUM 0
#define SST_MEAN 1

/* One detection (paper Sec. 2.1: a track with its motion, pixel coordinates
 * and S/N).  32 bytes. */
typedef struct sst_candidate {
    int32_t ivx, ivy; /* indices into vx[], vy[] */
    int32_t x, y;     /* pixel on the frame grid at t_ref */
    float snr;        /* S'/sqrt(V) */
    float flux;       /* S': background-subtracted stacked flux */
    int32_t coverage; /* number of frames whose sample fell inside the frame */
    int32_t rank;     /* 0-based position in this velocity's list; -1 = unused slot */
} sst_candidate;

/* Integer shift table (host only, no device work).
 * out[i*nv + a] = llround(v[a] * (t[i] - t_ref)), one double product, no FMA.
 * t: host [n] strictly increasing; v: host [nv]; out: host [n][nv].
 * Errors: SST_E_ARG, SST_E_UNSORTED, SST_E_RANGE (|shift| >= 2^30). */
int sst_shift_table(const double* t, int n, double t_ref, const double* v, int nv, int32_t* out);

/* Bytes of device workspace an operation needs for this problem (0 on error,
 * with sst_last_error set).  op = SST_OP_STACK, SST_OP_DETECT, SST_OP_STATS,
 * SST_OP_QUANT or SST_OP_REFINE (the last three need only n, h, w);
 * the shift tables enter because the zero-padded frame copy is sized by the
 * largest shift.  k_max is used by SST_OP_DETECT only. */
size_t sst_workspace_bytes(int op, int n, int h, int w, const double* t, double t_ref,
                           const double* vx, int nvx, const double* vy, int nvy, int k_max);

/* Work-item shapes.  The stacking kernels are compiled for several
 * shapes of the work of one workgroup (4 waves, three per compute unit): a
 * tile of 64 x 32 pixels or one 64 x 16 row half of it, and a block of
 * VBX x VBY trial velocities (the velocity grid is padded to whole blocks;
 * a block's frame window is widened by the spread of its x shifts).
 * Shape 0: whole tiles, 6 x 2 velocities, x-shift spread up to 25 px over
 * the block; shape 1: the same with a window for spreads up to 80 px (grids
 * whose shifts grow faster per velocity step); shape 2: row halves, 12 x 2
 * velocities, spreads up to 48 px (a lower window shared by more
 * velocities, four workgroups per compute unit in the plain stack, a
 * float32 search in two passes: every work item stacked at four workgroups
 * per compute unit without the candidate code, then the items that hold a
 * pixel above threshold again in full; and more border pixels evaluated on
 * their own).  Every shape gives the same lists and stacks.  The one-shot
 * calls, sst_workspace_bytes and sst_plan_detect take the first of shapes
 * 2, 0, 1 whose window holds the grid's shifts (shape 2, on the direct
 * path, if none does).  sst_shape_info writes the block size of
 * `shape` (vbx/vby may be NULL) and returns the number of shapes, or
 * SST_E_ARG for an unknown shape.  A tuner may time plans of each. */
int sst_shape_info(int shape, int* vbx, int* vby);

/* sst_workspace_bytes for velocity-block shape `shape` (0 .. number of
 * shapes - 1, or -1 for the default choice of sst_workspace_bytes): the
 * shift tables are padded to whole blocks and the slots of a detect launch
 * hold whole block rows. */
size_t sst_workspace_bytes_shape(int op, int shape, int n, int h, int w, const double* t, double t_ref,
                                 const double* vx, int nvx, const double* vy, int nvy, int k_max);

/* 16-bit storage of float32 frames with a per-frame offset and scale (a
 * data-layout step before the search, not part of the paper's method):
 *   offset[i] = float32 of the float64 mean of frame i if center != 0, else 0
 *   scale[i]  = max_p |F_i(p) - offset[i]| * 2^-14   (1 for a constant frame)
 *   q[i][p]   = round-to-nearest-even of the float32 quotient
 *               fl32(F_i(p) - offset[i]) / scale[i]
 * in bfloat16 (dtype SST_BF16) or IEEE half (SST_F16), as raw 16-bit words.
 * |q| <= 2^14, so neither format overflows; IEEE half keeps 11 significant
 * bits and bfloat16 8.  The stored frame value is scale[i] * q (pass q and
 * scale to the search as 16-bit frames); with center != 0 it is the frame
 * minus its offset, which leaves every S/N unchanged (the search removes
 * each frame's mean) while the rounding error scales with |F - mean| rather
 * than |F|.  Add offset[i] back for absolute levels.
 * frames: dev float32 [n][h][w] (finite); q: dev uint16 [n][h][w];
 * scale: dev float32 [n]; offset: dev float32 [n], written only when
 * center != 0 (may be NULL otherwise).
 * ws: dev, >= sst_workspace_bytes(SST_OP_QUANT, ...).
 * Errors: SST_E_ARG (NULL pointer, dtype not 16-bit, bad size),
 * SST_E_WORKSPACE.  Asynchronous on `stream`. */
int sst_quantize(const float* frames, int n, int h, int w, int dtype, int center, void* q, float* scale,
                 float* offset, void* ws, size_t ws_bytes, void* stream);

/* Per-frame statistics (the S/N normaliser's inputs): stats[2i] = mean of
 * frame i, stats[2i+1] = population variance, both float64, dev [n][2].
 * frames: dev [n][h][w] of `dtype`; scale: dev [n] per-frame multiplier for
 * SST_BF16/SST_F16 storage (frame value = scale[i] * stored value), NULL for
 * SST_F32.  ws: dev, >= sst_workspace_bytes(SST_OP_STATS, ...). */
int sst_frame_stats(const void* frames, int dtype, const float* scale, int n, int h, int w,
                    double* stats, void* ws, size_t ws_bytes, void* stream);

/* Plain shift-and-stack of every trial velocity (paper Sec. 2.1).
 * out: dev float32 [nvy][nvx][h][w]:
 *   SST_SUM : sum over in-frame samples of (F_i(p + d_i) - bg[i])
 *   SST_MEAN: that sum / c(p), 0 where c(p) = 0
 * bg: host [n] per-frame values to subtract, or NULL for none.
 * cov: dev int32 [nvy][nvx][h][w] receiving c(p), or NULL.
 * t, vx, vy: host.  Asynchronous on `stream`. */
int sst_stack(const void* frames, int dtype, const float* scale, int n, int h, int w,
              const double* t, double t_ref, const double* vx, int nvx, const double* vy, int nvy,
              const double* bg, int mode, float* out, int32_t* cov,
              void* ws, size_t ws_bytes, void* stream);

/* Shift-and-stack + S/N + peak extraction with per-velocity candidate lists.
 * cand: dev [nvy*nvx][k_max]; list k holds min(count[k], k_max) candidates
 *   sorted by (SN descending, raster index ascending); unused slots have
 *   rank = -1.
 * count: dev int32 [nvy*nvx], number of candidates before truncation.
 * threshold: S/N cut (strict >); min_coverage <= 0 means ceil(n/2) (the
 *   paper's pipeline only finds a mover seen in half or more of a group's
 *   frames, Sec. 2.1).
 * k_max in [1, 1024].  frame_stats: host [n][2] receiving each frame's mean
 *   and variance, or NULL; when non-NULL the call waits for the stream.
 * Asynchronous on `stream` otherwise. */
int sst_detect(const void* frames, int dtype, const float* scale, int n, int h, int w,
               const double* t, double t_ref, const double* vx, int nvx, const double* vy, int nvy,
               float threshold, int min_coverage, int k_max,
               sst_candidate* cand, int32_t* count, double* frame_stats,
               void* ws, size_t ws_bytes, void* stream);

/* sst_detect for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same search and results, with the library's own static device scratch of
 * sst_noalloc_scratch_bytes() bytes (256 MiB) as the workspace instead of
 * a caller's.  Each GPU the library runs on holds one such array until the
 * process ends; its address is looked up on the first call on a device.
 * All calls on one GPU share that array, so calls on one GPU that overlap in
 * time (other host threads, other streams) race; nothing needs clearing
 * between calls (every region the search reads is written by the same call
 * first).  Arguments as for sst_detect without ws/ws_bytes.  Errors: as
 * sst_detect; SST_E_WORKSPACE when the problem needs more workspace than
 * the scratch holds (sst_workspace_bytes(SST_OP_DETECT, ...) > the size),
 * checked before any device work.  The call allocates nothing on the
 * device (it waits for `stream` once, for the shift-table upload). */
int sst_detect_noalloc(const void* frames, int dtype, const float* scale, int n, int h, int w,
                       const double* t, double t_ref, const double* vx, int nvx, const double* vy, int nvy,
                       float threshold, int min_coverage, int k_max,
                       sst_candidate* cand, int32_t* count, double* frame_stats, void* stream);
size_t sst_noalloc_scratch_bytes(void);

/* ---- prepared searches: set-up once, enqueue-only runs ----
 * A run of a prepared plan enqueues kernels only: no host synchronisation,
 * no allocation and no memset, so it may be captured into a hipGraph (for
 * example many fields of a night in one graph) and replayed; replays read
 * the frames and write cand/count at the addresses given when captured. */
typedef struct sst_plan sst_plan;

/* Prepare sst_detect for one geometry (frame count and size, timestamps,
 * velocity grid) and detection settings.  Validates the arguments as
 * sst_detect does, computes the shift tables and uploads them into `ws`
 * (waits for `stream` once).  ws: dev, >= sst_workspace_bytes(SST_OP_DETECT,
 * ...); it belongs to the plan until sst_plan_destroy: do not use it for
 * other calls meanwhile.  *plan receives a host object (free it with
 * sst_plan_destroy).  Errors: as sst_detect. */
int sst_plan_detect(int n, int h, int w, const double* t, double t_ref, const double* vx, int nvx,
                    const double* vy, int nvy, float threshold, int min_coverage, int k_max,
                    void* ws, size_t ws_bytes, void* stream, sst_plan** plan);

/* sst_plan_detect with velocity-block shape `shape` (-1: the default choice
 * of sst_plan_detect; ws >= sst_workspace_bytes_shape(SST_OP_DETECT, shape,
 * ...)). 
 * Every shape gives the same candidate lists bit for bit; only the time
 * differs.  Errors: as sst_plan_detect, SST_E_ARG for an unknown shape. */
int sst_plan_detect_shape(int shape, int n, int h, int w, const double* t, double t_ref, const double* vx,
                          int nvx, const double* vy, int nvy, float threshold, int min_coverage, int k_max,
                          void* ws, size_t ws_bytes, void* stream, sst_plan** plan);

/* What a plan does: its shape, whether its velocity blocks are staged in
 * LDS (1) or read through L2 (0, much slower: blocks too spread for the
 * staging window, or padded frames of more than 2^31 bytes, which the
 * staged path's 31-bit offsets cannot address), and its stacking launches
 * per run (chunks of block
 * rows).  Any pointer may be NULL.  Errors: SST_E_ARG (plan NULL). */
int sst_plan_info(const sst_plan* plan, int* shape, int* staged, int* launches);

/* The search of sst_detect for frames of the prepared geometry (same
 * results bit for bit).  frames/dtype/scale/cand/count as for sst_detect.
 * Runs of plans that share a workspace must not overlap in time.
 * Errors: SST_E_ARG, SST_E_DEVICE (launch failures). */
int sst_plan_run(const sst_plan* plan, const void* frames, int dtype, const float* scale,
                 sst_candidate* cand, int32_t* count, void* stream);

/* Free a plan (NULL is ignored).  The workspace is the caller's again. */
void sst_plan_destroy(sst_plan* plan);

/* ---- batches of prepared searches: one persistent launch per round ----
 * Many fields of uneven frame count, size and velocity grid (the paper's
 * image groups of a night, Sec. 2.1 and 2.3) searched together: the
 * stacking work of all plans runs as persistent launches whose workgroups
 * take (tile, velocity block) items of any plan from work queues, one
 * launch per round (round r: chunk r of the velocity-block rows of every
 * plan that has one), each followed by the plans' merges.  Results are
 * those of sst_plan_run for each plan, bit for bit.  Plans whose velocity
 * blocks are too spread for LDS staging run on their own within the run. */
typedef struct sst_batch sst_batch;

/* Device workspace bytes of a batch's tables (0 and an error if a plan
 * pointer is NULL or nplans <= 0). */
size_t sst_batch_workspace_bytes(const sst_plan* const* plans, int nplans);

/* Build a batch of nplans plans (host array of plan pointers; the plans
 * must outlive the batch).  ws: dev, >= sst_batch_workspace_bytes, 256-byte
 * aligned; it holds the work tables, written here (waits for `stream`
 * once), and belongs to the batch until sst_batch_destroy.  The batch also
 * creates three streams (default priority) and four events on the current
 * device.  *batch receives a host object.  Errors: SST_E_ARG, SST_E_WORKSPACE, SST_E_RANGE (more
 * than 2^31 - 1 items in a round), SST_E_DEVICE. */
int sst_batch_create(const sst_plan* const* plans, int nplans, void* ws, size_t ws_bytes, void* stream,
                     sst_batch** batch);

/* Run every plan of the batch on its frames: host arrays of nplans entries
 * (frames[j], dtypes[j], scales[j] or scales == NULL for float32 frames,
 * cand[j], count[j], each as for sst_plan_run with plan j).  Enqueues
 * kernels only (no host synchronisation, allocation or memset; the queue
 * counters are cleared by a kernel): the plans' preparation kernels and
 * merges are spread over three streams of the batch, forked from `stream`
 * and joined back to it with events, so a run may be captured into a graph
 * from `stream`.  Runs of one batch, or of batches sharing plans, must not
 * overlap in time.  Errors: SST_E_ARG, SST_E_DEVICE. */
int sst_batch_run(const sst_batch* batch, const void* const* frames, const int* dtypes, const float* const* scales,
                  sst_candidate* const* cand, int32_t* const* count, void* stream);

/* Free a batch (NULL is ignored).  Its workspace is the caller's again. */
void sst_batch_destroy(sst_batch* batch);

/* Sub-pixel refinement of detections by gradient ascent on a differentiable
 * stacked S/N.  The search returns tracks on its integer grid (paper Sec.
 * 2.1); here theta = (x0, y0, vx, vy) is continuous.  For each candidate a
 * cutout x cutout stack is sampled bilinearly along the track,
 *   Cut(u,v) = sum_i bilin(F_i - b_i; x0 + u + vx dt_i, y0 + v + vy dt_i),
 *   dt_i = t[i] - t_ref, u, v in [-R, R], R = cutout / 2,
 * frame values outside the frame count as 0 (as in the search), b_i the
 * frame means; the objective is the PSF-weighted S/N
 *   SN = sum w(u,v) Cut(u,v) / sqrt(sum w(u,v)^2 * sum_i s2_i),
 *   w = Gaussian of the given FWHM centred on the track,
 * whose normaliser does not depend on theta (0 if every frame is constant).
 * Its gradient is exact almost everywhere (bilinear sampling is piecewise
 * linear; at an integer sample position the right derivative is taken).
 * `steps` ascent steps theta <- theta + lr * grad SN are taken inside the
 * call; steps = 0 only evaluates.  On return params holds the final theta,
 * snr[c] = SN(theta) and grad[c] = dSN/dtheta at that theta.
 * Arithmetic: float32 sums; float64 only in the frame statistics.
 * frames: dev [n][h][w] of dtype (scale as for sst_detect); t: host [n];
 * params: dev float32 [n_cand][4] (in/out); snr: dev float32 [n_cand];
 * grad: dev float32 [n_cand][4] or NULL.  cutout odd in 1..63; fwhm > 0.
 * ws: dev, >= sst_workspace_bytes(SST_OP_REFINE, ...).  The call waits for
 * the stream once (upload of the time offsets).
 * Errors: SST_E_ARG, SST_E_UNSORTED, SST_E_WORKSPACE, SST_E_DEVICE. */
int sst_refine(const void* frames, int dtype, const float* scale, int n, int h, int w,
               const double* t, double t_ref, int n_cand, float* params, int cutout, float fwhm,
               int steps, float lr, float* snr, float* grad, void* ws, size_t ws_bytes, void* stream);

/* ---- steps the paper runs before the search (float32 frames) ----
 * out must not overlap frames in any of the three. */

/* Static-source removal (paper Sec. 2.1: the median combination of a group's
 * frames is removed from each frame, leaving moving sources):
 *   med(p)    = median over i of F_i(p)  (odd n: the middle value; even n:
 *               the float32 mean of the two middle values, (a + b) * 0.5)
 *   out_i(p)  = F_i(p) - med(p)          (one float32 subtraction)
 * frames, out: dev float32 [n][h][w]; median: dev float32 [h][w] receiving
 * med, or NULL.  n <= 256 (SST_E_UNSUPPORTED beyond).  Finite input.
 * Errors: SST_E_ARG, SST_E_UNSUPPORTED, SST_E_DEVICE.  Asynchronous. */
int sst_median_subtract(const float* frames, int n, int h, int w, float* out, float* median, void* stream);

/* Co-adding (paper Sec. 2.1 and 2.2: every N consecutive frames are summed
 * into one longer exposure for the slow-mover search):
 *   out[g][p] = sum over j < group, ascending j, of F[g*group + j][p]  (float32)
 * for the n / group complete groups (trailing frames that do not fill a
 * group are not used).  t: host [n] or NULL; t_out: host [n / group]
 * receiving each group's mean timestamp (float64), or NULL (needs t).
 * frames: dev float32 [n][h][w]; out: dev float32 [n / group][h][w].
 * Errors: SST_E_ARG (group outside 1..n, NULL pointers, non-finite t),
 * SST_E_DEVICE.  Asynchronous on `stream` (t_out is written before return). */
int sst_coadd(const float* frames, int n, int h, int w, int group, float* out, const double* t, double* t_out,
              void* stream);

/* 2x2 binning (paper Sec. 2.3: binned frames for the fast-mover search):
 *   out[i][y][x] = (F[2y][2x] + F[2y][2x+1]) + (F[2y+1][2x] + F[2y+1][2x+1])
 * summed in float32 in that order; an odd last row or column is dropped.
 * frames: dev float32 [n][h][w] (h, w >= 2); out: dev float32
 * [n][h/2][w/2].  Errors: SST_E_ARG, SST_E_DEVICE.  Asynchronous. */
int sst_bin2x2(const float* frames, int n, int h, int w, float* out, void* stream);

/* Search of IEEE-half frames on their 16-bit samples (process-wide, off by
 * default; returns the previous setting).  Off, sst_detect and plan runs
 * widen 16-bit frames (with their scales) into the float32 padded copy and
 * search that, as for float32 frames.  On, a staged plan given SST_F16
 * frames stages the 16-bit samples themselves (half the bytes into LDS and
 * out of it) and adds each as one mixed-precision FMA, fma(q, scale_i, S),
 * subtracting the covering frames' means after the sum (a prefix sum of the
 * means, as for the variances); the candidate lists follow the same parity
 * rules against the oracle on the dequantised frames.  It is off by default
 * because on gfx950 the mixed-precision FMA issues at under half the rate of
 * a float32 add, which costs more than the halved LDS traffic saves on the
 * full-field search (about 20 ms against 16.4 ms).  Not used by batches. */
int sst_set_half_search(int on);

/* Work-item shape of sst_stack and its sst_workspace_bytes (process-wide;
 * -1, the default, chooses automatically: shape 2 when its window holds the
 * grid's shifts, whose plain-stack kernel runs four workgroups per compute
 * unit, else shape 0, else 1).  Writes the previous setting to *previous
 * (if not NULL) and returns SST_OK, or SST_E_ARG (setting unchanged) for a
 * shape outside -1 .. number of shapes - 1.  Every shape writes the same
 * stacks; the setting exists to test and time each.  Set it before sizing
 * the workspace of the calls it applies to. */
int sst_set_stack_shape(int shape, int* previous);

/* Two-pass search of shape 2 (process-wide).  A float32 search of shape 2
 * runs in two passes: the first stacks every work item at four workgroups
 * per compute unit and only marks the items that hold a pixel above
 * threshold (once more than one in eight of the items dealt so far are
 * marked, it marks the rest without running them); the second runs the
 * marked items in full.  SST_TWO_PASS_AUTO (the default) does so for
 * launches of at least 4096 work items, SST_TWO_PASS_NEVER never,
 * SST_TWO_PASS_ALWAYS for every launch.  Writes the previous setting to
 * *previous (if not NULL) and returns SST_OK, or SST_E_ARG (setting
 * unchanged) for another mode.  A run takes the mode in force when it is
 * enqueued (a captured graph keeps the mode of its capture).  Every mode
 * gives the same lists; the setting exists to test and time each.  The
 * persistent batch (sst_batch_run) runs one pass. */
#define SST_TWO_PASS_NEVER 0
#define SST_TWO_PASS_AUTO 1
#define SST_TWO_PASS_ALWAYS 2
int sst_set_two_pass(int mode, int* previous);

/* Candidate entries each (tile, row half, velocity) of a detect launch
 * keeps, at most (process-wide, for plans and calls prepared from now on;
 * 0 restores the automatic choice; returns the previous setting).  The
 * automatic choice keeps k_max when the whole grid's slots fit 256 MiB,
 * else what fits, but at least 4 (the full field, 81 x 81 velocities over
 * 1024 x 1024 pixels, keeps 4).  A velocity whose kept entries may miss one
 * of its k_max best (a slot found more candidates than it kept, and the
 * last kept ranks among the list's first k_max) is recomputed exactly after
 * the merge, so the setting changes memory and time, never the lists; it
 * exists to test and tune that path. */
int sst_set_slot_keep(int kt);

/* Kernel timing for measurements.  Between sst_profile_begin() and
 * sst_profile_end(), every launch of the stacking kernel (the dominant cost
 * of sst_stack and sst_detect) is bracketed by HIP events recorded on the
 * launch stream.  sst_profile_end waits for those events and returns the
 * summed kernel time in milliseconds and the number of launches (either
 * pointer may be NULL).  Process-wide state: do not overlap profiled calls
 * from several host threads.  Errors: SST_E_DEVICE, SST_E_RANGE (more than
 * 4096 launches in one profiled interval). */
int sst_profile_begin(void);
int sst_profile_end(double* stack_ms, int* stack_launches);

/* Message of the last error on the calling thread ("" if none). */
const char* sst_last_error(void);

/* Library version string. */
const char* sst_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SST_H */
