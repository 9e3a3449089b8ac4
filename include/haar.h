/*
 * haar.h -- C ABI of libhaar, the fast (polyphase) Haar wavelet transform
 * for AMD Instinct MI355X (gfx950).
 *
 * The transform (Ashok et al., "The Fast Haar Wavelet Transform for Signal &
 * Image Processing"):
 *   analysis bank, Sec. III, Eq. (11)-(12), Fig. 4: the input is split into
 *   its two polyphase components first and only the decimated outputs are
 *   computed; every pair (x0, x1) = (x[2m], x[2m+1]) gives
 *       a[m] = (x0 + x1) / sqrt2,      d[m] = (x1 - x0) / sqrt2;
 *   synthesis bank, Sec. IV, Eq. (19), Fig. 7: the exact inverse,
 *       x[2m] = (a[m] - d[m]) / sqrt2, x[2m+1] = (a[m] + d[m]) / sqrt2;
 *   Fig. 8: the two together reconstruct the input exactly.
 * Multi-level transforms recurse on the approximation (dyadic), and 2D
 * transforms apply one level along every row (width) of the current LL
 * region and then along every column (height).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every data pointer is a DEVICE pointer on the current HIP device,
 *   allocated and owned by the caller.  Tensors are contiguous, row-major and
 *   batch-major: 1D [batch][length], 2D [batch][height][width].
 * Layout.  Outputs have the shape of the inputs ("packed Mallat" layout).
 *   1D: [a_L | d_L | d_{L-1} | ... | d_1] with |a_j| = ceil(n_{j-1}/2),
 *   |d_j| = floor(n_{j-1}/2), n_0 = length.  2D, per level on the current
 *   h x w LL region: LL = rows [0, ceil(h/2)) x cols [0, ceil(w/2)),
 *   HL (high along width) = rows [0, ceil(h/2)) x cols [ceil(w/2), w),
 *   LH (high along height) = rows [ceil(h/2), h) x cols [0, ceil(w/2)),
 *   HH = the rest; the next level works on LL.
 * Odd lengths.  When a level sees an odd count, its last sample passes
 *   unscaled into the approximation and has no detail (the transform stays
 *   orthonormal; it equals the usual Haar transform when 2^L divides the
 *   size).
 * Types.  dtype selects the STORAGE type of input and output (haar_dtype).
 *   Reduced-precision results are rounded to nearest even.  Arithmetic:
 *   the 1D and 2D transforms, the fused shrinkage and the direct bank
 *   compute in FP32 (the approximation path of the analysis carries a
 *   compensated FP32 pair); the 3D transforms compute in FP64 on the device
 *   (the approximation grows by 2^(3/2) per level, and FP64 keeps every sum
 *   exact at the cost of unpacked-FP32 issue rate; the last synthesis level
 *   into 16-bit storage runs in FP32); haar_l1_grad_2d computes the
 *   transform in FP32 and sums the loss in FP64.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *   stream).  Calls are asynchronous: they enqueue kernels and return; they
 *   never synchronise.  Device faults surface at the caller's next
 *   synchronisation.
 * Errors.  Every function returns a haar_status.  Argument checks run before
 *   any HIP call, so an invalid call enqueues nothing.  On a non-OK return,
 *   haar_last_error() holds a message (thread-local).
 * Aliasing.  Out-of-place only: overlapping input and output ranges return
 *   HAAR_ERR_ALIAS (the fused tiles write into other tiles' input ranges).
 * Levels.  0 <= levels <= haar_max_levels_1d(length) (1D),
 *   haar_max_levels_2d(height, width) (2D) or haar_max_levels_3d (3D);
 *   levels = 0 copies.  batch = 0
 *   enqueues nothing and returns HAAR_OK.
 * Threading.  All entry points are reentrant; the tuning table is guarded by
 *   a mutex.
 * Scratch.  Most calls allocate nothing.  haar_l1_grad_2d keeps its tile
 *   loss partials in stream-ordered scratch.  Four more cases keep intermediate
 *   values in stream-ordered scratch obtained with hipMallocAsync on `stream`
 *   and released with hipFreeAsync on the same stream: 2D transforms deeper
 *   than one fused pass (levels > 5); 3D transforms deeper than one fused
 *   pass (levels > 3); 1D analyses deeper than one chunk
 *   (levels > 12 at the default 4096-sample chunk) in BF16/FP16 storage (one
 *   FP32 value per chunk) or on more than 1024 chunks per signal; and 1D
 *   syntheses more than 24 levels deeper than one chunk.
 * Deep 1D.  A 1D analysis deeper than one chunk runs as two kernels: the
 *   chunks, then one work-group per signal computing the remaining levels of
 *   the chunk approximations on chip.  The matching synthesis is one kernel:
 *   every chunk derives its own deepest approximation from a_L along its
 *   ancestor path.
 */
#ifndef HAAR_H_
#define HAAR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HAAR_F32 = 0,   /* IEEE binary32 storage               */
    HAAR_BF16 = 1,  /* bfloat16 storage, FP32 arithmetic    */
    HAAR_F16 = 2    /* IEEE binary16 storage, FP32 arithmetic */
} haar_dtype;

typedef enum {
    HAAR_OK = 0,
    HAAR_ERR_NULL = 1,        /* a required pointer is NULL                        */
    HAAR_ERR_DTYPE = 2,       /* dtype is not a haar_dtype                         */
    HAAR_ERR_SHAPE = 3,       /* a size < 1, batch < 0, or a size too large        */
    HAAR_ERR_LEVELS = 4,      /* levels outside [0, max levels]                   */
    HAAR_ERR_ALIAS = 5,       /* input and output byte ranges overlap              */
    HAAR_ERR_WORKSPACE = 6,   /* workspace NULL, too small or misaligned           */
    HAAR_ERR_HIP = 7,         /* a HIP runtime call failed (see haar_last_error)   */
    HAAR_ERR_PLAN = 8,        /* NULL / not uploaded plan, or an invalid plan item */
    HAAR_ERR_UNSUPPORTED = 9, /* valid arguments the library does not implement    */
    HAAR_ERR_ARG = 10         /* an argument value is invalid (mode, threshold)    */
} haar_status;

/* ------------------------------------------------------------------------
 * Plain transforms.
 * ------------------------------------------------------------------------ */

/* Multi-level 1D analysis (Sec. III, Eq. (11)-(12), Fig. 4, recursed on the
 * approximation).  x: [batch][length] input, y: [batch][length] output in
 * the packed layout.  Both device pointers, caller-owned, not overlapping. */
int haar_fwd_1d(const void* x, void* y, int64_t length, int32_t levels,
                int64_t batch, int32_t dtype, void* stream);

/* Multi-level 1D synthesis (Sec. IV, Eq. (19), Fig. 7): the exact inverse
 * (and, the transform being orthonormal, the adjoint) of haar_fwd_1d.
 * y: packed coefficients [batch][length], x: reconstruction. */
int haar_inv_1d(const void* y, void* x, int64_t length, int32_t levels,
                int64_t batch, int32_t dtype, void* stream);

/* Multi-level separable 2D analysis (rows, then columns, per level; Fig. 4
 * along each axis; the lowpass image of Sec. V is the LL band).
 * x: [batch][height][width], y: same shape, packed quadrant layout. */
int haar_fwd_2d(const void* x, void* y, int64_t height, int64_t width,
                int32_t levels, int64_t batch, int32_t dtype, void* stream);

/* Multi-level separable 2D synthesis: exact inverse / adjoint of
 * haar_fwd_2d (columns, then rows, per level, from level L down to 1). */
int haar_inv_2d(const void* y, void* x, int64_t height, int64_t width,
                int32_t levels, int64_t batch, int32_t dtype, void* stream);

/* Multi-level separable 3D analysis of volumes (the paper's medical-image
 * application, Sec. I and Sec. V, carried to three axes): per level one 1D
 * level (Sec. III, Eq. (11)-(12), Fig. 4) along every x line (width), then
 * every y line (height), then every z line (depth) of the current LLL
 * region; recursion on LLL.  x: [batch][depth][height][width], y: same
 * shape, packed octant layout: after level j the region D_{j-1} x H_{j-1} x
 * W_{j-1} is split at D_j = ceil(D_{j-1}/2), H_j, W_j, and the octant that
 * is high-pass along a set of axes lies on the high side of those axes.
 * Odd counts carry their last sample unscaled on each axis.  Three levels
 * are fused per pass; deeper transforms allocate stream-ordered scratch of
 * 8 bytes per element of the level-3 LLL region (twice).  Arithmetic is
 * FP64 on the device (samples are widened, every output is rounded once). */
int haar_fwd_3d(const void* x, void* y, int64_t depth, int64_t height,
                int64_t width, int32_t levels, int64_t batch, int32_t dtype,
                void* stream);

/* Multi-level separable 3D synthesis (Sec. IV, Eq. (19), Fig. 7 along z,
 * then y, then x per level, levels L..1): exact inverse and adjoint of
 * haar_fwd_3d.  y: packed coefficients, x: reconstruction, same shape. */
int haar_inv_3d(const void* y, void* x, int64_t depth, int64_t height,
                int64_t width, int32_t levels, int64_t batch, int32_t dtype,
                void* stream);

/* ------------------------------------------------------------------------
 * Fused shrinkage: analysis, thresholding of the detail coefficients,
 * synthesis, in ONE pass over HBM (each element is read once and written
 * once, against three passes for haar_fwd_*, an elementwise step and
 * haar_inv_*).  This is the decompose / act on the coefficients /
 * reconstruct pipeline of the applications named in Sec. I (compression,
 * signal and image analysis) and Sec. VI (biosignals, medical images).
 *
 * Every detail coefficient of level j (1D: d_j; 2D: HL_j, LH_j, HH_j) is
 * replaced with
 *   HAAR_SHRINK_HARD: d if |d| > t, else 0     (keep the large coefficients)
 *   HAAR_SHRINK_SOFT: sign(d) * max(|d| - t, 0) (shrink every coefficient)
 * with t = thresholds[j - 1]; the approximation a_L / LL_L is kept.  The
 * coefficients stay in FP32 on chip between the analysis and the synthesis;
 * only the output is rounded to the storage type.
 *
 * x, y: device pointers, [batch][length] or [batch][height][width], storage
 * dtype, out-of-place (overlap returns HAAR_ERR_ALIAS).  thresholds: HOST
 * array of `levels` floats, read during the call (may be NULL when levels
 * is 0), each >= 0 (+inf allowed); a negative or NaN threshold or an unknown
 * mode returns HAAR_ERR_ARG.  Fused depth: 1D levels <= 12 (one 4096-sample
 * chunk per work-group), 2D levels <= 5 (one 32-row tile per work-group);
 * deeper requests return HAAR_ERR_UNSUPPORTED.  levels = 0 copies.  The
 * calls allocate nothing and never synchronise.
 * ------------------------------------------------------------------------ */
typedef enum {
    HAAR_SHRINK_HARD = 0,
    HAAR_SHRINK_SOFT = 1
} haar_shrink_mode;

int haar_shrink_1d(const void* x, void* y, int64_t length, int32_t levels,
                   int64_t batch, int32_t dtype, int32_t mode,
                   const float* thresholds, void* stream);
int haar_shrink_2d(const void* x, void* y, int64_t height, int64_t width,
                   int32_t levels, int64_t batch, int32_t dtype, int32_t mode,
                   const float* thresholds, void* stream);

/* Fused training step of a sparsity loss through the 2D transform, in ONE
 * pass over HBM.  With c = W x the analysis of each item (haar_fwd_2d):
 *   loss  = sum |c| over the detail bands of levels 1..L
 *           + 0.5 * sum c^2 over LL_L,
 *   dloss/dc = sign(c) on the details (sign(0) = 0), c on LL_L,
 *   grad_x = W^T dloss/dc, the synthesis bank (Sec. IV, Eq. (19)) applied
 *            to dloss/dc: the transform is orthonormal, W^T = W^-1.
 * x, grad_x: [batch][height][width] device tensors of `dtype`, caller-owned,
 * not overlapping.  loss: device array of `batch` doubles, one loss per
 * item, written by the call (the tile partial sums are reduced in a fixed
 * order, so repeated calls agree bit for bit).  1 <= levels <=
 * min(5, haar_max_levels_2d): HAAR_ERR_LEVELS beyond the transform's depth,
 * HAAR_ERR_UNSUPPORTED for levels 0 or beyond one fused tile (5).  Uses
 * stream-ordered scratch of 8 bytes per tile (about 8 bytes per 8192 FP32
 * elements). */
int haar_l1_grad_2d(const void* x, void* grad_x, double* loss, int64_t height,
                    int64_t width, int32_t levels, int64_t batch,
                    int32_t dtype, void* stream);

/* The same training step without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc.  Arguments, results and
 * errors are those of haar_l1_grad_2d; the tile loss partials live in a
 * static device array of the library (2^19 doubles = 4 MiB, held on every
 * GPU the library runs on until the process ends) instead of stream-ordered
 * scratch.  One partial per tile: tiles are 32 rows x 128 columns (FP32) or
 * 32 x 256 (BF16/FP16), counting partial tiles at the right and bottom
 * edges, times batch; a call needing more than 2^19 returns
 * HAAR_ERR_WORKSPACE before enqueueing anything.  Calls that overlap in time
 * on one GPU share the array and race: serialise them (one stream, or
 * events).  The first call on a device looks the array's address up with
 * hipGetSymbolAddress (no allocation); nothing is enqueued for that. */
int haar_l1_grad_2d_noalloc(const void* x, void* grad_x, double* loss,
                            int64_t height, int64_t width, int32_t levels,
                            int64_t batch, int32_t dtype, void* stream);

/* ------------------------------------------------------------------------
 * The direct ("original") filter bank, for comparison with the fast bank.
 * Analysis per level (Fig. 1 / Fig. 2, taps of Eq. (8)-(9)): convolve the
 * approximation with b0 = [1, 1]/sqrt2 and b1 = [1, -1]/sqrt2 at the full
 * rate, then decimate (keep the odd phase, pairs aligned at even indices).
 * Synthesis per level (Fig. 5, Eq. (13), taps of Eq. (17)-(18)): up-sample
 * both channels by zero insertion, filter with a0 = [1, 1]/sqrt2 and
 * a1 = [-1, 1]/sqrt2, add.  Odd counts carry as in the fast bank, so the
 * results equal haar_fwd_1d / haar_inv_1d (up to FP32 rounding).
 * Every stage is a pass over the workspace, which holds the full-rate
 * streams: the work the fast bank avoids by computing only the decimated
 * outputs.  Plain FP32 arithmetic; x, y device pointers as in the plain
 * calls; inverse = 0 analysis, 1 synthesis.  workspace: caller-owned device
 * memory of at least haar_direct_workspace_size(length, batch) bytes,
 * 4-byte aligned (HAAR_ERR_WORKSPACE otherwise).
 * ------------------------------------------------------------------------ */
size_t haar_direct_workspace_size(int64_t length, int64_t batch);
int haar_direct_1d(const void* x, void* y, int64_t length, int32_t levels,
                   int64_t batch, int32_t dtype, int32_t inverse,
                   void* workspace, size_t workspace_bytes, void* stream);

/* ceil(log2(length)) for length >= 1 (0 for length 1); -1 if length < 1.
 * Beyond this depth every further level would be a no-op. */
int haar_max_levels_1d(int64_t length);

/* ceil(log2(max(height, width))); -1 if a size < 1. */
int haar_max_levels_2d(int64_t height, int64_t width);

/* ceil(log2(max(depth, height, width))); -1 if a size < 1. */
int haar_max_levels_3d(int64_t depth, int64_t height, int64_t width);

/* ------------------------------------------------------------------------
 * Batched transforms of uneven sizes (many signals or images of different
 * lengths / shapes in one launch).
 *
 * A plan lists the work units of all items (2D: tiles, 1D: chunks of 4096
 * samples), largest items first, and haar_plan_execute() enqueues ONE
 * kernel that drains the list, under one of the schedules of
 * haar_plan_set_config: a persistent grid (the resident work-groups of the
 * device) walking the list with a stride, a persistent grid claiming units
 * from an atomic counter, or one work-group per unit, the last for 2D also
 * with the units of each XCD contiguous (so that neighbouring tiles share
 * one L2), with or without write-back stores.  Defaults, as measured: 2D
 * analysis plans run one tile per work-group, XCD-contiguous, with
 * write-back stores (rows of most images start inside a cache line, and
 * neighbouring tiles then share lines); 2D synthesis plans and 1D plans run
 * one unit per work-group.  A 1D analysis plan with items deeper
 * than 12 levels enqueues a second, small kernel that finishes those items,
 * one work-group per item.  The plan itself holds host memory only; the
 * device-side tables and counters live in a caller-owned workspace of
 * haar_plan_workspace_size() bytes (256-byte aligned).
 *
 * haar_plan_upload() writes the tables and zeroes the counters (it enqueues a
 * memset and copies from memory the plan owns: do not destroy the plan, and
 * do not call it during stream capture, before the stream has passed them).
 * haar_plan_execute() allocates nothing, never synchronises, and leaves the
 * counters at zero when its kernel ends (the last work-group resets them), so
 * it may be captured into a hipGraph and replayed.  Executions sharing one
 * workspace must not overlap in time.  Item pointers are device pointers and
 * follow the plain-call rules (same dtype for all items, no aliasing).
 *
 * Limits: 2D items 1 <= levels <= min(5, haar_max_levels_2d); 1D items
 * 1 <= levels <= min(20, haar_max_levels_1d), and items with more than 12
 * levels at most 1024 * 4096 samples long (HAAR_ERR_UNSUPPORTED otherwise).
 * 1D items with more than 12 levels keep their level-12 approximation in
 * FP32 in the workspace between the two kernels.
 * ------------------------------------------------------------------------ */
typedef struct {
    const void* in;   /* [length] input (device)                */
    void* out;        /* [length] output (device)               */
    int64_t length;
    int32_t levels;
} haar_item_1d;

typedef struct {
    const void* in;   /* [height][width] input (device)         */
    void* out;        /* [height][width] output (device)        */
    int64_t height;
    int64_t width;
    int32_t levels;
} haar_item_2d;

typedef struct haar_plan haar_plan;

/* inverse = 0: analysis of every item; inverse = 1: synthesis. */
int haar_plan_create_1d(const haar_item_1d* items, int64_t count, int32_t dtype,
                        int32_t inverse, haar_plan** out);
int haar_plan_create_2d(const haar_item_2d* items, int64_t count, int32_t dtype,
                        int32_t inverse, haar_plan** out);
int haar_plan_workspace_size(const haar_plan* plan, size_t* bytes);
int haar_plan_upload(haar_plan* plan, void* workspace, void* stream);
int haar_plan_execute(const haar_plan* plan, void* workspace, void* stream);
/* Number of work units and the grid size (work-groups) of one execute. */
int haar_plan_info(const haar_plan* plan, int64_t* tiles, int32_t* grid);
/* Select a plan configuration; the plan must be uploaded again.  The
 * schedule is 0: a persistent grid of G work-groups, work-group b runs units
 * b, b + G, b + 2G, ... of the list; 1: a persistent grid whose work-groups
 * claim units from an atomic counter; 2: one work-group per unit; 3 (2D
 * only): one work-group per unit, the units of each XCD contiguous in the
 * list, outputs written with write-back instead of streaming stores; 4 (2D
 * only): one work-group per unit, the units of each XCD contiguous, streaming
 * stores.  2D: config = tile shape + 2 * schedule, tile shape 0: 32 rows x
 * 16 vectors, 1: 32 rows x 32 vectors (configs 0..9).  1D: config =
 * schedule (0..2). */
int haar_plan_set_config(haar_plan* plan, int32_t config);
/* Autotune a plan: time executes of every configuration on `stream`
 * (hipEvents; synchronises the stream; overwrites the items' outputs), keep
 * the fastest, upload it, and return its index in *choice.  Not during
 * capture. */
int haar_plan_tune(haar_plan* plan, void* workspace, void* stream, int32_t* choice);
int haar_plan_destroy(haar_plan* plan);

/* ------------------------------------------------------------------------
 * Tuning.  haar_tune_2d times the candidate tile shapes for one problem on
 * `stream` (hipEvents; it synchronises that stream) using caller-owned
 * device scratch of at least 2 * batch * height * width * element bytes
 * + 32 (two 16-byte-aligned tensors),
 * records the fastest in the process-wide table and returns its index in
 * *choice.  The table is consulted by later plain calls and plans with the
 * same (dtype, direction, levels, size class).  haar_tune_save/load write
 * and read the table as JSON text.  Never call these during capture.
 * ------------------------------------------------------------------------ */
int haar_tune_2d(int32_t dtype, int32_t inverse, int64_t height, int64_t width,
                 int32_t levels, int64_t batch, void* scratch, size_t scratch_bytes,
                 void* stream, int32_t* choice);
/* Same for the 1D chunk shapes (scratch: 2 * batch * length * element bytes
 * + 32). */
int haar_tune_1d(int32_t dtype, int32_t inverse, int64_t length, int32_t levels, int64_t batch,
                 void* scratch, size_t scratch_bytes, void* stream, int32_t* choice);
int haar_tune_save(const char* path);
int haar_tune_load(const char* path);
/* Number of 2D tile-shape candidates and a description of candidate i. */
int haar_tune_candidates_2d(int32_t dtype);
const char* haar_tune_candidate_name(int32_t dtype, int32_t index);
/* Force candidate `index` (or -1 to restore table/default choice) for 2D. */
int haar_force_config_2d(int32_t dtype, int32_t index);
/* Number of 1D chunk candidates: index -> (threads, samples per thread,
 * XCD-contiguous chunk order): 0: 256 x 16 (the default beyond 2048
 * samples), 1: 1024 x 16, 2: 64 x 16, 3: 128 x 16, 4: 256 x 16 in plain
 * block order. */
int haar_tune_candidates_1d(void);
/* Force 1D chunk candidate `index` (or -1 to restore the table/default
 * choice) for plain 1D calls of storage `dtype`; HAAR_ERR_UNSUPPORTED for an
 * index outside [-1, haar_tune_candidates_1d()). */
int haar_force_config_1d(int32_t dtype, int32_t index);

/* ------------------------------------------------------------------------
 * Diagnostics.
 * ------------------------------------------------------------------------ */
const char* haar_status_string(int status);
const char* haar_last_error(void);
const char* haar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HAAR_H_ */
