/* rapid.h -- C-ABI of the MI355X (gfx950) RAPID refinement library.
 *
 * The library segments an RGB image into superpixels with the coarse-to-fine
 * topology-preserving refinement of RAPID (Sulimowicz & Ahmad, ICME 2017):
 * the CTFTPS energy of Eq. (1), block moves of Eq. (3) restricted to
 * boundary blocks (Eq. (2); Eq. (7) under a prediction gate), the size
 * regularity of Sec. 3.1 as hard bounds (optionally with the merge on
 * underflow of Eqs. (4)-(5)), and the adaptive multi-level framework of
 * Sec. 3.2 (statistics computed once and reused; Eq. (8) holds by
 * construction because every sum is kept in fine-pixel units).
 *
 * Input: one HWC uint8 RGB image (or a batch) and a target superpixel count.
 * Output: one int32 label per pixel in [0, gx*gy).
 *
 * Conventions
 *  - Every pointer named *_dev is a device pointer (HIP memory on the
 *    context's device) owned by the caller; it must stay valid until the
 *    work queued on the context's stream completes.  The library never frees
 *    caller memory.  Host pointers (params, report, config) are read or
 *    written before the call returns.
 *  - Calls are ordered on the context's stream.  Argument errors are
 *    returned synchronously and nothing is queued.  rapid_segment,
 *    rapid_segment_batch and rapid_refine_level synchronise the stream
 *    before returning when a report is requested; otherwise they return
 *    after queueing.  A device fault surfaces as RAPID_EDEVICE.
 *  - On error the contents of output buffers are undefined.
 *  - Identical inputs give identical outputs (the schedule is deterministic
 *    and every statistic is an exact integer).
 */
#ifndef RAPID_H
#define RAPID_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAPID_ABI_VERSION 2
#define RAPID_MAX_LEVELS 4
#define RAPID_MAX_STAGES 8
#define RAPID_MAX_DIM 8192

typedef enum {
    RAPID_OK = 0,
    RAPID_EINVAL = -1,   /* bad argument: sizes, schedule, weights, NULL pointer */
    RAPID_ENOMEM = -2,   /* device or host allocation failed                     */
    RAPID_EDEVICE = -3,  /* a HIP call or kernel failed                           */
    RAPID_ESTATE = -4,   /* state used out of order (level already refined ...)  */
    RAPID_EGATE = -5     /* gate model unusable (non-finite weights)             */
} rapid_status;

typedef struct rapid_ctx rapid_ctx;       /* opaque, library-owned */
typedef struct rapid_state rapid_state;   /* opaque, library-owned */

#define RAPID_CFG_TIMING 1   /* record HIP events around every kernel launch */
#define RAPID_CFG_AUTOTUNE 2 /* tune the launch shape per problem shape (below) */
/* Test hook: every cooperative launch (one image on many workgroups) that
 * refines at least one stage starts with its abort word raised, so that every workgroup leaves the kernel at
 * its first grid barrier, as when a barrier's bounded wait gives up.  Such
 * a launch makes its call return RAPID_EDEVICE (a level-by-level state then
 * stays at the level it had); the autotuner drops such candidates. */
#define RAPID_CFG_TEST_ABORT 4

/* rapid_params.gate_features values */
#define RAPID_FEATURES_LEARNED 0
#define RAPID_FEATURES_ROI 1

/* rapid_params.gate_rule values */
#define RAPID_GATE_EITHER 0
#define RAPID_GATE_BOTH 1
#define RAPID_GATE_DIFFER 2

typedef struct {
    int32_t abi_version;   /* RAPID_ABI_VERSION */
    int32_t device;        /* HIP device ordinal */
    void *hip_stream;      /* hipStream_t to queue on; NULL = the null stream */
    int32_t flags;         /* RAPID_CFG_* bits */
    int32_t reserved;      /* 0 */
    /* Autotuning (RAPID_CFG_AUTOTUNE): the first segmentation call of each
     * problem shape (images, largest W, H and superpixel count, schedule,
     * gate and merge modes) runs its launch once per candidate shape --
     * workgroup size 256, 512 or 1024; per-superpixel state all in LDS,
     * the statistics packed with the flow counters (where the size bounds
     * allow the packing), the means records and flow counters, only the
     * means records, or nothing in LDS (as far as they fit); block-sum
     * pyramid inside the launch or in separate launches; and, for a single
     * image without merge, the image spread over 8 .. 128 workgroups of a
     * cooperative launch (which builds its pyramid over its own grid), with
     * small sweeps on the whole grid or on one workgroup --
     * and keeps the fastest (without tuning, a single image whose finest
     * stage has 2^20 blocks or more runs on 64 workgroups, sweeps of at
     * most 16384 active blocks on one); later calls of that
     * shape use it.  Every candidate computes the same labels (the result
     * never depends on the shape), so tuning costs time only.  Only calls
     * that start from the image tune (not rapid_refine_level).
     * autotune_cache: NULL, or a file that holds the choices across
     * processes: read by rapid_init when present (ignored when written for
     * another device architecture), rewritten after every new choice. */
    const char *autotune_cache;
} rapid_config;

/* Kernel durations of the last segmentation call (context created with
 * RAPID_CFG_TIMING), measured with HIP events on the context's stream. */
typedef struct {
    float block_sums_ms;   /* block-sum launches before the refinement
                              kernel (0 when that kernel builds the
                              pyramids itself)                        */
    float refine_ms;       /* the refinement kernel (all stages, and the
                              gate point of a gated call)             */
    int32_t threads;       /* launch shape of that call: workgroup size, */
    int32_t stats_lds;     /* per-superpixel state: 1 all in LDS, 3 the
                              means records and flow counters in LDS, 4
                              the packed statistics and flow counters in
                              LDS, 2 the means records in LDS, 0 all
                              global,                                   */
    int32_t pyramid;       /* pyramid inside the refinement launch (1)   */
    int32_t tuned;         /* 1 when this call ran the autotuner         */
    int32_t workgroups;    /* workgroups per image: 1, or the size of the
                              cooperative launch that spread a single
                              image over many workgroups                  */
} rapid_timings;

/* Method parameters, all integers (the paper gives no values for the
 * weights lambda_pos, lambda_b, the size bounds or the schedule).
 *  K          target superpixel count; the grid is gy = nearest integer to
 *             sqrt(K H / W), gx = nearest integer to K / gy (ties to the
 *             smaller).  K == 0: use gx, gy as given.
 *  levels     coarse to fine; a level pixel is factor x factor fine pixels
 *             and its stages are block sizes in level pixels.  The effective
 *             block size b * factor must not increase and must divide the
 *             previous one; at most 64.  The first effective size B0 is the
 *             grid block: gx * B0 <= W and gy * B0 <= H.
 *  gate_level first level refined under a gate (Algorithm RAPID applies
 *             the prediction at the second level); -1: never.
 *  frac_bits  F, fixed-point fraction bits of the means (0..4).
 *  max_sweeps sweep cap per stage (1 .. 2^20).
 *  gate_rule  how the per-superpixel gate bits g select the pairs (a, k)
 *             that may exchange blocks past the gate level (Eq. (7)):
 *             RAPID_GATE_EITHER  g_a or g_k (g = 1 everywhere is the plain
 *                                method),
 *             RAPID_GATE_BOTH    g_a and g_k,
 *             RAPID_GATE_DIFFER  g_a != g_k: g holds a predicted class and
 *                                only pairs across a class border refine,
 *                                as the paper's boundary superpixels.
 *  gate_features which feature vector the prediction step computes per
 *             superpixel (Eq. (6)):
 *             RAPID_FEATURES_LEARNED the sixteen features of the learned
 *                                gate (see rapid_gate_model),
 *             RAPID_FEATURES_ROI the paper's four ROI features (Sec. 4):
 *                                x0 absolute brightness (mean of the three
 *                                channel means) / 255; x1 comparative
 *                                brightness: x0 minus the mean brightness of
 *                                the 4-adjacent superpixels weighted by the
 *                                shared pixel edges (their fixed-point means
 *                                / 2^F), / 255; x2 extra-region
 *                                dissimilarity: the edge-weighted rms
 *                                distance of its fixed-point mean colour to
 *                                its neighbours' / (255 2^F); x3 intra-region
 *                                dissimilarity: sqrt of the mean channel
 *                                variance of its pixels / 64; x4..x14 zero,
 *                                x15 = 1.  x1 and x2 are 0 without
 *                                neighbours.  A model must be trained on the
 *                                feature vector it is used with.
 *  merge      0: plain size bounds.  1: merge on underflow (Sec. 3.1,
 *             Eqs. (4)-(5)): a superpixel that one of its blocks could not
 *             leave without going below min_size asks to merge; when a
 *             sweep commits nothing, every asker still below
 *             min_size + B^2 pixels picks the 4-adjacent superpixel of least
 *             merged energy (Eq. (1) after minus before, means of the
 *             union) among those with an active pair and a merged size
 *             within max_size (at most 8 distinct neighbour labels, else no
 *             pick; ties to the smaller label); an asker leaves when its
 *             pick picked nothing, or picked it back and has the smaller
 *             label; the smallest leaving label per target merges into it,
 *             then sweeping resumes around the merged blocks.  Merged
 *             labels end up empty (n = 0) and absent from the output.
 *             Per label 4-connected input is assumed (a state import
 *             with disconnected labels may merge differently).
 *  min_size, max_size  hard size bounds in pixels (Sec. 3.1, Eq. (5)).
 *  w_col, w_pos, w_bnd integer weights of colour, position and boundary
 *             terms (Eq. (1)); rejected when the worst-case block energy
 *             could leave the int64 range. */
typedef struct {
    int32_t K, gx, gy;
    int32_t n_levels;
    int32_t factor[RAPID_MAX_LEVELS];
    int32_t n_stages[RAPID_MAX_LEVELS];
    int32_t stages[RAPID_MAX_LEVELS][RAPID_MAX_STAGES];
    int32_t gate_level;
    int32_t frac_bits;
    int32_t max_sweeps;
    int32_t gate_rule;     /* RAPID_GATE_*: which pairs a gate lets move */
    int32_t merge;         /* 1: merge on underflow */
    int32_t gate_features; /* RAPID_FEATURES_*: the prediction step's features */
    int64_t min_size, max_size;
    int64_t w_col, w_pos, w_bnd;
} rapid_params;

/* One image.  rgb_dev: HWC uint8, row_stride_bytes >= 3 W.  labels_dev:
 * int32, label_stride (elements) >= W; receives one label per pixel. */
typedef struct {
    const uint8_t *rgb_dev;
    int32_t W, H;
    int64_t row_stride_bytes;
    int32_t *labels_dev;
    int64_t label_stride;
} rapid_image;

/* Per-stage counters (the complexity terms of Sec. 3.4: blocks visited from
 * the boundary queue, moves). */
typedef struct {
    int32_t level, block, sweeps, converged;
    int64_t active;      /* block visits summed over sweeps          */
    int64_t proposals;   /* best move differs from the current label */
    int64_t commits;     /* proposals admitted by the size filter     */
    int64_t skip_min;    /* visits skipped: source would fall below min */
    int64_t skip_topo;   /* visits skipped: not a simple point        */
    int64_t merges;      /* superpixels merged away (merge on)         */
} rapid_stage_report;

typedef struct {
    int32_t n_stages;    /* entries filled in stage[] */
    int32_t K;           /* superpixels gx * gy       */
    rapid_stage_report stage[RAPID_MAX_LEVELS * RAPID_MAX_STAGES];
} rapid_report;

/* Create a context on cfg->device: builds the 256-entry simple-point table
 * of the topology term (Eq. (1), E_topo) and uploads it.  *out receives the
 * context; rapid_destroy releases it.  Environment: RAPID_THREADS=n (64 ..
 * 1024, a multiple of 64) fixes the workgroup size; RAPID_SHAPE=t,l,p[,g[,s]]
 * fixes the whole launch shape (workgroup size, residency l as in
 * rapid_timings.stats_lds when it fits, pyramid inside the launch, g
 * workgroups per image where a single plain image may spread over a
 * cooperative launch, whose sweeps with at most s active blocks run on one
 * workgroup; a cooperative launch builds the pyramid itself whatever p says)
 * and bypasses the autotuner. */
rapid_status rapid_init(const rapid_config *cfg, rapid_ctx **out);
void rapid_destroy(rapid_ctx *ctx);   /* NULL-safe; waits for queued work */

/* Segment one image (Algorithm RAPID, all levels).  gate_dev: NULL for the
 * plain method, else gx*gy bytes (non-zero = superpixel marked by the
 * prediction of Eq. (6)) applied from params->gate_level on (Eq. (7)).
 * report may be NULL. */
rapid_status rapid_segment(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                           const uint8_t *gate_dev, rapid_report *report);

/* Segment n images in one launch, every image with the same params (the
 * grid is derived per image from K).  reports: NULL or n entries. */
rapid_status rapid_segment_batch(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                                 const rapid_params *params, rapid_report *reports);

/* rapid_segment for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same segmentation, labels and report as rapid_segment (gate_dev: the
 * caller's gate bits or NULL), with every byte of scratch in a fixed
 * library-owned device array of RAPID_NOALLOC_SCRATCH_BYTES per GPU (held
 * from the library's loading until the process ends; its address is taken
 * once per device by rapid_init).  The call itself allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  It runs the image on
 * one workgroup in the default launch shape (no autotuning, no cooperative
 * launch); the image's scratch (about 25 bytes per finest block plus 150
 * bytes per superpixel) must fit the array, else RAPID_EINVAL and nothing
 * is queued.  Every call on one GPU uses that GPU's single array: calls that
 * overlap on one GPU (other streams, contexts or threads) race and give
 * undefined results; calls ordered on one stream do not.  The array keeps
 * the last call's contents; each call initialises what it reads.  When a
 * report is requested the call synchronises the stream; without one (and
 * without RAPID_CFG_TIMING) it only queues kernels on the context's stream
 * (no memset, copy or synchronisation), so a caller may capture it in a HIP
 * graph and replay that graph on new contents of the same buffers. */
#define RAPID_NOALLOC_SCRATCH_BYTES 67108864   /* 64 MiB */
rapid_status rapid_segment_noalloc(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                                   const uint8_t *gate_dev, rapid_report *report);

/* Level-by-level use (the outer loop of Algorithm RAPID).  state_create
 * computes the grid labels and the statistics once (first level, Sec. 3.2);
 * each rapid_refine_level call runs every stage of one level, in order
 * 0, 1, ..., reusing the statistics; gate_dev as in rapid_segment but for
 * this level only.  rapid_state_export writes the current labels expanded to
 * pixels (labels_dev, W*H int32, row-major) and the statistics (stats_dev,
 * gx*gy*6 int64: n, colour sums R G B, coordinate sums x y); either may be
 * NULL. */
rapid_status rapid_state_create(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                                rapid_state **out);
rapid_status rapid_refine_level(rapid_ctx *ctx, rapid_state *st, int32_t level,
                                const uint8_t *gate_dev, rapid_report *report);
rapid_status rapid_state_export(rapid_ctx *ctx, rapid_state *st, int32_t *labels_dev,
                                int64_t *stats_dev);
void rapid_state_destroy(rapid_state *st);   /* NULL-safe */

/* Checkpoint resume: restore into st (created with the same image and
 * params) the point after next_level levels (0 .. n_levels) of Algorithm
 * RAPID.  labels_dev: W*H int32 pixel labels (row-major, stride W), as
 * rapid_state_export wrote them at that point; they must be constant on
 * every block of that point's block size (the last stage of level
 * next_level - 1, the first stage when next_level is 0) and lie in
 * [0, gx*gy).  stats_dev: gx*gy*6 int64 statistics as exported, or NULL to
 * recompute them exactly from the image and labels (Sec. 3.2 sums).  The
 * next rapid_refine_level call then takes level next_level.  Moved-pixel
 * tracking is not part of a checkpoint.  Labels that break the block or
 * range rule give RAPID_EINVAL and leave st unusable (RAPID_ESTATE) until a
 * later import succeeds.  Synchronous. */
rapid_status rapid_state_import(rapid_ctx *ctx, rapid_state *st, int32_t next_level, const int32_t *labels_dev,
                                const int64_t *stats_dev);

/* Waits for the last segmentation call and returns its kernel durations;
 * RAPID_ESTATE when the context does not time or nothing ran yet. */
rapid_status rapid_last_timings(rapid_ctx *ctx, rapid_timings *out);

/* The refinement kernel durations (rapid_timings.refine_ms) of the last
 * min(max_n, 128, timed calls so far) segmentation calls of a timing
 * context, oldest first, into refine_ms (max_n floats); *n_out receives
 * their number.  Each timed call records its HIP events in the next slot of
 * a ring of 128, so calls queued back to back need one synchronisation
 * (this call waits for the last).  RAPID_ESTATE when the context does not
 * time or nothing ran yet. */
rapid_status rapid_timing_history(rapid_ctx *ctx, float *refine_ms, int32_t max_n, int32_t *n_out);

/* ---------------------------------------------------------------- gate
 * The prediction step of Algorithm RAPID: at the start of the gate level
 * every superpixel gets a feature vector x and a classifier decides
 * y = [h(x) >= thresh] (Eq. (6)); from then on a move between superpixels a
 * and k is allowed only when y_a or y_k is set (Eq. (7), read per
 * superpixel).  h is a multilayer perceptron 16 -> 64 -> 64 -> 1 (ReLU,
 * logit output) with 5313 bf16 parameters: W1 (64x16, row = output), b1
 * (64), W2 (64x64), b2 (64), w3 (64), b3 (1).
 *
 * Features (16 float32 per superpixel, computed from exact integer sums at
 * the last stage before the gate): mean colour / 255 (3), colour standard
 * deviation / 64 (3), size / A, boundary length / (4 sqrt A), boundary
 * length^2 / (16 size), centroid drift from the initial cell centre /
 * sqrt A, max / edge-weighted rms / min colour contrast to neighbours /
 * (255 2^F) (3), pixels moved so far / size, max colour deviation / 64, 1;
 * A = floor(W H / (gx gy)). */
typedef struct {
    const uint16_t *w_bf16_dev;   /* 5313 bf16 parameters (device)            */
    float thresh;                 /* decision threshold on the logit (0: p >= 1/2) */
} rapid_gate_model;

/* Like rapid_segment_batch, with the gate: levels before params->gate_level
 * run plain, then features and the network decide the gate bits, then the
 * remaining levels run gated.  features_dev (nullable) receives the
 * features of all images' superpixels, image after image (sum of gx*gy rows
 * of 16 floats); gate_dev (nullable) the gate bits in the same order.
 * gate_level must be in [1, n_levels).  A model with non-finite weights is
 * refused: the images are segmented plain and RAPID_EGATE is returned.
 * Every call is one refinement launch that decides the gate inside (one
 * workgroup per image, or a single image spread over the workgroups of a
 * cooperative launch, which computes the features and the network across
 * them); every launch shape decides the same bits and labels. */
rapid_status rapid_segment_gated(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                                 const rapid_params *params, const rapid_gate_model *model,
                                 float *features_dev, uint8_t *gate_dev, rapid_report *reports);

/* State tracking for training data: involved_dev (nullable, gx*gy bytes)
 * has bytes set to 1 for superpixels that are the source or target of any
 * proposal in later rapid_refine_level calls; moved_dev (nullable, gx*gy
 * int64) accumulates the pixels moved into or out of each superpixel.  Both
 * are caller-owned and must be zeroed by the caller. */
rapid_status rapid_state_track(rapid_state *st, uint8_t *involved_dev, int64_t *moved_dev);

/* The 16 gate features of the state's superpixels at its current stage
 * (X_dev: gx*gy rows of 16 float32).  Feature 13 uses the moved counts
 * tracked so far (zero when not tracked). */
rapid_status rapid_state_features(rapid_ctx *ctx, rapid_state *st, float *X_dev);

/* The prediction step of Algorithm RAPID on a level-by-level state
 * (Eq. (6)): the features of its superpixels at the current stage as in
 * rapid_state_features, then gate_dev[k] = [h(x_k) >= model->thresh]
 * (gx*gy bytes), to pass to the following rapid_refine_level calls
 * (Eq. (7)).  features_dev (nullable): the gx*gy feature rows.  With
 * rapid_state_track's moved counts on from the first level, the bits equal
 * those rapid_segment_gated decides for the same image.  A model with
 * non-finite weights is refused: every byte of gate_dev is set to 1 (refine
 * all) and RAPID_EGATE is returned. */
rapid_status rapid_gate(rapid_ctx *ctx, rapid_state *st, const rapid_gate_model *model, float *features_dev,
                        uint8_t *gate_dev);

/* Misses of the boundary recall (Sec. 4.2) of test against ref, two W x H
 * int32 label maps on the device with the same row stride (in elements):
 * a boundary pixel of ref (one with a 4-neighbour of another label) is
 * missed when test has no boundary pixel within Chebyshev distance radius
 * (0..4).  Each miss adds 1 to miss_dev[ref label] and 1 to
 * miss_dev[test label] (2 when they agree) for labels in [0, K); miss_dev
 * (nullable, K int32) and totals_dev (nullable, 2 int64: ref boundary
 * pixels, misses) accumulate, so the caller zeroes them.  Boundary recall is
 * 1 - totals[1] / totals[0].  With ref the final plain labels and test the
 * labels at the gate point, miss_dev counts how far each superpixel's
 * boundary still travels: the gate's training target.  Stream-ordered. */
rapid_status rapid_boundary_miss(rapid_ctx *ctx, const int32_t *ref_dev, const int32_t *test_dev, int32_t W,
                                 int32_t H, int64_t stride, int32_t radius, int32_t K, int32_t *miss_dev,
                                 int64_t *totals_dev);

/* Network forward pass on n feature rows: logits_dev (nullable) receives
 * h(x); gate_dev (nullable) receives [h(x) >= thresh]. */
rapid_status rapid_mlp_forward(rapid_ctx *ctx, const float *X_dev, int64_t n, const uint16_t *w_bf16_dev,
                               float thresh, float *logits_dev, uint8_t *gate_dev);

/* Gradient of the mean binary cross-entropy with logits over the nb
 * samples idx_dev[0..nb) of (X_dev, t_dev): grads_dev receives 5313
 * floats; logits_dev (nullable) the nb logits.  Deterministic. */
rapid_status rapid_mlp_grad(rapid_ctx *ctx, const float *X_dev, const uint8_t *t_dev, const int32_t *idx_dev,
                            int32_t nb, const uint16_t *w_bf16_dev, float *grads_dev, float *logits_dev);

typedef struct {
    int32_t epochs;       /* passes of floor(n / batch) batches               */
    int32_t batch;        /* even; half positive, half negative samples       */
    float lr, beta1, beta2, eps;   /* Adam (Kingma & Ba, 2015)                 */
    uint64_t seed;        /* sample order                                     */
} rapid_train_cfg;

/* Train the gate network on n samples (features X_dev, targets t_dev in
 * {0,1}) with balanced batches and Adam.  master_dev: 5313 float32 master
 * weights, initial values in, trained values out; w_bf16_dev receives their
 * bf16 copy. */
rapid_status rapid_gate_train(rapid_ctx *ctx, const float *X_dev, const uint8_t *t_dev, int64_t n,
                              const rapid_train_cfg *cfg, float *master_dev, uint16_t *w_bf16_dev);

/* ------------------------------------------------------------- slides
 * A whole slide is cut into tiles of tile x tile pixels (the last row and
 * column ragged), each refined as an independent image over its core plus a
 * halo of `halo` pixels (clipped at the slide edge), all tiles in one
 * launch.  A tile's grid is the slide-wide grid of cell x cell superpixel
 * cells over its extended region (the last cell of an axis absorbs a
 * remainder narrower than a cell).  Only core pixels are written, each with
 * the slide-wide id (row * ceil(W / cell) + col) of the initial cell of its
 * superpixel; superpixels are not stitched across tiles.  tile and halo must
 * be multiples of cell, tile + 2 halo <= RAPID_MAX_DIM.  params->K, gx, gy
 * are ignored. */
typedef struct {
    const uint8_t *rgb_dev;      /* HWC uint8 slide                           */
    int64_t W, H, row_stride_bytes;
    int32_t *labels_dev;         /* int32 slide labels, label_stride elements */
    int64_t label_stride;
    int32_t tile, halo, cell;
    int32_t reserved;
} rapid_slide;

/* Number of tiles of a slide (host only). */
rapid_status rapid_slide_tiles(const rapid_slide *slide, int32_t *n_tiles);

/* Segment a slide (plain when model is NULL, else gated as in
 * rapid_segment_gated).  reports: NULL or rapid_slide_tiles() entries, tile
 * order row-major. */
rapid_status rapid_segment_slide(rapid_ctx *ctx, const rapid_slide *slide, const rapid_params *params,
                                 const rapid_gate_model *model, rapid_report *reports);

/* A slide under the prediction step (Algorithm RAPID's gate, Eqs. (6)-(7)),
 * as rapid_segment_slide with a model, one launch over all tiles, each tile
 * deciding the gate bits of its own superpixels inside the launch.
 * features_dev (nullable) receives the 16 features of every tile's
 * superpixels, tile after tile in row-major tile order (the sum over tiles
 * of gx*gy rows of 16 float32; a tile's rows in its own label order);
 * gate_dev (nullable) the gate bytes in the same order.  model must not be
 * NULL; a model with non-finite weights is refused as in
 * rapid_segment_gated (the slide is segmented plain, RAPID_EGATE). */
rapid_status rapid_segment_slide_gated(rapid_ctx *ctx, const rapid_slide *slide, const rapid_params *params,
                                       const rapid_gate_model *model, float *features_dev, uint8_t *gate_dev,
                                       rapid_report *reports);

/* Grid of a target count (see rapid_params.K).  Host only, no device. */
rapid_status rapid_grid(int32_t W, int32_t H, int32_t K, int32_t *gx, int32_t *gy);

/* The 256-entry simple-point table of the topology term (E_topo of
 * Eq. (1)) that the kernels use, as 8 words: bit m of word m/32 is set when
 * a block whose 3x3 ring has same-label mask m (bit r = neighbour r in
 * row-major order, centre skipped; out-of-image is "other") may leave its
 * label: its same-label ring blocks 4-connected to an edge neighbour form one
 * component and the other ring blocks one 8-connected component.  Host only. */
rapid_status rapid_simple_lut(uint32_t out[8]);

/* Validate params for a W x H image exactly as rapid_segment would;
 * *K_out (nullable) receives gx * gy.  Host only, no device. */
rapid_status rapid_check_params(int32_t W, int32_t H, const rapid_params *params, int32_t *K_out);

const char *rapid_status_str(rapid_status s);

#ifdef __cplusplus
}
#endif
#endif
