/* Plain single-threaded CPU oracle of the RAPID coarse-to-fine superpixel
 * refinement sweep (CTFTPS energy with size regularity, prediction gate and
 * coarse-level reuse).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; it exists so that the tests, the smoke check and the CPU
 * baseline of the benchmark have an obviously-correct result to compare the
 * GPU library against.  It shares no code, header, table or generator with
 * the GPU library.
 *
 * Conventions (all integer; see oracle/rapid_oracle.c for the citations):
 *   image   HWC uint8 RGB, row stride in bytes, pixel p = (x, y) 0-based.
 *   labels  int32, row-major, one per pixel.
 *   stats   per superpixel k: n_k, S_k (3 colour sums), T_k (x and y sums),
 *           exported as 6 int64 per superpixel in that order.
 */
#ifndef RAPID_ORACLE_H
#define RAPID_ORACLE_H
#include <stdint.h>

#define ORC_MAX_LEVELS 4
#define ORC_MAX_STAGES 8

typedef struct {
    int32_t K;                 /* target superpixel count, or 0 to use gx, gy   */
    int32_t gx, gy;            /* explicit grid (used when K == 0)              */
    int32_t n_levels;          /* image levels, coarse to fine                  */
    int32_t factor[ORC_MAX_LEVELS];   /* a level pixel is factor x factor fine px */
    int32_t n_stages[ORC_MAX_LEVELS];
    int32_t stages[ORC_MAX_LEVELS][ORC_MAX_STAGES]; /* block sizes, level px   */
    int32_t gate_level;        /* first level refined under the gate; -1 never  */
    int32_t frac_bits;         /* F: fixed-point fraction bits of the means      */
    int32_t max_sweeps;
    int32_t shuffle_seed;      /* 0: natural block order; else a permutation    */
    int32_t gate_rule;         /* ORC_GATE_*: pairs a gate lets move            */
    int32_t merge;             /* 1: merge on underflow (Sec. 3.1, Eqs. (4)-(5)) */
    int32_t pad_;
    int64_t min_size, max_size;
    int64_t w_col, w_pos, w_bnd;
} orc_params;

typedef struct {
    int32_t level, block, sweeps, converged;
    int64_t active, proposals, commits, skip_min, skip_topo;
    int64_t merges;            /* superpixels merged away in the stage          */
} orc_stage_report;

/* merge on underflow: a superpixel with more distinct neighbour labels than
 * this does not merge */
#define ORC_MERGE_MAX_NB 8

/* gate rules (which pairs (a, k) may move past the gate level) */
#define ORC_GATE_EITHER 0      /* g_a or g_k                                    */
#define ORC_GATE_BOTH   1      /* g_a and g_k                                   */
#define ORC_GATE_DIFFER 2      /* g_a != g_k (predicted classes differ)         */

/* error codes */
#define ORC_OK        0
#define ORC_EINVAL   -1
#define ORC_ENOMEM   -2
#define ORC_EBLOCK   -3   /* a block's pixels disagree on their label          */
#define ORC_EINVAR   -4   /* a debug-mode invariant failed                      */

int orc_grid(int32_t W, int32_t H, int32_t K, int32_t *gx, int32_t *gy);
int orc_init_labels(int32_t W, int32_t H, int32_t B0, int32_t gx, int32_t gy,
                    int32_t *labels);
int orc_simple(int32_t ring_mask);
int orc_segment(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                const orc_params *p, const uint8_t *gate,
                int32_t *labels, int64_t *stats_out,
                orc_stage_report *rep, int32_t max_rep, int32_t debug);
int orc_segment_ex(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                   const orc_params *p, const uint8_t *gate,
                   int32_t *labels, int64_t *stats_out,
                   orc_stage_report *rep, int32_t max_rep, int32_t debug,
                   uint8_t *involved, int64_t *moved);
int orc_segment_fifo(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride, const orc_params *p,
                     int32_t *labels, int64_t *stats_out, int64_t *moves_out, int32_t debug);
int64_t orc_energy(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride, const orc_params *p,
                   const int32_t *labels, int32_t K);
int64_t orc_merge_cost(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                       const orc_params *p, const int32_t *labels, int32_t K, int32_t m, int32_t k);
int orc_features(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                 const int32_t *labels, int32_t B, const int64_t *stats, const int64_t *moved,
                 int32_t gx, int32_t gy, int32_t F, float *out);
int orc_roi_features(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                     const int32_t *labels, const int64_t *stats, int32_t gx, int32_t gy, int32_t F,
                     float *out);
int orc_propose_class(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                      const orc_params *p, const int32_t *labels, int32_t K,
                      int32_t B, int32_t cls, const uint8_t *gate,
                      int32_t *props, int64_t *eprime, int32_t max_props);
int64_t orc_block_energy(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                         const orc_params *p, const int32_t *labels, int32_t K,
                         int32_t B, int32_t bx, int32_t by, int32_t k);
#endif
