// rapid_internal.h -- data shared by the host driver and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include "rapid.h"

namespace rapid {

constexpr int MAXST = RAPID_MAX_LEVELS * RAPID_MAX_STAGES;
// gated runs keep one gate bit per superpixel in LDS: at most 2^18 per image
constexpr int MAX_GATE_WORDS = 8192;

// FLAG_INIT: grid labels and statistics first; FLAG_OUT: write the pixel
// labels; FLAG_GATE: evaluate the gate in place at the first gated stage
// (features, network, gate bits) and track moved pixels before it;
// FLAG_PYRAMID: with FLAG_INIT, each workgroup builds its job's block-sum
// pyramid (else separate launches have).
// FLAG_OWN_STATS: without FLAG_INIT, the statistics at the launch's start
// were made by this library from the grid (not imported), so their bounds
// are those of a launch from the image.
enum { FLAG_INIT = 1, FLAG_OUT = 2, FLAG_GATE = 4, FLAG_PYRAMID = 8, FLAG_OWN_STATS = 16 };

// jobs from which the refinement launch builds the block-sum pyramids itself
constexpr int PYRAMID_MIN_JOBS = 128;

// The schedule, flattened: effective block size of every stage.
struct Sched {
    int32_t n_stages;
    int32_t B[MAXST];
    int32_t level[MAXST];
    int32_t f64[MAXST];      // 1: every intermediate of E' at this stage is an
                             // integer below 2^53, so fp64 evaluates it exactly
    int32_t gate_stage;      // first stage refined under the gate
    int32_t gate_rule;       // RAPID_GATE_*
    int32_t merge;           // 1: merge on underflow
    int32_t feat_set;        // RAPID_FEATURES_*: the gate's feature vector
    int32_t F, max_sweeps;
    int32_t pk_bn, pk_bx;    // residency 4: bits of n and of T_x in the packed
                             // position word (T_y takes the bits above)
    int64_t min_size, max_size, w_col, w_pos, w_bnd;
    double d_wc, d_wp, d_wb, d_fs;   // w_col, w_pos, w_bnd 2^(2F), 2^(F+1) as doubles
    double d_wcfs, d_wpfs;           // w_col 2^(F+1), w_pos 2^(F+1)
    const uint16_t *mlp_w;           // FLAG_GATE: bf16 network parameters
    float mlp_thresh;                // FLAG_GATE: gate bit = logit >= mlp_thresh
};

// A proposal: block, source and destination labels, packed colour sum of
// the block (21 bits per channel).
struct Prop {
    int32_t bi, a, k, pad;
    uint64_t I;
};

// LDS carve-up of the refinement kernel (byte offsets into dynamic LDS).
// Statistics at offset 0 when stats_lds; work lists hold their first
// cap* entries in LDS and spill to global scratch; the visit bitmap of the
// frontier rebuild is used when it covers the stage's blocks.
struct LdsPlan {
    int32_t stats_lds;       // 0 global, 1 statistics, means, flow in LDS, 2 means in LDS,
                             // 3 means and flow in LDS, 4 packed statistics and flow in LDS
    int32_t capl, capp, capx, bm_words;
    int32_t gate_words;      // LDS bitmap of the gate bits (0: no gate in this launch)
    uint32_t off_lists, off_props, off_chg, off_bm, off_gate;
    uint32_t total;
};

// One image (or tile) and its scratch, all device pointers.
struct Job {
    const uint8_t *rgb;
    int64_t rgb_stride;
    int32_t W, H, gx, gy, K, pad;
    int32_t *out;            // pixel labels
    int64_t out_stride;
    int32_t *lab[2];         // label maps, ping-pong by stage parity
    uint64_t *sums[MAXST];   // packed block sums per stage (B >= 2)
    int32_t *lists;          // 9 class lists of capc entries
    int64_t capc;
    Prop *props;             // proposals beyond the LDS capacity
    int32_t *changed;        // changed blocks of a sweep
    int32_t *stamp;          // per block visit stamp (when the LDS bitmap is too small)
    int64_t *stats;          // K x 6 int64: n, S_r, S_g, S_b, T_x, T_y
    int32_t *means;          // K records of MN_STRIDE words (global working set)
    int32_t *flow;           // K x 2 out/in (global working set), twice
                             // (the cooperative kernel alternates buffers)
    rapid_stage_report *rep; // per stage
    const uint8_t *gate;     // K bytes or null
    // optional tracking (null: off)
    uint8_t *involved;       // K: source or target of a proposal at stage >= involve_stage
    int64_t *moved;          // K: pixels moved in or out by committed moves
    int32_t involve_stage, pad2;
    // gate feature scratch
    int32_t *fmean;          // K x 3 fixed-point means
    int64_t *facc;           // K x FACC accumulators
    // FLAG_GATE outputs: K feature rows of 16 floats and K gate bytes (the
    // gated stages then read gate == gate_out)
    float *xrow;
    uint8_t *gate_out;
    // per-block pixel second moments (3 x uint32 per block) of stage
    // moms_stage, written with the block-sum pyramid for the gate's features
    uint32_t *moms;
    int32_t moms_stage, pad4;
    // slide tiles: only the core [core_x0, +core_w) x [core_y0, +core_h) of
    // the tile is written, label k as the slide cell id
    // (gid_y0 + k / gx) * gid_w + gid_x0 + k % gx
    int32_t tile, core_x0, core_y0, core_w, core_h, pad3;
    int64_t gid_x0, gid_y0, gid_w;
    // merge on underflow (null when off): ask bits (K bits), askers in
    // order of asking (K), per asker its window of blocks and MERGE_NB
    // neighbour slots (label, shared length) with a state word, per label
    // its pick and the smallest leaving label that picked it
    uint32_t *mreq;
    int32_t *mlist;
    int4 *mbox;
    int32_t *mkey, *mlen, *mstate;
    int32_t *mpick, *mwin;
    // control words of a launch that spreads this job over many workgroups
    // (CTL_WORDS, zeroed by the host before each such launch)
    uint32_t *ctl;
};

// Control words of a cooperative launch (k_refine_mc): the grid barrier's
// arrival counter and abort word on lines of their own, the class counts
// (two buffers of 9), the proposal counter, the changed-block counters (two
// buffers) and the stage counters (6 x uint64 at a 64-bit aligned word).
enum { CTL_BAR = 0, CTL_ABORT = 32, CTL_CNT = 64, CTL_NPROP = 96, CTL_NCHG = 98, CTL_CTR = 128, CTL_WORDS = 256 };

// merge on underflow: neighbour slots per asker
constexpr int MERGE_NB = 8;

// rapid_segment_noalloc: the fixed device scratch per GPU, the job record in
// its first NOALLOC_JOB_BYTES, the image's scratch layout after it.
// noalloc_scratch: the calling thread's current device's copy (taken once
// per device); launch_store_job: writes a job record on the stream.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)RAPID_NOALLOC_SCRATCH_BYTES;
constexpr size_t NOALLOC_JOB_BYTES = 4096;
static_assert(sizeof(Job) <= NOALLOC_JOB_BYTES, "job record must fit its slot");
hipError_t noalloc_scratch(int device, char **out);
hipError_t launch_store_job(const Job &j, Job *dst, hipStream_t stream);

hipError_t launch_block_sums(const Job *jobs_dev, int n_jobs, int s, int B, int64_t max_nb, hipStream_t stream);
hipError_t launch_expand(const int32_t *L, int W, int H, int B, int32_t *out, int64_t stride,
                         hipStream_t stream);
// launch_refine: queue (a device word, nullable) turns a launch of more
// jobs than wgs workgroups (0: as many as the chip holds at once) into a
// persistent launch over a work queue in jobs_dev order
hipError_t launch_refine(const Job *jobs_dev, int n_jobs, uint32_t *queue, int wgs, const Sched &sc,
                         const LdsPlan &lp, int s_begin, int s_end, int flags, const uint32_t *lut_dev, int threads,
                         hipStream_t stream);
// one job on `groups` workgroups of a cooperative launch (no merge, not a
// slide tile, gate bits from the caller or none: gate_words > 0 loads them);
// sweeps with at most solo_max active blocks run on the
// first workgroup alone (solo_max < 0: never); max_coop_groups: the most
// workgroups of `threads` lanes that can be resident together on the
// current device
hipError_t launch_refine_mc(const Job *jobs_dev, int groups, const Sched &sc, int s_begin, int s_end, int flags,
                            const uint32_t *lut_dev, int threads, int64_t solo_max, int gate_words,
                            hipStream_t stream);
hipError_t max_coop_groups(int threads, int *out);

// gate network size and feature accumulators
constexpr int MLP_PARAMS = 5313;
constexpr int FACC = 8;

// per-superpixel means record: c_r c_g c_b mu_x mu_y n packed into four
// 32-bit words (16 bytes; two records per 32-byte sector)
constexpr int MN_STRIDE = 4;

hipError_t launch_features(const Job *jobs_dev, int n_jobs, int B, int lab_buf, int F, int fset, int32_t Kmax,
                           int64_t max_nb, const int64_t *xoff_dev, float *X, hipStream_t stream);
hipError_t launch_mlp_fwd(const float *X, int64_t N, const uint16_t *P, float thresh, float *logits,
                          uint8_t *gate, hipStream_t stream);
hipError_t launch_mlp_grad(const float *X, const uint8_t *T, const int32_t *idx, int32_t nb, float scale,
                           const uint16_t *P, float *part, int n_waves, float *grads, float *logits,
                           hipStream_t stream);
hipError_t launch_adam(float *theta, float *m, float *v, const float *g, uint16_t *wbf, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream);
hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t stream);
constexpr int BOUNDARY_MISS_RMAX = 4;
hipError_t launch_boundary_miss(const int32_t *ref, const int32_t *test, int W, int H, int64_t stride, int r,
                                int32_t K, int32_t *miss, int64_t *totals, hipStream_t stream);

// bytes of LDS per superpixel when the statistics live in LDS: sums, means
// record, flow counters
constexpr size_t LDS_PER_SP = 6 * 8 + MN_STRIDE * 4 + 2 * 4;
// bytes of LDS per superpixel when only the means records live in LDS, and
// when the flow counters join them
constexpr size_t LDS_MEANS_PER_SP = MN_STRIDE * 4;
constexpr size_t LDS_MEANS_FLOW_PER_SP = MN_STRIDE * 4 + 2 * 4;
// ... and when the statistics, packed into two 64-bit words, live there with
// the flow counters (residency 4; the means are computed where they are read)
constexpr size_t LDS_PACKED_FLOW_PER_SP = 2 * 8 + 2 * 4;

}  // namespace rapid
