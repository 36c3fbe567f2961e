// rapid_internal.h -- data shared by the host driver and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "rapid.h"

namespace rapid {

constexpr int MAXST = RAPID_MAX_LEVELS * RAPID_MAX_STAGES;

enum { FLAG_INIT = 1, FLAG_OUT = 2 };

// The schedule, flattened: effective block size of every stage.
struct Sched {
    int32_t n_stages;
    int32_t B[MAXST];
    int32_t level[MAXST];
    int32_t gate_stage;      // first stage refined under the gate
    int32_t F, max_sweeps;
    int64_t min_size, max_size, w_col, w_pos, w_bnd;
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
    int32_t *props;          // 3 ints per proposal
    int32_t *changed;        // changed blocks of a sweep
    int32_t *stamp;          // per block visit stamp
    int64_t *stats;          // K x 6 int64: n, S_r, S_g, S_b, T_x, T_y
    int32_t *means;          // K x MN_STRIDE (global working set)
    int32_t *flow;           // K x 2 out/in (global working set)
    int32_t *touched;        // K flags + K list (global working set)
    rapid_stage_report *rep; // per stage
    const uint8_t *gate;     // K bytes or null
};

hipError_t launch_block_sums(const Job *jobs_dev, int n_jobs, int s, int B, int64_t max_nb,
                             hipStream_t stream);
hipError_t launch_expand(const int32_t *L, int W, int H, int B, int32_t *out, int64_t stride,
                         hipStream_t stream);
hipError_t launch_refine(const Job *jobs_dev, int n_jobs, const Sched &sc, int s_begin, int s_end,
                         int flags, const uint32_t *lut_dev, bool lds, size_t lds_bytes, int threads,
                         hipStream_t stream);

// per-superpixel means record: c_r c_g c_b mu_x mu_y n (int32)
constexpr int MN_STRIDE = 6;

// bytes of LDS per superpixel when the statistics live in LDS
constexpr size_t LDS_PER_SP = 6 * 8 + MN_STRIDE * 4 + 2 * 4 + 4 + 4;

}  // namespace rapid
