// rapid_state_kernels.h -- restoring a refinement state from a checkpoint.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rapid {

// Pixel labels (W x H, row stride in elements) to the B x B block map L
// (ceil(W/B) x ceil(H/B), row-major).  Every pixel of a block must carry the
// block's top-left label and every label must lie in [0, K); a violation
// sets *err to non-zero (the caller zeroes it first), and L is then
// undefined but holds labels in [0, K) only.
hipError_t launch_import_labels(const int32_t *labels, int64_t stride, int W, int H, int B, int32_t K,
                                int32_t *L, uint32_t *err, hipStream_t stream);

// Exact statistics of the block map L (block size B) over the image:
// stats[6k..6k+6) += n, sum R, sum G, sum B, sum x, sum y of label k's
// pixels.  The caller zeroes stats.
hipError_t launch_import_stats(const uint8_t *rgb, int64_t rgb_stride, int W, int H, int B, const int32_t *L,
                               int64_t *stats, hipStream_t stream);

}  // namespace rapid
