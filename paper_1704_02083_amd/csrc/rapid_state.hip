// rapid_state.hip -- checkpoint import of a level-by-level refinement state.
//
// The sweep state between two levels of Algorithm RAPID is the label map at
// the last stage's block size plus the per-superpixel sums (n, colour, x, y)
// that the levels reuse (Sec. 3.2).  Importing reduces a pixel label map to
// that block map, checking that it is constant on every block, and can
// rebuild the sums exactly from the image.  Neither is on the refinement's
// hot path: one pass over the pixels each.
#include "rapid_state_kernels.h"

namespace rapid {

__global__ void k_import_labels(const int32_t *__restrict__ lab, int64_t stride, int W, int H, int B, int32_t K,
                                int32_t *__restrict__ L, uint32_t *__restrict__ err)
{
    const int nbx = (W + B - 1) / B;
    const int64_t N = (int64_t)W * H;
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % W), y = (int)(i / W);
        const int bx = x / B, by = y / B;
        const int32_t v = lab[(int64_t)y * stride + x];
        const int32_t t = lab[(int64_t)(by * B) * stride + (int64_t)bx * B];
        const bool in_range = v >= 0 && v < K;
        bad |= (!in_range || v != t) ? 1u : 0u;
        if (x == bx * B && y == by * B) L[(int64_t)by * nbx + bx] = in_range ? v : 0;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 1u);
}

__global__ void k_import_stats(const uint8_t *__restrict__ rgb, int64_t rgb_stride, int W, int H, int B,
                               const int32_t *__restrict__ L, int64_t *__restrict__ stats)
{
    const int nbx = (W + B - 1) / B, nby = (H + B - 1) / B;
    const int64_t nb = (int64_t)nbx * nby;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int bx = (int)(i % nbx), by = (int)(i / nbx);
        const int x0 = bx * B, y0 = by * B;
        const int x1 = min(x0 + B, W), y1 = min(y0 + B, H);
        int64_t s[6] = {0, 0, 0, 0, 0, 0};
        for (int y = y0; y < y1; y++) {
            const uint8_t *row = rgb + (int64_t)y * rgb_stride;
            for (int x = x0; x < x1; x++) {
                s[1] += row[3 * x + 0];
                s[2] += row[3 * x + 1];
                s[3] += row[3 * x + 2];
                s[4] += x;
            }
            s[5] += (int64_t)y * (x1 - x0);
        }
        s[0] = (int64_t)(x1 - x0) * (y1 - y0);
        unsigned long long *r = reinterpret_cast<unsigned long long *>(stats + 6 * (int64_t)L[i]);
        for (int c = 0; c < 6; c++) atomicAdd(r + c, (unsigned long long)s[c]);
    }
}

static unsigned grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_import_labels(const int32_t *labels, int64_t stride, int W, int H, int B, int32_t K,
                                int32_t *L, uint32_t *err, hipStream_t stream)
{
    hipLaunchKernelGGL(k_import_labels, dim3(grid_for((int64_t)W * H, 256)), dim3(256), 0, stream, labels, stride,
                       W, H, B, K, L, err);
    return hipGetLastError();
}

hipError_t launch_import_stats(const uint8_t *rgb, int64_t rgb_stride, int W, int H, int B, const int32_t *L,
                               int64_t *stats, hipStream_t stream)
{
    const int64_t nb = (int64_t)((W + B - 1) / B) * ((H + B - 1) / B);
    hipLaunchKernelGGL(k_import_stats, dim3(grid_for(nb, 256)), dim3(256), 0, stream, rgb, rgb_stride, W, H, B, L,
                       stats);
    return hipGetLastError();
}

}  // namespace rapid
