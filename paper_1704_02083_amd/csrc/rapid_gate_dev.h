// rapid_gate_dev.h -- device code of the prediction gate shared by the
// stand-alone gate kernels and the refinement kernel, which evaluates the
// gate in place at the gate point of a fused launch.
//
// Features (Eq. (6) needs a feature vector per superpixel): sixteen values
// from exact integer accumulators over the blocks of the stage before the
// gate.  Network: 16 -> 64 -> 64 -> 1 (ReLU), bf16 MFMA
// (v_mfma_f32_16x16x16bf16_1k) with fp32 accumulation, computed transposed
// (H^T = W X^T): the weights are the A operand, the activations the B
// operand, and the D fragment of one layer is the B fragment of the next.
// Parameter vector (5313 values): W1 (64x16, row = output neuron), b1 (64),
// W2 (64x64), b2 (64), w3 (64), b3 (1).
#pragma once
#include "rapid_internal.h"

namespace rapid {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int P_W1 = 0, P_B1 = 1024, P_W2 = 1088, P_B2 = 5184, P_W3 = 5248, P_B3 = 5312;

// fp32 -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b)
{
    return __uint_as_float((uint32_t)b << 16);
}

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    v4s r;
    r[0] = (short)f2bf(a);
    r[1] = (short)f2bf(b);
    r[2] = (short)f2bf(c);
    r[3] = (short)f2bf(d);
    return r;
}

__device__ __forceinline__ v4s load4bf(const uint16_t *p)
{
    v4s r;
    r[0] = (short)p[0];
    r[1] = (short)p[1];
    r[2] = (short)p[2];
    r[3] = (short)p[3];
    return r;
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// x fragment of one 16-sample tile in B layout: features 4*(lane/16)+r of
// sample n = 16 t + lane%16 (zeros past N)
__device__ __forceinline__ v4s load_x(const float *__restrict__ X, int64_t n, int64_t N, int grp)
{
    if (n >= N) {
        v4s z = {0, 0, 0, 0};
        return z;
    }
    const float *p = X + 16 * n + 4 * grp;
    return pack4(p[0], p[1], p[2], p[3]);
}

// Logit of the tile's sample lane%16 (valid in lanes 0-15), weight
// fragments read from P as they are needed (few registers held).
__device__ __forceinline__ float mlp_logit(const uint16_t *__restrict__ P, v4s bx, int lane)
{
    const int col = lane & 15, grp = lane >> 4;
    v4s h1[4], h2[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint16_t *b = P + P_B1 + 16 * i + 4 * grp;
        v4f c = {bf2f(b[0]), bf2f(b[1]), bf2f(b[2]), bf2f(b[3])};
        c = mfma(load4bf(P + P_W1 + (16 * i + col) * 16 + 4 * grp), bx, c);
        h1[i] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint16_t *b = P + P_B2 + 16 * i + 4 * grp;
        v4f c = {bf2f(b[0]), bf2f(b[1]), bf2f(b[2]), bf2f(b[3])};
#pragma unroll
        for (int j = 0; j < 4; j++) c = mfma(load4bf(P + P_W2 + (16 * i + col) * 64 + 16 * j + 4 * grp), h1[j], c);
        h2[i] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    }
    v4f c = {grp == 0 ? bf2f(P[P_B3]) : 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; j++) {
        v4s a = {0, 0, 0, 0};
        if (col == 0) a = load4bf(P + P_W3 + 16 * j + 4 * grp);
        c = mfma(a, h2[j], c);
    }
    return c[0];   // row 0 of the output
}

// ------------------------------------------------------------- features

// Step A for superpixel k: fixed-point colour means, accumulators cleared.
// st: K x 6 statistics (n, S_rgb, T_xy).
__device__ __forceinline__ void feat_init_sp(const int64_t *st, int32_t *fmean, int64_t *facc, int k, int F)
{
    const int64_t *r = st + 6 * (int64_t)k;
    const int64_t n = r[0];
    for (int ch = 0; ch < 3; ch++) fmean[3 * k + ch] = (int32_t)(((r[1 + ch] << (F + 1)) + n) / (2 * n));
    int64_t *a = facc + FACC * (int64_t)k;
    for (int q = 0; q < FACC; q++) a[q] = 0;
    a[7] = INT64_MAX;   // min contrast
}

// Sums of three values over the runs of equal keys in consecutive lanes of
// a wave (a segmented inclusive scan); true in the last lane of each run,
// which then holds the run's sums.  Every lane of the wave must call it.
__device__ __forceinline__ bool run_sums3(int32_t key, int64_t &a, int64_t &b, int64_t &c)
{
    const int lane = threadIdx.x & 63;
    const int32_t kup = __shfl_up(key, 1);
    int head = (lane == 0 || kup != key) ? 1 : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t ua = __shfl_up(a, off), ub = __shfl_up(b, off), uc = __shfl_up(c, off);
        const int uh = __shfl_up(head, off);
        if (lane >= off && !head) {
            a += ua;
            b += ub;
            c += uc;
            head = uh;
        }
    }
    const int32_t kdn = __shfl_down(key, 1);
    return lane == 63 || kdn != key;
}

// Step B for the blocks i of one wave (valid: i < number of blocks; every
// lane of the wave calls it): pixel second moments of the block (from moms
// when the block-sum pass stored them, else from the pixels) per
// superpixel, and for its right and lower neighbour blocks of another label
// the shared edge length and the squared distance of the two fixed-point
// means, for both superpixels.
__device__ __forceinline__ void feat_block(const Job &J, const int32_t *__restrict__ L, int B, int nbx, int nby,
                                           int64_t i, bool valid, const uint32_t *__restrict__ moms,
                                           const int32_t *__restrict__ fmean, int64_t *__restrict__ facc)
{
    const int W = J.W, H = J.H;
    int32_t k = -1;
    int64_t q0 = 0, q1 = 0, q2 = 0;
    int bx = 0, by = 0, x0 = 0, y0 = 0, x1 = 0, y1 = 0;
    if (valid) {
        bx = (int)(i % nbx);
        by = (int)(i / nbx);
        x0 = bx * B;
        y0 = by * B;
        x1 = min(x0 + B, W);
        y1 = min(y0 + B, H);
        k = L[i];
        if (moms) {
            // written by the block-sum pass of this stage
            q0 = moms[3 * i];
            q1 = moms[3 * i + 1];
            q2 = moms[3 * i + 2];
        } else {
            for (int y = y0; y < y1; y++) {
                const uint8_t *row = J.rgb + (int64_t)y * J.rgb_stride + 3 * (int64_t)x0;
                for (int x = 0; x < x1 - x0; x++) {
                    const int r = row[3 * x], g = row[3 * x + 1], b = row[3 * x + 2];
                    q0 += r * r;
                    q1 += g * g;
                    q2 += b * b;
                }
            }
        }
    }
    if (run_sums3(k, q0, q1, q2) && k >= 0) {
        int64_t *ak = facc + FACC * (int64_t)k;
        atomicAdd(reinterpret_cast<unsigned long long *>(ak + 0), (unsigned long long)q0);
        atomicAdd(reinterpret_cast<unsigned long long *>(ak + 1), (unsigned long long)q1);
        atomicAdd(reinterpret_cast<unsigned long long *>(ak + 2), (unsigned long long)q2);
    }
    if (!valid) return;
    for (int d = 0; d < 2; d++) {
        const int nx = bx + (d == 0), ny = by + (d == 1);
        if (nx >= nbx || ny >= nby) continue;
        const int32_t j = L[(int64_t)ny * nbx + nx];
        if (j == k) continue;
        const int64_t e = d == 0 ? (y1 - y0) : (x1 - x0);
        int64_t d2 = 0;
        for (int ch = 0; ch < 3; ch++) {
            const int64_t df = (int64_t)fmean[3 * k + ch] - fmean[3 * j + ch];
            d2 += df * df;
        }
        const int32_t both[2] = {k, j};
        for (int u = 0; u < 2; u++) {
            int64_t *a = facc + FACC * (int64_t)both[u];
            atomicAdd(reinterpret_cast<unsigned long long *>(a + 3), (unsigned long long)e);
            atomicAdd(reinterpret_cast<unsigned long long *>(a + 4), (unsigned long long)(e * d2));
            atomicMax(reinterpret_cast<unsigned long long *>(a + 6), (unsigned long long)d2);
            atomicMin(reinterpret_cast<unsigned long long *>(a + 7), (unsigned long long)d2);
        }
    }
}

// Step C for superpixel k: the sixteen features (double arithmetic without
// contraction, so that every value is the correctly rounded result of the
// same expression on any IEEE machine):
//   0-2 mean colour / 255, 3-5 colour std / 64, 6 size / A, 7 boundary
//   length / (4 sqrt A), 8 compactness bl^2 / (16 n), 9 centroid drift from
//   the initial cell centre / sqrt A, 10-12 max / edge-weighted rms / min
//   neighbour contrast / (255 2^F), 13 moved pixels / n, 14 max colour std
//   / 64, 15 one.
__device__ __forceinline__ void feat_final_sp(const Job &J, const int64_t *st, const int64_t *facc,
                                              const int64_t *moved, int k, int F, float *f)
{
#pragma clang fp contract(off)
    const double A = (double)(((int64_t)J.W * J.H) / J.K);
    const double sA = sqrt(A);
    const double cs = 255.0 * (double)(1 << F);
    const int64_t *r = st + 6 * (int64_t)k;
    const int64_t *a = facc + FACC * (int64_t)k;
    const double n = (double)r[0];
    double sd[3];
    for (int ch = 0; ch < 3; ch++) {
        double mu = (double)r[1 + ch] / n;
        double v = (double)a[ch] / n - mu * mu;
        sd[ch] = sqrt(v > 0.0 ? v : 0.0);
        f[ch] = (float)(mu / 255.0);
        f[3 + ch] = (float)(sd[ch] / 64.0);
    }
    const double bl = (double)a[3];
    f[6] = (float)(n / A);
    f[7] = (float)(bl / (4.0 * sA));
    f[8] = (float)(bl * bl / (16.0 * n));
    const int col = k % J.gx, row = k / J.gx;
    const double cx0 = (double)(2 * col + 1) * (double)J.W / (2.0 * J.gx) - 0.5;
    const double cy0 = (double)(2 * row + 1) * (double)J.H / (2.0 * J.gy) - 0.5;
    const double dx = (double)r[4] / n - cx0, dy = (double)r[5] / n - cy0;
    f[9] = (float)(sqrt(dx * dx + dy * dy) / sA);
    f[10] = (float)(sqrt((double)a[6]) / cs);
    f[11] = (float)(a[3] ? sqrt((double)a[4] / bl) / cs : 0.0);
    f[12] = (float)(a[7] != INT64_MAX ? sqrt((double)a[7]) / cs : 0.0);
    f[13] = (float)((moved ? (double)moved[k] : 0.0) / n);
    double m3 = sd[0] > sd[1] ? sd[0] : sd[1];
    m3 = m3 > sd[2] ? m3 : sd[2];
    f[14] = (float)(m3 / 64.0);
    f[15] = 1.0f;
}

}  // namespace rapid
