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
    // a superpixel merged away (n = 0) has mean 0
    for (int ch = 0; ch < 3; ch++) fmean[3 * k + ch] = n ? (int32_t)(((r[1 + ch] << (F + 1)) + n) / (2 * n)) : 0;
    int64_t *a = facc + FACC * (int64_t)k;
    for (int q = 0; q < FACC; q++) a[q] = 0;
    a[7] = INT64_MAX;   // min contrast
}

// Per-block contributions to a superpixel's feature accumulators.
struct FeatAcc {
    int64_t q[3];    // pixel second moments per channel
    int64_t bl;      // boundary edge length (pixel edges to other labels)
    int64_t ed2;     // sum over those edges of length x squared mean distance
    int64_t nbs;     // sum over those edges of length x the neighbour's three
                     // fixed-point channel means
    uint64_t mx;     // largest squared mean distance to a neighbour
    uint64_t mn;     // smallest (UINT64_MAX: none)
};

__device__ __forceinline__ void feat_zero(FeatAcc &v)
{
    v.q[0] = v.q[1] = v.q[2] = 0;
    v.bl = v.ed2 = v.nbs = 0;
    v.mx = 0;
    v.mn = ~0ull;
}

// Adds one run's totals to superpixel k's accumulators in global memory.
__device__ __forceinline__ void feat_flush(int64_t *__restrict__ facc, int32_t k, const FeatAcc &v)
{
    unsigned long long *a = reinterpret_cast<unsigned long long *>(facc + FACC * (int64_t)k);
    atomicAdd(a + 0, (unsigned long long)v.q[0]);
    atomicAdd(a + 1, (unsigned long long)v.q[1]);
    atomicAdd(a + 2, (unsigned long long)v.q[2]);
    if (v.bl) {
        atomicAdd(a + 3, (unsigned long long)v.bl);
        atomicAdd(a + 4, (unsigned long long)v.ed2);
        atomicAdd(a + 5, (unsigned long long)v.nbs);
        atomicMax(a + 6, (unsigned long long)v.mx);
        atomicMin(a + 7, (unsigned long long)v.mn);
    }
}

// Blocks per segment of a row in step B.
constexpr int FEAT_SEG = 16;

// Step B for one segment: blocks [bx0, bx1) of block row by, whose labels
// are row[], the row above up[] and below dn[] (nullptr, or -1 entries,
// outside the image).  A block adds to its own superpixel:
// the pixel second moments of the block (from moms when the block-sum pass
// stored them, else from the pixels) and, for each 4-neighbour block of
// another label, the shared edge length and the squared distance of the two
// fixed-point means.  Both sides of an edge count it for their own
// superpixel, so every total is a sum over the superpixel's boundary edges.
// The lane walks its segment in order and adds to the accumulators once per
// run of equal labels.
struct GlobalSink {
    int64_t *facc;
    __device__ void operator()(int32_t k, const FeatAcc &v) const { feat_flush(facc, k, v); }
};

template <class Sink>
__device__ __forceinline__ void feat_segment(const Job &J, const int32_t *row, const int32_t *up, const int32_t *dn,
                                             int B, int nbx, int by, int bx0, int bx1,
                                             const uint32_t *__restrict__ moms, const int32_t *fmean,
                                             const Sink &sink)
{
    const int W = J.W, H = J.H;
    const int y0 = by * B, y1 = min(y0 + B, H);
    int32_t cur = -1;
    FeatAcc v;
    feat_zero(v);
    int32_t left = bx0 > 0 ? row[bx0 - 1] : -1;
    int32_t k = row[bx0];
    for (int bx = bx0; bx < bx1; bx++) {
        const int32_t right = bx + 1 < nbx ? row[bx + 1] : -1;
        if (k != cur) {
            if (cur >= 0) sink(cur, v);
            cur = k;
            feat_zero(v);
        }
        const int x0 = bx * B, x1 = min(x0 + B, W);
        const int64_t i = (int64_t)by * nbx + bx;
        if (moms) {
            v.q[0] += moms[3 * i];
            v.q[1] += moms[3 * i + 1];
            v.q[2] += moms[3 * i + 2];
        } else {
            for (int y = y0; y < y1; y++) {
                const uint8_t *px = J.rgb + (int64_t)y * J.rgb_stride + 3 * (int64_t)x0;
                for (int x = 0; x < x1 - x0; x++) {
                    const int r = px[3 * x], gg = px[3 * x + 1], b = px[3 * x + 2];
                    v.q[0] += r * r;
                    v.q[1] += gg * gg;
                    v.q[2] += b * b;
                }
            }
        }
        const int32_t nbr[4] = {left, right, up ? up[bx] : -1, dn ? dn[bx] : -1};
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const int32_t j = nbr[d];
            if (j < 0 || j == k) continue;
            const int64_t e = d < 2 ? (y1 - y0) : (x1 - x0);
            int64_t d2 = 0, bj = 0;
            for (int ch = 0; ch < 3; ch++) {
                const int64_t df = (int64_t)fmean[3 * k + ch] - fmean[3 * j + ch];
                d2 += df * df;
                bj += fmean[3 * j + ch];
            }
            v.bl += e;
            v.ed2 += e * d2;
            v.nbs += e * bj;
            v.mx = (uint64_t)d2 > v.mx ? (uint64_t)d2 : v.mx;
            v.mn = (uint64_t)d2 < v.mn ? (uint64_t)d2 : v.mn;
        }
        left = k;
        k = right;
    }
    if (cur >= 0) sink(cur, v);
}

// Step C for superpixel k (double arithmetic without contraction, so that
// every value is the correctly rounded result of the same expression on any
// IEEE machine).  fset RAPID_FEATURES_LEARNED, the sixteen features of the
// learned gate:
//   0-2 mean colour / 255, 3-5 colour std / 64, 6 size / A, 7 boundary
//   length / (4 sqrt A), 8 compactness bl^2 / (16 n), 9 centroid drift from
//   the initial cell centre / sqrt A, 10-12 max / edge-weighted rms / min
//   neighbour contrast / (255 2^F), 13 moved pixels / n, 14 max colour std
//   / 64, 15 one.
// fset RAPID_FEATURES_ROI, the paper's four ROI features (Sec. 4): 0
// absolute brightness / 255, 1 comparative brightness (own minus the
// edge-weighted neighbour brightness) / 255, 2 extra-region dissimilarity
// (edge-weighted rms mean-colour distance to the neighbours) / (255 2^F),
// 3 intra-region dissimilarity (sqrt of the mean channel variance) / 64,
// 4-14 zero, 15 one.
__device__ __forceinline__ void feat_final_sp(const Job &J, const int64_t *st, const int64_t *facc,
                                              const int64_t *moved, int k, int F, int fset, float *f)
{
#pragma clang fp contract(off)
    const double A = (double)(((int64_t)J.W * J.H) / J.K);
    const double sA = sqrt(A);
    const double cs = 255.0 * (double)(1 << F);
    const int64_t *r = st + 6 * (int64_t)k;
    const int64_t *a = facc + FACC * (int64_t)k;
    if (r[0] == 0) {   // merged away: all features 0
        for (int i = 0; i < 16; i++) f[i] = 0.0f;
        return;
    }
    const double n = (double)r[0];
    if (fset == RAPID_FEATURES_ROI) {
        const double br = ((double)r[1] + (double)r[2] + (double)r[3]) / (3.0 * n);
        double var = 0.0;
        for (int ch = 0; ch < 3; ch++) {
            const double mu = (double)r[1 + ch] / n;
            const double v = (double)a[ch] / n - mu * mu;
            var += v > 0.0 ? v : 0.0;
        }
        const double bl = (double)a[3];
        f[0] = (float)(br / 255.0);
        f[1] = (float)(a[3] ? (br - (double)a[5] / (3.0 * bl * (double)(1 << F))) / 255.0 : 0.0);
        f[2] = (float)(a[3] ? sqrt((double)a[4] / bl) / cs : 0.0);
        f[3] = (float)(sqrt(var / 3.0) / 64.0);
        for (int i = 4; i < 15; i++) f[i] = 0.0f;
        f[15] = 1.0f;
        return;
    }
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
