// rapid_gate.hip -- the prediction gate of RAPID on gfx950.
//
// Algorithm RAPID extracts features of every superpixel at the second level
// and classifies it (Eq. (6)); past that point only "boundary superpixel"
// pairs are refined (Eq. (7)).  Here the classifier is a small MLP
// 16 -> 64 -> 64 -> 1 (ReLU, logistic output) evaluated and trained with
// bf16 MFMA (v_mfma_f32_16x16x16bf16_1k) and fp32 accumulation.
//
// MLP layout: the layers are computed transposed, H^T = W X^T, so the
// weights are the MFMA A operand and the activations the B operand.  The
// D fragment of layer l (lane holds rows 4*(lane/16)+r, column lane%16) is
// then exactly the B fragment of layer l+1 for the matching K step: no data
// movement between layers.
//
// Parameter vector (5313 values): W1 (64x16, row = output neuron), b1 (64),
// W2 (64x64), b2 (64), w3 (64), b3 (1).
#include "rapid_gate_dev.h"

namespace rapid {

// ------------------------------------------------------------- features

// Stand-alone feature passes (one job per blockIdx.y); the steps are the
// device functions of rapid_gate_dev.h.
__global__ void k_feat_init(const Job *__restrict__ jobs, int F)
{
    const Job &J = jobs[blockIdx.y];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < J.K; k += gridDim.x * blockDim.x)
        feat_init_sp(J.stats, J.fmean, J.facc, k, F);
}

__global__ void k_feat_blocks(const Job *__restrict__ jobs, int B, int lab_buf)
{
    const Job &J = jobs[blockIdx.y];
    const int nbx = (J.W + B - 1) / B, nby = (J.H + B - 1) / B;
    const int spr = (nbx + FEAT_SEG - 1) / FEAT_SEG;
    const int64_t nseg = (int64_t)spr * nby;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t *L = J.lab[lab_buf];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nseg; g += stride) {
        const int by = (int)(g / spr), bx0 = (int)(g % spr) * FEAT_SEG;
        const int32_t *row = L + (int64_t)by * nbx;
        feat_segment(J, row, by > 0 ? row - nbx : nullptr, by + 1 < nby ? row + nbx : nullptr, B, nbx, by, bx0,
                     min(bx0 + FEAT_SEG, nbx), nullptr, J.fmean, GlobalSink{J.facc});
    }
}

__global__ void k_feat_final(const Job *__restrict__ jobs, const int64_t *__restrict__ xoff, int F, int fset,
                             float *__restrict__ X)
{
    const Job &J = jobs[blockIdx.y];
    float *Xj = X + 16 * xoff[blockIdx.y];
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < J.K; k += gridDim.x * blockDim.x)
        feat_final_sp(J, J.stats, J.facc, J.moved, k, F, fset, Xj + 16 * (int64_t)k);
}

// ------------------------------------------------------------ MLP forward

struct WFrag {
    v4s a1[4];        // W1 rows 16i + lane%16, inputs 4*(lane/16) + r
    v4s a2[4][4];     // W2 rows 16i + lane%16, inputs 16j + 4*(lane/16) + r
    v4s a3[4];        // w3 inputs 16j + 4*(lane/16) + r in row 0 only
    float b1[4][4], b2[4][4], b3;
};

__device__ __forceinline__ void load_wfrag(WFrag &w, const uint16_t *__restrict__ P, int lane)
{
    const int col = lane & 15, grp = lane >> 4;
    for (int i = 0; i < 4; i++) {
        w.a1[i] = load4bf(P + P_W1 + (16 * i + col) * 16 + 4 * grp);
        for (int j = 0; j < 4; j++) w.a2[i][j] = load4bf(P + P_W2 + (16 * i + col) * 64 + 16 * j + 4 * grp);
        if (col == 0) {
            w.a3[i] = load4bf(P + P_W3 + 16 * i + 4 * grp);
        } else {
            v4s z = {0, 0, 0, 0};
            w.a3[i] = z;
        }
        for (int r = 0; r < 4; r++) {
            w.b1[i][r] = bf2f(P[P_B1 + 16 * i + 4 * grp + r]);
            w.b2[i][r] = bf2f(P[P_B2 + 16 * i + 4 * grp + r]);
        }
    }
    w.b3 = bf2f(P[P_B3]);
}

// One 16-sample tile: x fragment in B layout (features 4*(lane/16)+r of
// sample lane%16).  Outputs the pre-activations of both hidden layers
// (D layout), their bf16 activations (B layout) and the logit (lanes 0-15).
struct Fwd {
    v4f a1[4], a2[4];
    v4s h1[4], h2[4];
    float z;
};

__device__ __forceinline__ void mlp_tile(const WFrag &w, v4s bx, int lane, Fwd &o)
{
    const int grp = lane >> 4;
    for (int i = 0; i < 4; i++) {
        v4f c = {w.b1[i][0], w.b1[i][1], w.b1[i][2], w.b1[i][3]};
        c = mfma(w.a1[i], bx, c);
        o.a1[i] = c;
        o.h1[i] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    }
    for (int i = 0; i < 4; i++) {
        v4f c = {w.b2[i][0], w.b2[i][1], w.b2[i][2], w.b2[i][3]};
        for (int j = 0; j < 4; j++) c = mfma(w.a2[i][j], o.h1[j], c);
        o.a2[i] = c;
        o.h2[i] = pack4(fmaxf(c[0], 0.f), fmaxf(c[1], 0.f), fmaxf(c[2], 0.f), fmaxf(c[3], 0.f));
    }
    v4f c = {grp == 0 ? w.b3 : 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 4; j++) c = mfma(w.a3[j], o.h2[j], c);
    o.z = c[0];   // row 0: meaningful in lanes 0-15
}

// logits of N samples; gate[n] = logit >= thresh (gate may be null).  One
// wave per 16-sample tile.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ X, int64_t N,
                                                 const uint16_t *__restrict__ P, float thresh,
                                                 float *__restrict__ logits, uint8_t *__restrict__ gate)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t ntiles = (N + 15) / 16;
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t n = 16 * t + (lane & 15);
        const float z = mlp_logit(P, load_x(X, n, N, lane >> 4), lane);
        if (lane < 16 && n < N) {
            if (logits) logits[n] = z;
            if (gate) gate[n] = z >= thresh ? 1 : 0;
        }
    }
}

// ----------------------------------------------------------- MLP training

// The staging tiles are private to a wave: its LDS writes complete in
// order, so a wait on the LDS counter plus a compiler barrier orders the
// writes of one lane before the reads of another (and reads before
// overwrites).
__device__ __forceinline__ void lds_fence()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Butterfly sum over the 16 lanes that share lane/16 (fixed order).
__device__ __forceinline__ float sum16(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Gradient of the mean binary cross-entropy with logits over a batch of
// samples idx[0..nb) (scale = 1 / batch size).  Each wave takes tiles
// t = wave, wave + nwaves, ... and writes its partial gradient (5313
// floats) to part[wave]; k_grad_reduce sums the partials in wave order.
// Rounding to bf16 happens where the reference rounds: inputs, weights,
// hidden activations and back-propagated hidden gradients.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X, const uint8_t *__restrict__ T,
                                                  const int32_t *__restrict__ idx, int32_t nb, float scale,
                                                  const uint16_t *__restrict__ P, float *__restrict__ part,
                                                  float *__restrict__ logits)
{
    __shared__ float s_t[4][2][64][17];   // per wave: two 64 x 16 tiles (padded)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    WFrag w;
    load_wfrag(w, P, lane);
    // W2 transposed as A operand: rows k = 16m + col, inputs i = 16j + 4 grp + r
    v4s a2t[4][4];
    float w3v[4][4];
    for (int m = 0; m < 4; m++)
        for (int j = 0; j < 4; j++) {
            v4s v;
            for (int r = 0; r < 4; r++) v[r] = (short)P[P_W2 + (16 * j + 4 * grp + r) * 64 + 16 * m + col];
            a2t[m][j] = v;
        }
    for (int j = 0; j < 4; j++)
        for (int r = 0; r < 4; r++) w3v[j][r] = bf2f(P[P_W3 + 16 * j + 4 * grp + r]);
    v4f gW2[4][4], gW1[4];
    float gb1[4][4], gb2[4][4], gw3[4][4], gb3 = 0.f;
    for (int i = 0; i < 4; i++) {
        for (int j = 0; j < 4; j++) gW2[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
        gW1[i] = (v4f){0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < 4; r++) gb1[i][r] = gb2[i][r] = gw3[i][r] = 0.f;
    }
    float(*tA)[17] = s_t[wv][0];
    float(*tB)[17] = s_t[wv][1];
    const int64_t ntiles = (nb + 15) / 16;
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t e = 16 * t + col;             // this lane's sample slot
        const bool valid = e < nb;
        const int64_t n = valid ? idx[e] : 0;
        Fwd o;
        mlp_tile(w, valid ? load_x(X, n, 0x7fffffffffffffffLL, grp) : (v4s){0, 0, 0, 0}, lane, o);
        // dz of sample col, computed in lanes 0-15 and broadcast
        float dz = 0.f;
        if (lane < 16 && valid) {
            const float p = 1.f / (1.f + __expf(-o.z));
            dz = (p - (float)T[n]) * scale;
            if (logits) logits[e] = o.z;
        }
        dz = __shfl(dz, col);
        if (grp == 0) gb3 += dz;
        // layer 3 and dH2 (D layout of layer 2: rows 16i + 4 grp + r, sample col)
        v4s dh2[4];
        for (int i = 0; i < 4; i++) {
            float v[4];
            for (int r = 0; r < 4; r++) {
                gw3[i][r] += dz * bf2f((uint16_t)o.h2[i][r]);
                v[r] = o.a2[i][r] > 0.f ? w3v[i][r] * dz : 0.f;
            }
            dh2[i] = pack4(v[0], v[1], v[2], v[3]);
            for (int r = 0; r < 4; r++) gb2[i][r] += bf2f((uint16_t)dh2[i][r]);
        }
        // dH1^T = W2^T dH2^T, masked
        v4s dh1[4];
        for (int m = 0; m < 4; m++) {
            v4f c = {0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j < 4; j++) c = mfma(a2t[m][j], dh2[j], c);
            float v[4];
            for (int r = 0; r < 4; r++) v[r] = o.a1[m][r] > 0.f ? c[r] : 0.f;
            dh1[m] = pack4(v[0], v[1], v[2], v[3]);
            for (int r = 0; r < 4; r++) gb1[m][r] += bf2f((uint16_t)dh1[m][r]);
        }
        // stage dH2^T and H1^T (rows = neurons, columns = samples) for the
        // weight-gradient products, which need samples as the K dimension
        for (int i = 0; i < 4; i++)
            for (int r = 0; r < 4; r++) {
                tA[16 * i + 4 * grp + r][col] = bf2f((uint16_t)dh2[i][r]);
                tB[16 * i + 4 * grp + r][col] = bf2f((uint16_t)o.h1[i][r]);
            }
        lds_fence();
        // dW2[i][k] += sum_n dH2^T[i][n] H1^T[k][n]: A = dH2^T tile i
        // (row 16i + col, samples 4 grp + r), B = H1 (samples 4 grp + r,
        // neuron 16j + col)
        for (int i = 0; i < 4; i++) {
            const v4s A = pack4(tA[16 * i + col][4 * grp], tA[16 * i + col][4 * grp + 1],
                                tA[16 * i + col][4 * grp + 2], tA[16 * i + col][4 * grp + 3]);
            for (int j = 0; j < 4; j++) {
                const v4s Bf = pack4(tB[16 * j + col][4 * grp], tB[16 * j + col][4 * grp + 1],
                                     tB[16 * j + col][4 * grp + 2], tB[16 * j + col][4 * grp + 3]);
                gW2[i][j] = mfma(A, Bf, gW2[i][j]);
            }
        }
        lds_fence();
        // stage dH1^T; dW1[i][f] += sum_n dH1^T[i][n] X[n][f]
        for (int m = 0; m < 4; m++)
            for (int r = 0; r < 4; r++) tA[16 * m + 4 * grp + r][col] = bf2f((uint16_t)dh1[m][r]);
        lds_fence();
        v4s bxs;
        {
            float v[4];
            for (int r = 0; r < 4; r++) {
                const int64_t es = 16 * t + 4 * grp + r;
                v[r] = es < nb ? X[16 * (int64_t)idx[es] + col] : 0.f;
            }
            bxs = pack4(v[0], v[1], v[2], v[3]);
        }
        for (int i = 0; i < 4; i++) {
            const v4s A = pack4(tA[16 * i + col][4 * grp], tA[16 * i + col][4 * grp + 1],
                                tA[16 * i + col][4 * grp + 2], tA[16 * i + col][4 * grp + 3]);
            gW1[i] = mfma(A, bxs, gW1[i]);
        }
        lds_fence();
    }
    // write this wave's partial gradient
    float *out = part + wave * (int64_t)MLP_PARAMS;
    for (int i = 0; i < 4; i++)
        for (int r = 0; r < 4; r++) {
            const int row = 16 * i + 4 * grp + r;
            out[P_W1 + row * 16 + col] = gW1[i][r];
            for (int j = 0; j < 4; j++) out[P_W2 + row * 64 + 16 * j + col] = gW2[i][j][r];
            const float s1 = sum16(gb1[i][r]), s2 = sum16(gb2[i][r]), s3 = sum16(gw3[i][r]);
            if (col == 0) {
                out[P_B1 + row] = s1;
                out[P_B2 + row] = s2;
                out[P_W3 + row] = s3;
            }
        }
    const float sb3 = sum16(gb3);
    if (lane == 0) out[P_B3] = sb3;
}

// grads[p] = sum over waves w = 0 .. nw-1 of part[w][p], in that order.
__global__ void k_grad_reduce(const float *__restrict__ part, int nw, float *__restrict__ grads)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int w = 0; w < nw; w++) s += part[(int64_t)w * MLP_PARAMS + p];
        grads[p] = s;
    }
}

// One Adam step (step counts from 1) on the fp32 master weights; the bf16
// copy is refreshed from them.
__global__ void k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, uint16_t *__restrict__ wbf, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x) {
        const float gp = g[p];
        const float mp = b1 * m[p] + (1.f - b1) * gp;
        const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
        m[p] = mp;
        v[p] = vp;
        const float th = theta[p] - lr * (mp / c1) / (sqrtf(vp / c2) + eps);
        theta[p] = th;
        wbf[p] = f2bf(th);
    }
}

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = f2bf(src[i]);
}

// ------------------------------------------------- boundary-recall misses

// Boundary pixels of `ref` (a 4-neighbour with another label) with no
// boundary pixel of `test` within Chebyshev distance r: the misses of the
// boundary recall of Sec. 4.2.  Each miss adds 1 to miss[ref label] and 1 to
// miss[test label]; totals gets (ref boundary pixels, misses).  One
// workgroup per 64 x 16 pixel tile; the test boundary of the tile plus an
// r-pixel apron is staged in LDS as bytes.
constexpr int BM_TX = 64, BM_TY = 16, BM_RMAX = 4;

__device__ __forceinline__ bool is_bnd(const int32_t *__restrict__ M, int x, int y, int W, int H, int64_t stride)
{
    const int32_t *row = M + (int64_t)y * stride;
    const int32_t l = row[x];
    return (x > 0 && row[x - 1] != l) || (x + 1 < W && row[x + 1] != l) ||
           (y > 0 && row[x - stride] != l) || (y + 1 < H && row[x + stride] != l);
}

__global__ __launch_bounds__(256) void k_boundary_miss(const int32_t *__restrict__ ref,
                                                       const int32_t *__restrict__ test, int W, int H,
                                                       int64_t stride, int r, int32_t K,
                                                       int32_t *__restrict__ miss,
                                                       unsigned long long *__restrict__ totals)
{
    __shared__ uint8_t tb[(BM_TY + 2 * BM_RMAX) * (BM_TX + 2 * BM_RMAX)];
    __shared__ unsigned s_tot[2];
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * BM_TX, y0 = blockIdx.y * BM_TY;
    const int EW = BM_TX + 2 * r, EH = BM_TY + 2 * r;
    if (tid < 2) s_tot[tid] = 0;
    for (int i = tid; i < EW * EH; i += 256) {
        const int x = x0 - r + i % EW, y = y0 - r + i / EW;
        tb[i] = (x >= 0 && y >= 0 && x < W && y < H) ? is_bnd(test, x, y, W, H, stride) : 0;
    }
    __syncthreads();
    unsigned nb = 0, nm = 0;
    for (int i = tid; i < BM_TX * BM_TY; i += 256) {
        const int tx = i % BM_TX, ty = i / BM_TX;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H || !is_bnd(ref, x, y, W, H, stride)) continue;
        nb++;
        bool near = false;
        for (int dy = 0; dy <= 2 * r && !near; dy++)
            for (int dx = 0; dx <= 2 * r; dx++) near |= tb[(ty + dy) * EW + tx + dx] != 0;
        if (near) continue;
        nm++;
        if (miss) {
            const int64_t o = (int64_t)y * stride + x;
            const int32_t la = ref[o], lb = test[o];
            if ((uint32_t)la < (uint32_t)K) atomicAdd(&miss[la], 1);
            if ((uint32_t)lb < (uint32_t)K) atomicAdd(&miss[lb], 1);
        }
    }
    if (nb) atomicAdd(&s_tot[0], nb);
    if (nm) atomicAdd(&s_tot[1], nm);
    __syncthreads();
    if (tid == 0 && totals) {
        atomicAdd(&totals[0], (unsigned long long)s_tot[0]);
        atomicAdd(&totals[1], (unsigned long long)s_tot[1]);
    }
}

// ------------------------------------------------------------- launchers

hipError_t launch_boundary_miss(const int32_t *ref, const int32_t *test, int W, int H, int64_t stride, int r,
                                int32_t K, int32_t *miss, int64_t *totals, hipStream_t stream)
{
    dim3 grid((unsigned)((W + BM_TX - 1) / BM_TX), (unsigned)((H + BM_TY - 1) / BM_TY));
    hipLaunchKernelGGL(k_boundary_miss, grid, dim3(256), 0, stream, ref, test, W, H, stride, r, K, miss,
                       reinterpret_cast<unsigned long long *>(totals));
    return hipGetLastError();
}

hipError_t launch_features(const Job *jobs_dev, int n_jobs, int B, int lab_buf, int F, int fset, int32_t Kmax,
                           int64_t max_nb, const int64_t *xoff_dev, float *X, hipStream_t stream)
{
    unsigned gk = (unsigned)std::max<int64_t>(1, std::min<int64_t>((Kmax + 255) / 256, 1024));
    unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_nb + 255) / 256, 4096));
    hipLaunchKernelGGL(k_feat_init, dim3(gk, n_jobs), dim3(256), 0, stream, jobs_dev, F);
    hipLaunchKernelGGL(k_feat_blocks, dim3(gb, n_jobs), dim3(256), 0, stream, jobs_dev, B, lab_buf);
    hipLaunchKernelGGL(k_feat_final, dim3(gk, n_jobs), dim3(256), 0, stream, jobs_dev, xoff_dev, F, fset, X);
    return hipGetLastError();
}

hipError_t launch_mlp_fwd(const float *X, int64_t N, const uint16_t *P, float thresh, float *logits,
                          uint8_t *gate, hipStream_t stream)
{
    int64_t tiles = (N + 15) / 16;
    int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 2048));
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)blocks), dim3(256), 0, stream, X, N, P, thresh, logits, gate);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *X, const uint8_t *T, const int32_t *idx, int32_t nb, float scale,
                           const uint16_t *P, float *part, int n_waves, float *grads, float *logits,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)(n_waves / 4)), dim3(256), 0, stream, X, T, idx, nb, scale, P,
                       part, logits);
    hipLaunchKernelGGL(k_grad_reduce, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, stream, part, n_waves, grads);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *g, uint16_t *wbf, float lr, float b1,
                       float b2, float eps, int step, hipStream_t stream)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, stream, theta, m, v, g, wbf, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024))),
                       dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

}  // namespace rapid
