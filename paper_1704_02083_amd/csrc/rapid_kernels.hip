// rapid_kernels.hip -- gfx950 kernels of the RAPID refinement sweep.
//
// One workgroup owns one image (or tile): every phase of the sweep is a
// workgroup-wide pass separated by workgroup barriers, so the ~10^3 dependent
// phases of a segmentation never leave the CU.  Per-superpixel statistics
// live in LDS when they fit (integer LDS atomics), else in the image's own
// global scratch.  Labels, block sums and work lists live in HBM/L2.
//
// The sweep (paper: CTFTPS energy Eq. (1), move Eq. (3), boundary rule
// Eq. (2)/(7), size regularity Sec. 3.1, stage loop of Algorithm RAPID):
//   for each stage (block size B):
//     split the previous label map (or lay the grid), scan for boundary blocks
//     for each sweep: for each of the 9 classes (bx mod 3, by mod 3):
//       P1 propose from the class-start state (size, topology, argmin E')
//       P2 class-wide size filter, commit, integer stat moves
//       P3 refresh means of touched superpixels, clear the flow counters
//     rebuild the boundary set around changed blocks
#include "rapid_internal.h"

namespace rapid {

__device__ __forceinline__ int lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Wave-aggregated append: one LDS/global atomic per wave.  Returns the slot
// of a thread whose pred is true, -1 otherwise.
__device__ __forceinline__ int wave_append(int32_t *counter, bool pred)
{
    uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((unsigned long long)m) - 1;
    int prefix = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    return pred ? base + prefix : -1;
}

__device__ __forceinline__ void wave_count(unsigned long long *ctr, bool pred)
{
    uint64_t m = __ballot(pred);
    if (m == 0) return;
    int leader = __ffsll((unsigned long long)m) - 1;
    if (lane_id() == leader) atomicAdd(ctr, (unsigned long long)__popcll(m));
}

__device__ __forceinline__ void add64(int64_t *p, int64_t v)
{
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

struct Geo {
    int32_t w, h;
    int64_t m, px, py;
};

// Block (bx, by) of size B clipped to the image, its pixel count and its
// coordinate sums (h * sum x, w * sum y) in closed form.
__device__ __forceinline__ Geo block_geo(int bx, int by, int B, int W, int H)
{
    Geo g;
    int x0 = bx * B, y0 = by * B;
    int x1 = min(x0 + B, W), y1 = min(y0 + B, H);
    g.w = x1 - x0;
    g.h = y1 - y0;
    g.m = (int64_t)g.w * g.h;
    g.px = (int64_t)g.h * (((int64_t)(x0 + x1 - 1) * g.w) >> 1);
    g.py = (int64_t)g.w * (((int64_t)(y0 + y1 - 1) * g.h) >> 1);
    return g;
}

__device__ __forceinline__ void block_rgb(const Job &J, int s, int B, int64_t bi, int bx, int by,
                                          int64_t I[3])
{
    if (B == 1) {
        const uint8_t *p = J.rgb + (int64_t)by * J.rgb_stride + 3 * (int64_t)bx;
        I[0] = p[0];
        I[1] = p[1];
        I[2] = p[2];
    } else {
        uint64_t v = J.sums[s][bi];
        I[0] = (int64_t)(v & 0x1FFFFFull);
        I[1] = (int64_t)((v >> 21) & 0x1FFFFFull);
        I[2] = (int64_t)(v >> 42);
    }
}

// E'(beta, k) of the block with the means of k held fixed (Eq. (1) minus
// the terms that do not depend on k; difference form of Sec. 3.1).
__device__ __forceinline__ int64_t block_energy(const int32_t *mn, int k, const Geo &g,
                                                const int64_t I[3], int bnd, const Sched &sc)
{
    const int32_t *c = mn + MN_STRIDE * (int64_t)k;
    int64_t c0 = c[0], c1 = c[1], c2 = c[2], mx = c[3], my = c[4];
    int64_t col = c0 * c0 + c1 * c1 + c2 * c2;
    int64_t dot = c0 * I[0] + c1 * I[1] + c2 * I[2];
    int64_t e_col = g.m * col - (dot << (sc.F + 1));
    int64_t pos = mx * mx + my * my;
    int64_t pdot = mx * g.px + my * g.py;
    int64_t e_pos = g.m * pos - (pdot << (sc.F + 1));
    return sc.w_col * e_col + sc.w_pos * e_pos + ((sc.w_bnd * (int64_t)bnd) << (2 * sc.F));
}

// Means in fixed point, rounded half up, plus the size n: the class-start
// snapshot that every proposal and every size-filter decision of the next
// class reads while the integer atomics of that class update the sums.
__device__ __forceinline__ void refresh_means(const int64_t *st, int32_t *mn, int k, int F)
{
    const int64_t *r = st + 6 * (int64_t)k;
    int64_t n = r[0];
    int64_t d = 2 * n;
    int32_t *o = mn + MN_STRIDE * (int64_t)k;
#pragma unroll
    for (int q = 0; q < 5; q++) o[q] = (int32_t)(((r[1 + q] << (F + 1)) + n) / d);
    o[5] = (int32_t)n;
}

__device__ __forceinline__ int32_t lab_at(const int32_t *L, int bx, int by, int nbx, int nby)
{
    return (bx >= 0 && by >= 0 && bx < nbx && by < nby) ? L[(int64_t)by * nbx + bx] : -1;
}

__device__ __forceinline__ bool pair_on(const uint8_t *gate, int a, int k)
{
    return gate == nullptr || gate[a] || gate[k];
}

__device__ __forceinline__ bool eligible(const int32_t *L, int bx, int by, int nbx, int nby,
                                         const uint8_t *gate)
{
    int32_t a = L[(int64_t)by * nbx + bx];
    int32_t k;
    if ((k = lab_at(L, bx - 1, by, nbx, nby)) >= 0 && k != a && pair_on(gate, a, k)) return true;
    if ((k = lab_at(L, bx + 1, by, nbx, nby)) >= 0 && k != a && pair_on(gate, a, k)) return true;
    if ((k = lab_at(L, bx, by - 1, nbx, nby)) >= 0 && k != a && pair_on(gate, a, k)) return true;
    if ((k = lab_at(L, bx, by + 1, nbx, nby)) >= 0 && k != a && pair_on(gate, a, k)) return true;
    return false;
}

__device__ __forceinline__ void wg_sync()
{
    __syncthreads();
}

// --------------------------------------------------------------- k_sums
// Packed per-block RGB sums (21 bits per channel) for a stage of block size B.
__global__ void k_block_sums(const Job *__restrict__ jobs, int s, int B)
{
    const Job &J = jobs[blockIdx.y];
    int nbx = (J.W + B - 1) / B, nby = (J.H + B - 1) / B;
    int64_t nb = (int64_t)nbx * nby;
    uint64_t *out = J.sums[s];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb;
         i += (int64_t)gridDim.x * blockDim.x) {
        int bx = (int)(i % nbx), by = (int)(i / nbx);
        int x0 = bx * B, y0 = by * B;
        int x1 = min(x0 + B, J.W), y1 = min(y0 + B, J.H);
        uint32_t r = 0, g = 0, b = 0;
        for (int y = y0; y < y1; y++) {
            const uint8_t *row = J.rgb + (int64_t)y * J.rgb_stride + 3 * (int64_t)x0;
            for (int x = 0; x < x1 - x0; x++) {
                r += row[3 * x];
                g += row[3 * x + 1];
                b += row[3 * x + 2];
            }
        }
        out[i] = (uint64_t)r | ((uint64_t)g << 21) | ((uint64_t)b << 42);
    }
}

// ------------------------------------------------------------- k_expand
// Block labels of size B to pixel labels (row stride in elements).
__global__ void k_expand(const int32_t *__restrict__ L, int W, int H, int B,
                         int32_t *__restrict__ out, int64_t stride)
{
    int nbx = (W + B - 1) / B;
    int64_t N = (int64_t)W * H;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        int x = (int)(i % W), y = (int)(i / W);
        out[(int64_t)y * stride + x] = L[(int64_t)(y / B) * nbx + x / B];
    }
}

// ------------------------------------------------------------- k_refine
template <bool LDS>
__global__ __launch_bounds__(1024) void k_refine(const Job *__restrict__ jobs, Sched sc,
                                                  int s_begin, int s_end, int flags,
                                                  const uint32_t *__restrict__ lut_g)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_lut[8];
    __shared__ int32_t s_cnt[9];
    __shared__ int32_t s_nprop, s_nchg, s_ntch, s_commits;
    __shared__ unsigned long long s_ctr[5];   // active proposals commits skip_min skip_topo

    const Job &J = jobs[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int W = J.W, H = J.H, K = J.K;
    int64_t *st;
    int32_t *mn, *fl, *tch, *tl;
    if (LDS) {
        st = reinterpret_cast<int64_t *>(smem);
        mn = reinterpret_cast<int32_t *>(st + 6 * (int64_t)K);  // K x MN_STRIDE
    } else {
        st = J.stats;
        mn = J.means;
    }
    fl = LDS ? mn + MN_STRIDE * (int64_t)K : J.flow;
    tch = LDS ? fl + 2 * (int64_t)K : J.touched;
    tl = LDS ? tch + K : J.touched + K;

    if (tid < 8) s_lut[tid] = lut_g[tid];
    if (tid == 0) {
        s_nprop = 0;
        s_nchg = 0;
        s_ntch = 0;
        s_commits = 0;
    }
    for (int64_t i = tid; i < 2 * (int64_t)K; i += nt) fl[i] = 0;
    for (int64_t i = tid; i < K; i += nt) tch[i] = 0;

    if (flags & FLAG_INIT) {
        // grid initialisation (Algorithm RAPID, first step) and the
        // statistics, computed once for all levels (Sec. 3.2)
        for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) st[i] = 0;
        wg_sync();
        const int B0 = sc.B[0];
        const int nbx = (W + B0 - 1) / B0, nby = (H + B0 - 1) / B0;
        int32_t *L = J.lab[0];
        for (int64_t i = tid; i < (int64_t)nbx * nby; i += nt) {
            int bx = (int)(i % nbx), by = (int)(i / nbx);
            Geo g = block_geo(bx, by, B0, W, H);
            int64_t row = ((2 * (int64_t)by * B0 + g.h) * J.gy) / (2 * (int64_t)H);
            int64_t col = ((2 * (int64_t)bx * B0 + g.w) * J.gx) / (2 * (int64_t)W);
            int32_t k = (int32_t)(row * J.gx + col);
            L[i] = k;
            int64_t I[3];
            block_rgb(J, 0, B0, i, bx, by, I);
            int64_t *r = st + 6 * (int64_t)k;
            add64(r + 0, g.m);
            add64(r + 1, I[0]);
            add64(r + 2, I[1]);
            add64(r + 3, I[2]);
            add64(r + 4, g.px);
            add64(r + 5, g.py);
        }
    } else if (LDS) {
        for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) st[i] = J.stats[i];
    }
    wg_sync();
    for (int64_t k = tid; k < K; k += nt) refresh_means(st, mn, (int)k, sc.F);
    wg_sync();

    const int64_t capc = J.capc;
    for (int s = s_begin; s < s_end; s++) {
        const int B = sc.B[s];
        const int nbx = (W + B - 1) / B, nby = (H + B - 1) / B;
        const int64_t nb = (int64_t)nbx * nby;
        int32_t *L = J.lab[s & 1];
        const uint8_t *gate = (J.gate && s >= sc.gate_stage) ? J.gate : nullptr;
        if (s > 0) {
            // split: each block inherits the label of the block that holds it
            const int Bp = sc.B[s - 1];
            const int nbxp = (W + Bp - 1) / Bp;
            const int32_t *Lp = J.lab[(s - 1) & 1];
            const int r = Bp / B;
            for (int64_t i = tid; i < nb; i += nt) {
                int bx = (int)(i % nbx), by = (int)(i / nbx);
                L[i] = Lp[(int64_t)(by / r) * nbxp + bx / r];
            }
        }
        if (tid < 9) s_cnt[tid] = 0;
        if (tid < 5) s_ctr[tid] = 0;
        wg_sync();
        // boundary blocks of the stage (Eq. (2); Eq. (7) under the gate)
        for (int64_t i0 = 0; i0 < nb; i0 += nt) {
            int64_t i = i0 + tid;
            bool e = false;
            int cls = 0;
            if (i < nb) {
                int bx = (int)(i % nbx), by = (int)(i / nbx);
                J.stamp[i] = 0;
                e = eligible(L, bx, by, nbx, nby, gate);
                cls = 3 * (by % 3) + (bx % 3);
            }
            // one append per class: loop over the classes present in the wave
            for (int c = 0; c < 9; c++) {
                int slot = wave_append(&s_cnt[c], e && cls == c);
                if (slot >= 0) J.lists[c * capc + slot] = (int32_t)i;
            }
        }
        wg_sync();

        int sweeps = 0, converged = 0;
        for (int t = 0; t < sc.max_sweeps; t++) {
            if (tid == 0) {
                int64_t tot = 0;
                for (int c = 0; c < 9; c++) tot += s_cnt[c];
                s_ctr[0] += (unsigned long long)tot;
                s_commits = 0;
            }
            wg_sync();
            for (int c = 0; c < 9; c++) {
                const int ncls = s_cnt[c];
                if (ncls == 0) continue;
                const int32_t *lst = J.lists + c * capc;
                // ---- P1: propose
                for (int e0 = 0; e0 < ncls; e0 += nt) {
                    int e = e0 + tid;
                    bool prop = false, smin = false, stopo = false;
                    int32_t bi = 0, a = 0, best = 0;
                    int64_t m = 0;
                    if (e < ncls) {
                        bi = lst[e];
                        int bx = bi % nbx, by = bi / nbx;
                        a = L[bi];
                        Geo g = block_geo(bx, by, B, W, H);
                        m = g.m;
                        if ((int64_t)mn[MN_STRIDE * (int64_t)a + 5] - g.m < sc.min_size) {
                            smin = true;
                        } else {
                            int32_t rl[8];
                            rl[0] = lab_at(L, bx - 1, by - 1, nbx, nby);
                            rl[1] = lab_at(L, bx, by - 1, nbx, nby);
                            rl[2] = lab_at(L, bx + 1, by - 1, nbx, nby);
                            rl[3] = lab_at(L, bx - 1, by, nbx, nby);
                            rl[4] = lab_at(L, bx + 1, by, nbx, nby);
                            rl[5] = lab_at(L, bx - 1, by + 1, nbx, nby);
                            rl[6] = lab_at(L, bx, by + 1, nbx, nby);
                            rl[7] = lab_at(L, bx + 1, by + 1, nbx, nby);
                            uint32_t mask = 0;
#pragma unroll
                            for (int q = 0; q < 8; q++) mask |= (rl[q] == a ? 1u : 0u) << q;
                            if (!((s_lut[mask >> 5] >> (mask & 31)) & 1u)) {
                                stopo = true;
                            } else {
                                // 4-neighbours W, E, N, S and their shared edge lengths
                                int32_t nl[4] = {rl[3], rl[4], rl[1], rl[6]};
                                int el[4] = {g.h, g.h, g.w, g.w};
                                int32_t cand[4];
                                int nc = 0;
#pragma unroll
                                for (int d = 0; d < 4; d++) {
                                    int32_t k = nl[d];
                                    bool ok = k >= 0 && k != a;
                                    for (int q = 0; q < d; q++) ok = ok && nl[q] != k;
                                    if (ok) cand[nc++] = k;
                                }
                                // ascending order
                                for (int u = 1; u < nc; u++)
                                    for (int v = u; v > 0 && cand[v - 1] > cand[v]; v--) {
                                        int32_t tmp = cand[v];
                                        cand[v] = cand[v - 1];
                                        cand[v - 1] = tmp;
                                    }
                                int64_t I[3];
                                block_rgb(J, s, B, bi, bx, by, I);
                                int bnd_a = 0;
#pragma unroll
                                for (int d = 0; d < 4; d++) bnd_a += (nl[d] >= 0 && nl[d] != a) ? el[d] : 0;
                                int64_t estar = block_energy(mn, a, g, I, bnd_a, sc);
                                best = a;
                                for (int u = 0; u < nc; u++) {
                                    int32_t k = cand[u];
                                    if ((int64_t)mn[MN_STRIDE * (int64_t)k + 5] + g.m > sc.max_size) continue;
                                    int bnd = 0;
#pragma unroll
                                    for (int d = 0; d < 4; d++) bnd += (nl[d] >= 0 && nl[d] != k) ? el[d] : 0;
                                    int64_t ek = block_energy(mn, k, g, I, bnd, sc);
                                    if (ek < estar) {
                                        estar = ek;
                                        best = k;
                                    }
                                }
                                prop = best != a && pair_on(gate, a, best);
                            }
                        }
                    }
                    wave_count(&s_ctr[3], smin);
                    wave_count(&s_ctr[4], stopo);
                    int slot = wave_append(&s_nprop, prop);
                    if (slot >= 0) {
                        J.props[3 * (int64_t)slot] = bi;
                        J.props[3 * (int64_t)slot + 1] = a;
                        J.props[3 * (int64_t)slot + 2] = best;
                        atomicAdd(&fl[2 * (int64_t)a], (int32_t)m);
                        atomicAdd(&fl[2 * (int64_t)best + 1], (int32_t)m);
                    }
                }
                wg_sync();
                const int np = s_nprop;
                if (np == 0) continue;   // uniform: nothing proposed in this class
                // ---- P2: class-wide size filter, commit, stat moves
                for (int e0 = 0; e0 < np; e0 += nt) {
                    int e = e0 + tid;
                    bool com = false;
                    int32_t bi = 0;
                    if (e < np) {
                        bi = J.props[3 * (int64_t)e];
                        int32_t a = J.props[3 * (int64_t)e + 1];
                        int32_t k = J.props[3 * (int64_t)e + 2];
                        // sizes from the class-start snapshot: the atomics of
                        // this phase are already moving the live counts
                        com = (int64_t)mn[MN_STRIDE * (int64_t)a + 5] - fl[2 * (int64_t)a] >= sc.min_size &&
                              (int64_t)mn[MN_STRIDE * (int64_t)k + 5] + fl[2 * (int64_t)k + 1] <= sc.max_size;
                        if (com) {
                            int bx = bi % nbx, by = bi / nbx;
                            Geo g = block_geo(bx, by, B, W, H);
                            int64_t I[3];
                            block_rgb(J, s, B, bi, bx, by, I);
                            L[bi] = k;
                            int64_t *ra = st + 6 * (int64_t)a, *rk = st + 6 * (int64_t)k;
                            add64(ra + 0, -g.m);
                            add64(rk + 0, g.m);
                            add64(ra + 1, -I[0]);
                            add64(rk + 1, I[0]);
                            add64(ra + 2, -I[1]);
                            add64(rk + 2, I[1]);
                            add64(ra + 3, -I[2]);
                            add64(rk + 3, I[2]);
                            add64(ra + 4, -g.px);
                            add64(rk + 4, g.px);
                            add64(ra + 5, -g.py);
                            add64(rk + 5, g.py);
                            if (atomicExch(&tch[a], 1) == 0) tl[atomicAdd(&s_ntch, 1)] = a;
                            if (atomicExch(&tch[k], 1) == 0) tl[atomicAdd(&s_ntch, 1)] = k;
                        }
                    }
                    int slot = wave_append(&s_nchg, com);
                    if (slot >= 0) J.changed[slot] = bi;
                    wave_count(&s_ctr[2], com);
                    {
                        uint64_t mk = __ballot(com);
                        if (mk && lane_id() == __ffsll((unsigned long long)mk) - 1)
                            atomicAdd(&s_commits, __popcll(mk));
                    }
                }
                wg_sync();
                // ---- P3: refresh means of touched superpixels, clear flows
                const int ntouch = s_ntch;
                for (int e = tid; e < ntouch; e += nt) {
                    int32_t k = tl[e];
                    tch[k] = 0;
                    refresh_means(st, mn, k, sc.F);
                }
                for (int e = tid; e < np; e += nt) {
                    fl[2 * (int64_t)J.props[3 * (int64_t)e + 1]] = 0;
                    fl[2 * (int64_t)J.props[3 * (int64_t)e + 2] + 1] = 0;
                }
                // every thread read np before the P2 barrier: safe to reset
                if (tid == 0) {
                    s_ctr[1] += (unsigned long long)np;
                    s_nprop = 0;
                }
                wg_sync();
                // ntouch was read after the P2 barrier; the next writer of
                // s_ntch (P2 of the next class) runs after the next barrier
                if (tid == 0) s_ntch = 0;
            }
            wg_sync();
            sweeps = t + 1;
            const int commits = s_commits;
            if (commits == 0) {
                converged = 1;
                break;
            }
            // next boundary set: eligible blocks within one block of a change
            const int nchg = s_nchg;
            wg_sync();
            if (tid < 9) s_cnt[tid] = 0;
            wg_sync();
            const int32_t stamp = t + 1;
            for (int64_t q0 = 0; q0 < 9 * (int64_t)nchg; q0 += nt) {
                int64_t q = q0 + tid;
                bool e = false;
                int cls = 0;
                int32_t ni = 0;
                if (q < 9 * (int64_t)nchg) {
                    int32_t bi = J.changed[q / 9];
                    int d = (int)(q % 9);
                    int bx = bi % nbx + (d % 3) - 1, by = bi / nbx + (d / 3) - 1;
                    if (bx >= 0 && by >= 0 && bx < nbx && by < nby) {
                        ni = by * nbx + bx;
                        if (atomicExch(&J.stamp[ni], stamp) != stamp) {
                            e = eligible(L, bx, by, nbx, nby, gate);
                            cls = 3 * (by % 3) + (bx % 3);
                        }
                    }
                }
                for (int c = 0; c < 9; c++) {
                    int slot = wave_append(&s_cnt[c], e && cls == c);
                    if (slot >= 0) J.lists[c * capc + slot] = ni;
                }
            }
            wg_sync();
            if (tid == 0) s_nchg = 0;
            wg_sync();
        }
        if (tid == 0) {
            rapid_stage_report r;
            r.level = sc.level[s];
            r.block = B;
            r.sweeps = sweeps;
            r.converged = converged;
            r.active = (int64_t)s_ctr[0];
            r.proposals = (int64_t)s_ctr[1];
            r.commits = (int64_t)s_ctr[2];
            r.skip_min = (int64_t)s_ctr[3];
            r.skip_topo = (int64_t)s_ctr[4];
            J.rep[s] = r;
            s_nchg = 0;
        }
        wg_sync();
    }
    if (LDS)
        for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) J.stats[i] = st[i];
    if ((flags & FLAG_OUT) && s_end > 0) {
        const int B = sc.B[s_end - 1];
        const int nbx = (W + B - 1) / B;
        const int32_t *L = J.lab[(s_end - 1) & 1];
        if (!(B == 1 && L == J.out)) {
            for (int64_t i = tid; i < (int64_t)W * H; i += nt) {
                int x = (int)(i % W), y = (int)(i / W);
                J.out[(int64_t)y * J.out_stride + x] = L[(int64_t)(y / B) * nbx + x / B];
            }
        }
    }
}

// ------------------------------------------------------------ launchers

hipError_t launch_block_sums(const Job *jobs_dev, int n_jobs, int s, int B, int64_t max_nb,
                             hipStream_t stream)
{
    int64_t blocks = (max_nb + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)blocks, (unsigned)n_jobs), dim3(256), 0, stream,
                       jobs_dev, s, B);
    return hipGetLastError();
}

hipError_t launch_expand(const int32_t *L, int W, int H, int B, int32_t *out, int64_t stride,
                         hipStream_t stream)
{
    int64_t N = (int64_t)W * H;
    int64_t blocks = (N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_expand, dim3((unsigned)blocks), dim3(256), 0, stream, L, W, H, B, out, stride);
    return hipGetLastError();
}

hipError_t launch_refine(const Job *jobs_dev, int n_jobs, const Sched &sc, int s_begin, int s_end,
                         int flags, const uint32_t *lut_dev, bool lds, size_t lds_bytes, int threads,
                         hipStream_t stream)
{
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void *)k_refine<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_refine<true>, dim3((unsigned)n_jobs), dim3(threads), lds_bytes, stream,
                           jobs_dev, sc, s_begin, s_end, flags, lut_dev);
    } else {
        hipLaunchKernelGGL(k_refine<false>, dim3((unsigned)n_jobs), dim3(threads), 0, stream,
                           jobs_dev, sc, s_begin, s_end, flags, lut_dev);
    }
    return hipGetLastError();
}

}  // namespace rapid
