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
//       P3 refresh means of the moved superpixels, clear the flow counters
//     rebuild the boundary set around changed blocks
#include "rapid_gate_dev.h"

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
    // the leader is wave-uniform: a scalar lane read, no LDS round trip
    base = __builtin_amdgcn_readlane(base, leader);
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

// Means record of a superpixel, 16 bytes (4 words):
//   c_r | c_g << 16,  c_b | (n & 0xFFFF) << 16,  mu_x | (n >> 16) << 17,  mu_y
// with the fixed-point means c <= 255 * 2^4 < 2^16 and mu_x <= 8191 * 2^4 <
// 2^17 (F <= 4, W, H <= 8192) and the size n <= 2^26.  Unpacked to
// lo = (c_r, c_g, c_b, mu_x) and hi = (mu_y, n).
__device__ __forceinline__ void unpack_mn(const uint4 &w, int4 &lo, int2 &hi)
{
    lo.x = (int)(w.x & 0xFFFFu);
    lo.y = (int)(w.x >> 16);
    lo.z = (int)(w.y & 0xFFFFu);
    lo.w = (int)(w.z & 0x1FFFFu);
    hi.x = (int)w.w;
    hi.y = (int)((w.y >> 16) | ((w.z >> 17) << 16));
}

__device__ __forceinline__ void load_mn(const int32_t *mn, int k, int4 &lo, int2 &hi)
{
    unpack_mn(reinterpret_cast<const uint4 *>(mn)[k], lo, hi);
}

// size n of superpixel k from its means record
__device__ __forceinline__ int64_t mn_size(const int32_t *mn, int k)
{
    const uint32_t *w = reinterpret_cast<const uint32_t *>(mn) + MN_STRIDE * (int64_t)k;
    return (int64_t)((w[1] >> 16) | ((w[2] >> 17) << 16));
}

// E'(beta, k) of the block with the means of k (record lo, hi) held fixed
// (Eq. (1) minus the terms that do not depend on k; difference form of
// Sec. 3.1).
__device__ __forceinline__ int64_t block_energy(const int4 &lo, const int2 &hi, const Geo &g,
                                                const int64_t I[3], int bnd, const Sched &sc)
{
    int64_t c0 = lo.x, c1 = lo.y, c2 = lo.z, mx = lo.w, my = hi.x;
    int64_t col = c0 * c0 + c1 * c1 + c2 * c2;
    int64_t dot = c0 * I[0] + c1 * I[1] + c2 * I[2];
    int64_t e_col = g.m * col - (dot << (sc.F + 1));
    int64_t pos = mx * mx + my * my;
    int64_t pdot = mx * g.px + my * g.py;
    int64_t e_pos = g.m * pos - (pdot << (sc.F + 1));
    return sc.w_col * e_col + sc.w_pos * e_pos + ((sc.w_bnd * (int64_t)bnd) << (2 * sc.F));
}

// The fixed-point means of a superpixel with exact integer sums r = (n,
// S_r, S_g, S_b, T_x, T_y): q[j] = floor((2^(F+1) S_j + n) / (2 n)) (rounded
// half up; colour then position).  The quotients use one reciprocal and an
// exact correction step (all products stay below 2^53).  A superpixel merged
// away (n = 0, sums 0) gets means 0.
__device__ __forceinline__ void fixed_means(const int64_t r[6], const Sched &sc, uint32_t q[5])
{
    const int64_t n = r[0];
    const double dd = (double)(2 * max(n, (int64_t)1)), dn0 = (double)n;
    const double rcp = 1.0 / dd;
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const double dn = fma((double)r[1 + j], sc.d_fs, dn0);   // 2^(F+1) S + n, exact
        double v = floor(dn * rcp);
        if (v * dd > dn) v -= 1.0;
        else if ((v + 1.0) * dd <= dn) v += 1.0;
        q[j] = (uint32_t)v;
    }
}

// Refresh superpixel k from its exact integer sums (st[k]): mn[k] holds its
// means in fixed point and its size n -- the class-start snapshot every
// proposal and every size-filter decision of the next class reads while the
// integer atomics of that class update the sums.
__device__ __forceinline__ void refresh_sp(const int64_t *st, int32_t *mn, int k, const Sched &sc)
{
    const int64_t *r = st + 6 * (int64_t)k;
    uint32_t q[5];
    fixed_means(r, sc, q);
    const uint32_t un = (uint32_t)r[0];
    reinterpret_cast<uint4 *>(mn)[k] =
        make_uint4(q[0] | (q[1] << 16), q[2] | ((un & 0xFFFFu) << 16), q[3] | ((un >> 16) << 17), q[4]);
}

// Packed statistics (residency 4): superpixel k's six sums in two 64-bit
// words, w0 = S_r | S_g << 21 | S_b << 42 and w1 = n | T_x << bn | T_y <<
// (bn + bx), with bn, bx from the host, which checked that every field
// stays non-negative and below its width between class phases (n below the
// larger of the maximum size and the largest initial cell).  The words are
// sums of the fields' place values, so signed deltas add exactly modulo
// 2^64 in any order, whatever the intermediate carries.
__device__ __forceinline__ void pk_add(unsigned long long *w, int64_t dn, int64_t dr, int64_t dg, int64_t db,
                                       int64_t dx, int64_t dy, const Sched &sc)
{
    const unsigned long long c =
        (unsigned long long)dr + ((unsigned long long)dg << 21) + ((unsigned long long)db << 42);
    const unsigned long long p = (unsigned long long)dn + ((unsigned long long)dx << sc.pk_bn) +
                                 ((unsigned long long)dy << (sc.pk_bn + sc.pk_bx));
    atomicAdd(w, c);
    atomicAdd(w + 1, p);
}

__device__ __forceinline__ void pk_unpack(const unsigned long long *w, int64_t r[6], const Sched &sc)
{
    const unsigned long long w0 = w[0], w1 = w[1];
    r[1] = (int64_t)(w0 & 0x1FFFFFull);
    r[2] = (int64_t)((w0 >> 21) & 0x1FFFFFull);
    r[3] = (int64_t)(w0 >> 42);
    r[0] = (int64_t)(w1 & ((1ull << sc.pk_bn) - 1));
    r[4] = (int64_t)((w1 >> sc.pk_bn) & ((1ull << sc.pk_bx) - 1));
    r[5] = (int64_t)(w1 >> (sc.pk_bn + sc.pk_bx));
}

__device__ __forceinline__ int64_t pk_size(const unsigned long long *pk, int k, const Sched &sc)
{
    return (int64_t)(pk[2 * (int64_t)k + 1] & ((1ull << sc.pk_bn) - 1));
}

// The means record (unpacked as load_mn gives it) of superpixel k from its
// packed statistics.
__device__ __forceinline__ void pk_means(const unsigned long long *pk, int k, const Sched &sc, int4 &lo, int2 &hi)
{
    int64_t r[6];
    pk_unpack(pk + 2 * (int64_t)k, r, sc);
    uint32_t q[5];
    fixed_means(r, sc, q);
    lo = make_int4((int)q[0], (int)q[1], (int)q[2], (int)q[3]);
    hi = make_int2((int)q[4], (int)r[0]);
}

__device__ __forceinline__ void pk_store(unsigned long long *pk, int k, const int64_t *r, const Sched &sc)
{
    pk[2 * (int64_t)k] = (unsigned long long)r[1] | ((unsigned long long)r[2] << 21) | ((unsigned long long)r[3] << 42);
    pk[2 * (int64_t)k + 1] = (unsigned long long)r[0] | ((unsigned long long)r[4] << sc.pk_bn) |
                             ((unsigned long long)r[5] << (sc.pk_bn + sc.pk_bx));
}

// E' in fp64 from a means record: m A - <c', I> - <mu', P> + w_bnd 2^(2F) bnd
// with A = w_col |c|^2 + w_pos |mu|^2, c' = w_col 2^(F+1) c and
// mu' = w_pos 2^(F+1) mu.  Used only where every product and partial sum is
// an integer below 2^53 (checked on the host per stage): then exact.
__device__ __forceinline__ double energy_f64(const int4 &lo, const int2 &hi, const Sched &sc, double m, double I0,
                                             double I1, double I2, double px, double py, double wbnd)
{
    const double q0 = lo.x, q1 = lo.y, q2 = lo.z, q3 = lo.w, q4 = hi.x;
    const double A = fma(sc.d_wc, fma(q0, q0, fma(q1, q1, q2 * q2)), sc.d_wp * fma(q3, q3, q4 * q4));
    const double lin =
        fma(sc.d_wcfs * q0, I0, fma(sc.d_wcfs * q1, I1, fma(sc.d_wcfs * q2, I2, fma(sc.d_wpfs * q3, px, (sc.d_wpfs * q4) * py))));
    return fma(m, A, -lin) + wbnd;
}

__device__ __forceinline__ int32_t lab_at(const int32_t *L, int bx, int by, int nbx, int nby)
{
    return (bx >= 0 && by >= 0 && bx < nbx && by < nby) ? L[by * nbx + bx] : -1;
}

// Gate modes of the refinement kernel (a template parameter, so that the
// plain kernel carries no gate code): no gate, gate bits from the caller,
// gate evaluated in place at the gate point (FLAG_GATE).
enum { GM_NONE = 0, GM_BITS = 1, GM_FUSED = 2 };

// The gate of a stage: the gate bits of all superpixels as an LDS bitmap
// (nullptr: no gate, every pair active) and the pair rule as a truth table
// indexed by 2 g_a + g_k.
struct GateView {
    const uint32_t *bits;
    uint32_t tt;
};

__device__ __forceinline__ uint32_t rule_table(int rule)
{
    // (g_a, g_k) = (0,0) (0,1) (1,0) (1,1) -> bits 0..3
    return rule == RAPID_GATE_BOTH ? 0x8u : rule == RAPID_GATE_DIFFER ? 0x6u : 0xEu;
}

// Eq. (7): may superpixels a and k exchange blocks under the gate?
__device__ __forceinline__ bool pair_on(const GateView &gv, int a, int k)
{
    if (gv.bits == nullptr) return true;
    const uint32_t ga = (gv.bits[a >> 5] >> (a & 31)) & 1u;
    const uint32_t gk = (gv.bits[k >> 5] >> (k & 31)) & 1u;
    return (gv.tt >> (2 * ga + gk)) & 1u;
}

__device__ __forceinline__ bool eligible(const int32_t *L, int bx, int by, int nbx, int nby,
                                         const GateView &gv)
{
    // the five labels are loaded together (one memory round trip, not one
    // per neighbour), then tested without short-circuiting
    const int32_t a = L[by * nbx + bx];
    const int32_t k0 = lab_at(L, bx - 1, by, nbx, nby), k1 = lab_at(L, bx + 1, by, nbx, nby);
    const int32_t k2 = lab_at(L, bx, by - 1, nbx, nby), k3 = lab_at(L, bx, by + 1, nbx, nby);
    const int e = (int)(k0 >= 0 && k0 != a && pair_on(gv, a, k0)) | (int)(k1 >= 0 && k1 != a && pair_on(gv, a, k1)) |
                  (int)(k2 >= 0 && k2 != a && pair_on(gv, a, k2)) | (int)(k3 >= 0 && k3 != a && pair_on(gv, a, k3));
    return e != 0;
}

// Inserts block index ni into the LDS hash set tab (mask + 1 words, keys
// stored as ni + 1, 0 = empty, linear probing).  True for the first
// insertion of ni.  The caller keeps the load at most one half, so a free
// word is always found.
__device__ __forceinline__ bool hash_insert(uint32_t *tab, int mask, int32_t ni)
{
    const uint32_t key = (uint32_t)ni + 1u;
    uint32_t h = ((uint32_t)ni * 2654435761u) & (uint32_t)mask;
    for (int probe = 0; probe <= mask; probe++) {
        const uint32_t old = atomicCAS(&tab[h], 0u, key);
        if (old == 0u) return true;
        if (old == key) return false;
        h = (h + 1u) & (uint32_t)mask;
    }
    return false;
}

__device__ __forceinline__ void wg_sync()
{
    __syncthreads();
}

// Passes of one workgroup over many elements (the pyramid, a stage split,
// the output, the gate point's band copy, a frontier rebuild) take several
// elements per lane and pass and issue all their loads before using any:
// one element per lane and pass would wait for one memory round trip per
// element.
constexpr int OUT_UNROLL = 4;     // output pixels (or band words) per lane and pass
constexpr int SPLIT_UNROLL = 4;   // parent blocks per lane and pass of a stage split
constexpr int SUMS_UNROLL = 2;    // 2x2 blocks per lane and pass of the pyramid's finest stage
constexpr int FRONT_UNROLL = 2;   // neighbourhood blocks per lane and pass of a frontier rebuild

// ------------------------------------------------------- block-sum pyramid
// Packed per-block RGB sums (21 bits per channel; B <= 64 keeps every
// channel below 2^21) of one stage of block size B straight from the
// pixels, by the whole workgroup; with MOMS also the pixel second moments
// per channel (at most 64^2 * 255^2 < 2^32) that the gate's features read.
template <bool SUMS, bool MOMS>
__device__ __forceinline__ void sums_from_pixels(const Job &J, int s, int B, int tid, int nt)
{
    const int nbx = (J.W + B - 1) / B, nby = (J.H + B - 1) / B;
    const int64_t nb = (int64_t)nbx * nby;
    if (B == 2) {
        // 2x2 blocks (the finest stage of the usual schedules): SUMS_UNROLL
        // blocks per lane and pass, the bytes of their (up to) four pixels
        // loaded together; pixels past the image edge count as zero
        for (int64_t i0 = tid; i0 < nb; i0 += SUMS_UNROLL * (int64_t)nt) {
            uint32_t v[SUMS_UNROLL][12];
#pragma unroll
            for (int u = 0; u < SUMS_UNROLL; u++) {
                const int64_t i = i0 + (int64_t)u * nt;
                const int bx = (int)((uint32_t)i % (uint32_t)nbx), by = (int)((uint32_t)i / (uint32_t)nbx);
                const bool in = i < nb, tx = in && 2 * bx + 1 < J.W, ty = in && 2 * by + 1 < J.H;
                const uint8_t *r0 = J.rgb + (int64_t)(2 * by) * J.rgb_stride + 6 * (int64_t)bx;
                const uint8_t *r1 = r0 + J.rgb_stride;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    v[u][c] = in ? r0[c] : 0u;
                    v[u][3 + c] = tx ? r0[3 + c] : 0u;
                    v[u][6 + c] = ty ? r1[c] : 0u;
                    v[u][9 + c] = tx && ty ? r1[3 + c] : 0u;
                }
            }
#pragma unroll
            for (int u = 0; u < SUMS_UNROLL; u++) {
                const int64_t i = i0 + (int64_t)u * nt;
                if (i >= nb) continue;
                uint32_t c3[3], q3[3];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    c3[c] = v[u][c] + v[u][3 + c] + v[u][6 + c] + v[u][9 + c];
                    q3[c] = v[u][c] * v[u][c] + v[u][3 + c] * v[u][3 + c] + v[u][6 + c] * v[u][6 + c] +
                            v[u][9 + c] * v[u][9 + c];
                }
                if (SUMS) J.sums[s][i] = (uint64_t)c3[0] | ((uint64_t)c3[1] << 21) | ((uint64_t)c3[2] << 42);
                if (MOMS) {
                    J.moms[3 * i] = q3[0];
                    J.moms[3 * i + 1] = q3[1];
                    J.moms[3 * i + 2] = q3[2];
                }
            }
        }
        return;
    }
    for (int64_t i = tid; i < nb; i += nt) {
        const int bx = (int)(i % nbx), by = (int)(i / nbx);
        const int x0 = bx * B, y0 = by * B;
        const int x1 = min(x0 + B, J.W), y1 = min(y0 + B, J.H);
        uint32_t r = 0, g = 0, b = 0, qr = 0, qg = 0, qb = 0;
        for (int y = y0; y < y1; y++) {
            const uint8_t *row = J.rgb + (int64_t)y * J.rgb_stride + 3 * (int64_t)x0;
            for (int x = 0; x < x1 - x0; x++) {
                const uint32_t pr = row[3 * x], pg = row[3 * x + 1], pb = row[3 * x + 2];
                r += pr;
                g += pg;
                b += pb;
                if (MOMS) {
                    qr += pr * pr;
                    qg += pg * pg;
                    qb += pb * pb;
                }
            }
        }
        if (SUMS) J.sums[s][i] = (uint64_t)r | ((uint64_t)g << 21) | ((uint64_t)b << 42);
        if (MOMS) {
            J.moms[3 * i] = qr;
            J.moms[3 * i + 1] = qg;
            J.moms[3 * i + 2] = qb;
        }
    }
}

// Block sums of stage s for every job by a separate launch (grid-stride
// over blockIdx.x, one job per blockIdx.y): used when the jobs are too few
// to fill the chip with the refinement kernel's workgroups.
__global__ void k_block_sums(const Job *__restrict__ jobs, int s, int B)
{
    const Job &J = jobs[blockIdx.y];
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    if (J.moms && s == J.moms_stage) sums_from_pixels<true, true>(J, s, B, tid, nt);
    else sums_from_pixels<true, false>(J, s, B, tid, nt);
}

// The pyramid of the schedule (Sec. 3.2's levels as exact box sums) for
// every stage with B >= 2: the finest such stage from the pixels, each
// coarser one as the sum of its children in the next finer stage (block
// sizes divide each other; packed fields add without carries).  Lanes tid
// of nt share the work; sync() separates the levels and ends the build (a
// workgroup barrier on one workgroup, a grid barrier on a cooperative
// launch, which returns false when the barrier gave up).
template <class Sync>
__device__ __forceinline__ bool build_pyramid(const Job &J, const Sched &sc, int tid, int nt, Sync sync)
{
    int sf = -1;
    for (int s = 0; s < sc.n_stages; s++)
        if (sc.B[s] >= 2) sf = s;
    if (sf >= 0) {
        if (J.moms && J.moms_stage == sf) sums_from_pixels<true, true>(J, sf, sc.B[sf], tid, nt);
        else sums_from_pixels<true, false>(J, sf, sc.B[sf], tid, nt);
        for (int s = sf - 1; s >= 0; s--) {
            if (!sync()) return false;
            const int B = sc.B[s], Bc = sc.B[s + 1], r = B / Bc;
            const int nbx = (J.W + B - 1) / B, nby = (J.H + B - 1) / B;
            const int nbxc = (J.W + Bc - 1) / Bc, nbyc = (J.H + Bc - 1) / Bc;
            const uint64_t *child = J.sums[s + 1];
            const int64_t nbs = (int64_t)nbx * nby;
            if (r == 2) {
                // SUMS_UNROLL parents per lane and pass, their four children
                // loaded together (a child past the edge counts as zero)
                for (int64_t i0 = tid; i0 < nbs; i0 += SUMS_UNROLL * (int64_t)nt) {
                    uint64_t c4[SUMS_UNROLL][4];
#pragma unroll
                    for (int u = 0; u < SUMS_UNROLL; u++) {
                        const int64_t i = i0 + (int64_t)u * nt;
                        const int bx = (int)((uint32_t)i % (uint32_t)nbx), by = (int)((uint32_t)i / (uint32_t)nbx);
                        const bool in = i < nbs, tx = in && 2 * bx + 1 < nbxc, ty = in && 2 * by + 1 < nbyc;
                        const uint64_t *c0 = child + (int64_t)(2 * by) * nbxc + 2 * bx;
                        c4[u][0] = in ? c0[0] : 0ull;
                        c4[u][1] = tx ? c0[1] : 0ull;
                        c4[u][2] = ty ? c0[nbxc] : 0ull;
                        c4[u][3] = tx && ty ? c0[nbxc + 1] : 0ull;
                    }
#pragma unroll
                    for (int u = 0; u < SUMS_UNROLL; u++) {
                        const int64_t i = i0 + (int64_t)u * nt;
                        if (i < nbs) J.sums[s][i] = c4[u][0] + c4[u][1] + c4[u][2] + c4[u][3];
                    }
                }
            } else {
                for (int64_t i = tid; i < nbs; i += nt) {
                    const int bx = (int)(i % nbx), by = (int)(i / nbx);
                    const int cx1 = min((bx + 1) * r, nbxc), cy1 = min((by + 1) * r, nbyc);
                    uint64_t acc = 0;
                    for (int cy = by * r; cy < cy1; cy++)
                        for (int cx = bx * r; cx < cx1; cx++) acc += child[(int64_t)cy * nbxc + cx];
                    J.sums[s][i] = acc;
                }
            }
        }
        if (J.moms && J.moms_stage >= 0 && J.moms_stage < sf)
            sums_from_pixels<false, true>(J, J.moms_stage, sc.B[J.moms_stage], tid, nt);
    }
    return sync();
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

// Work lists live in LDS up to a capacity and spill to the image's global
// scratch beyond it (same index space).
__device__ __forceinline__ int32_t list_get(const int32_t *lds, int cap, const int32_t *glob,
                                            int64_t gbase, int e)
{
    return e < cap ? lds[e] : glob[gbase + e];
}

__device__ __forceinline__ void list_put(int32_t *lds, int cap, int32_t *glob, int64_t gbase, int e,
                                         int32_t v)
{
    if (e < cap) lds[e] = v;
    else glob[gbase + e] = v;
}

__device__ __forceinline__ uint64_t pack_rgb(int64_t r, int64_t g, int64_t b)
{
    return (uint64_t)r | ((uint64_t)g << 21) | ((uint64_t)b << 42);
}

// Append v to the list of class cls (LDS atomic on the class counter; the
// hardware serialises lanes hitting the same counter, which is cheaper than
// nine rounds of wave-level aggregation).
__device__ __forceinline__ void class_push(int32_t *cnt, int32_t *lds, int capl, int32_t *glob,
                                           int64_t capg, int cls, int32_t v)
{
    int slot = atomicAdd(&cnt[cls], 1);
    list_put(lds + cls * capl, capl, glob, cls * capg, slot, v);
}

// ------------------------------------------------------ merge on underflow
// Sec. 3.1, Eqs. (4)-(5).  A superpixel asks to merge when one of its
// blocks cannot leave it without going below min_size (P1); the askers of a
// stage are a bit per label plus a list in order of asking.  When a sweep
// commits nothing, merge_pass settles them all at once.

__device__ __forceinline__ void merge_ask(const Job &J, int32_t a, int32_t *s_nreq)
{
    const uint32_t bit = 1u << (a & 31);
    if (!(atomicOr(&J.mreq[a >> 5], bit) & bit)) J.mlist[atomicAdd(s_nreq, 1)] = a;
}

// n |c|^2 - 2^(F+1) c S for one component: the part of the sum over a
// superpixel's pixels of (2^F v - c)^2 that depends on the mean c.
__device__ __forceinline__ __int128 fit_term(int64_t c, int64_t S, int64_t n, int F)
{
    return (__int128)n * c * c - ((__int128)2 << F) * c * S;
}

// Energy change of Eq. (1) when m is merged into k: colour and position
// terms re-fitted to the union's fixed-point means (rounded half up), and
// len shared boundary pixel pairs that stop being boundary.  Exact.
__device__ __forceinline__ __int128 merge_cost(const int64_t *st, const int32_t *mn, int m, int k, int64_t len, const Sched &sc)
{
    const int F = sc.F;
    const int64_t *rm = st + 6 * (int64_t)m, *rk = st + 6 * (int64_t)k;
    const int64_t nm = rm[0], nk = rk[0], nu = nm + nk;
    int4 lm, lk;
    int2 hm, hk;
    load_mn(mn, m, lm, hm);
    load_mn(mn, k, lk, hk);
    const int32_t cm[5] = {lm.x, lm.y, lm.z, lm.w, hm.x}, ck[5] = {lk.x, lk.y, lk.z, lk.w, hk.x};
    __int128 dc = 0, dp = 0;
#pragma unroll
    for (int j = 0; j < 5; j++) {
        const int64_t Su = rm[1 + j] + rk[1 + j];
        const int64_t cu = ((Su << (F + 1)) + nu) / (2 * nu);
        const __int128 d = fit_term(cu, Su, nu, F) - fit_term(cm[j], rm[1 + j], nm, F) -
                           fit_term(ck[j], rk[1 + j], nk, F);
        if (j < 3) dc += d;
        else dp += d;
    }
    return (__int128)sc.w_col * dc + (__int128)sc.w_pos * dp - (__int128)sc.w_bnd * ((__int128)len << (2 * F));
}

// One merge pass, by the whole workgroup; returns the number of merges.
// Askers still below min_size + B^2 pixels are candidates.  A candidate's
// blocks lie within n - 1 pixels of its centroid (a 4-connected set of n
// pixels), so its window of blocks is scanned for the labels 4-adjacent to
// it and their shared lengths (MERGE_NB slots per candidate filled with
// atomic compare-and-swap; a full set means no pick).  Each candidate picks
// the adjacent label of least merge_cost with an active pair and a merged
// size within max_size (ties to the smaller label); it leaves when its pick
// picked nothing or picked it back with a smaller label; per target the
// smallest leaving label merges.  Merges are then disjoint pairs: the sums
// move in parallel and the merged blocks go to the changed list.  mstate
// bits: 1 not a candidate, 2 slots full, 4 leaves, 8 merges.
__device__ __forceinline__ int merge_pass(const Job &J, int64_t *st, int32_t *mn, int32_t *L, int B,
                                                    int nbx, int nby, const Sched &sc, const GateView &gv,
                                                    int32_t *s_nreq, int32_t *s_nchg, int32_t *s_merged,
                                                    int32_t *l_chg, int capx, int tid, int nt)
{
    const int nreq = *s_nreq;
    // candidates, their windows, empty slots
    for (int r = tid; r < nreq; r += nt) {
        const int32_t m = J.mlist[r];
        const int64_t *rm = st + 6 * (int64_t)m;
        const int64_t n = rm[0];
        bool cand = n > 0 && n < sc.min_size + (int64_t)B * B;
        for (int j = 0; j < MERGE_NB; j++) {
            J.mkey[MERGE_NB * r + j] = -1;
            J.mlen[MERGE_NB * r + j] = 0;
        }
        if (cand) {
            const int64_t x0 = max((int64_t)0, rm[4] / n - (n - 1));
            const int64_t x1 = min((int64_t)J.W - 1, (rm[4] + n - 1) / n + (n - 1));
            const int64_t y0 = max((int64_t)0, rm[5] / n - (n - 1));
            const int64_t y1 = min((int64_t)J.H - 1, (rm[5] + n - 1) / n + (n - 1));
            // sums consistent with the labels always give a non-empty window
            cand = x0 <= x1 && y0 <= y1;
            J.mbox[r] = make_int4((int)(x0 / B), (int)(y0 / B), (int)(x1 / B), (int)(y1 / B));
        }
        J.mstate[r] = cand ? 0 : 1;
    }
    if (tid == 0) *s_merged = 0;
    wg_sync();
    // shared boundary lengths with the adjacent labels
    for (int r = 0; r < nreq; r++) {
        if (J.mstate[r] != 0) continue;   // uniform
        const int32_t m = J.mlist[r];
        const int4 bb = J.mbox[r];
        const int ww = bb.z - bb.x + 1;
        const int64_t cnt = (int64_t)ww * (bb.w - bb.y + 1);
        int32_t *keys = J.mkey + MERGE_NB * r;
        int32_t *lens = J.mlen + MERGE_NB * r;
        for (int64_t i = tid; i < cnt; i += nt) {
            const int bx = bb.x + (int)(i % ww), by = bb.y + (int)(i / ww);
            const int64_t bi = (int64_t)by * nbx + bx;
            if (L[bi] != m) continue;
            const Geo g = block_geo(bx, by, B, J.W, J.H);
            const int32_t nl[4] = {bx > 0 ? L[bi - 1] : -1, bx + 1 < nbx ? L[bi + 1] : -1,
                                   by > 0 ? L[bi - nbx] : -1, by + 1 < nby ? L[bi + nbx] : -1};
            const int el[4] = {g.h, g.h, g.w, g.w};
            for (int d = 0; d < 4; d++) {
                const int32_t k = nl[d];
                if (k < 0 || k == m) continue;
                int j = 0;
                for (; j < MERGE_NB; j++) {
                    const int32_t old = atomicCAS(&keys[j], -1, k);
                    if (old == -1 || old == k) {
                        atomicAdd(&lens[j], el[d]);
                        break;
                    }
                }
                if (j == MERGE_NB) atomicOr(&J.mstate[r], 2);
            }
        }
    }
    wg_sync();
    // picks (Eq. (4) under the size bound of Eq. (5))
    for (int r = tid; r < nreq; r += nt) {
        if (J.mstate[r] != 0) continue;
        const int32_t m = J.mlist[r];
        const int64_t nm = st[6 * (int64_t)m];
        int32_t best = -1;
        __int128 bc = 0;
        for (int j = 0; j < MERGE_NB; j++) {
            const int32_t k = J.mkey[MERGE_NB * r + j];
            if (k < 0) break;
            if (nm + st[6 * (int64_t)k] > sc.max_size || !pair_on(gv, m, k)) continue;
            const __int128 c = merge_cost(st, mn, m, k, J.mlen[MERGE_NB * r + j], sc);
            if (best < 0 || c < bc || (c == bc && k < best)) {
                best = k;
                bc = c;
            }
        }
        J.mpick[m] = best;
    }
    wg_sync();
    // who leaves, and the smallest leaving label per target
    for (int r = tid; r < nreq; r += nt) {
        const int32_t m = J.mlist[r];
        const int32_t t = J.mstate[r] == 0 ? J.mpick[m] : -1;
        if (t < 0) continue;
        const int32_t tt = J.mpick[t];
        if (tt < 0 || (tt == m && m > t)) {
            atomicMin(&J.mwin[t], m);
            J.mstate[r] = 4;
        }
    }
    wg_sync();
    // merges: each target absorbs one superpixel and none leaves, so the
    // rows touched here are distinct
    for (int r = tid; r < nreq; r += nt) {
        if (J.mstate[r] != 4) continue;
        const int32_t m = J.mlist[r], t = J.mpick[m];
        if (J.mwin[t] != m) continue;
        J.mstate[r] = 8;
        int64_t *rt = st + 6 * (int64_t)t, *rm = st + 6 * (int64_t)m;
        for (int j = 0; j < 6; j++) {
            rt[j] += rm[j];
            rm[j] = 0;
        }
        refresh_sp(st, mn, t, sc);
        refresh_sp(st, mn, m, sc);
        atomicAdd(s_merged, 1);
    }
    wg_sync();
    // relabel the merged blocks; they seed the next sweep
    for (int r = 0; r < nreq; r++) {
        if (J.mstate[r] != 8) continue;   // uniform
        const int32_t m = J.mlist[r], t = J.mpick[m];
        const int4 bb = J.mbox[r];
        const int ww = bb.z - bb.x + 1;
        const int64_t cnt = (int64_t)ww * (bb.w - bb.y + 1);
        for (int64_t i0 = 0; i0 < cnt; i0 += nt) {
            const int64_t i = i0 + tid;
            bool hit = false;
            int32_t bi = 0;
            if (i < cnt) {
                bi = (bb.y + (int)(i / ww)) * nbx + bb.x + (int)(i % ww);
                hit = L[bi] == m;
                if (hit) L[bi] = t;
            }
            const int slot = wave_append(s_nchg, hit);
            if (slot >= 0) list_put(l_chg, capx, J.changed, 0, slot, bi);
        }
    }
    wg_sync();
    // clear the askers and the per-label pick state
    for (int r = tid; r < nreq; r += nt) {
        const int32_t m = J.mlist[r];
        atomicAnd(&J.mreq[m >> 5], ~(1u << (m & 31)));
        const int32_t t = J.mpick[m];
        if (t >= 0) J.mwin[t] = INT32_MAX;
    }
    wg_sync();
    for (int r = tid; r < nreq; r += nt) J.mpick[J.mlist[r]] = -1;
    const int merged = *s_merged;
    wg_sync();
    if (tid == 0) *s_nreq = 0;
    wg_sync();
    return merged;
}

// Accumulators of one superpixel in the LDS window of the gate point.
struct WinAcc {
    unsigned long long q[3], ed2, nbs;
    unsigned bl, mx, mn, pad;
};

// Runs of superpixels whose initial grid row lies in [ky0, ky0 + rows) go
// to the LDS window (LDS atomics), any other run straight to global memory.
struct WindowSink {
    WinAcc *win;
    int64_t *facc;
    int gx, ky0, rows;
    __device__ void operator()(int32_t k, const FeatAcc &v) const
    {
        const int r = k / gx - ky0;
        if (r < 0 || r >= rows) {
            feat_flush(facc, k, v);
            return;
        }
        WinAcc &w = win[r * gx + k % gx];
        atomicAdd(&w.q[0], (unsigned long long)v.q[0]);
        atomicAdd(&w.q[1], (unsigned long long)v.q[1]);
        atomicAdd(&w.q[2], (unsigned long long)v.q[2]);
        if (v.bl) {
            atomicAdd(&w.bl, (unsigned)v.bl);
            atomicAdd(&w.ed2, (unsigned long long)v.ed2);
            atomicAdd(&w.nbs, (unsigned long long)v.nbs);
            atomicMax(&w.mx, (unsigned)v.mx);
            atomicMin(&w.mn, (unsigned)v.mn);
        }
    }
};

// The gate point of a fused launch (Algorithm RAPID, before the gated
// level), run by the whole workgroup: features of every superpixel on the
// labels of the previous stage (block size Bq), the network's logit and the
// gate bits (Eq. (6)).  Only the fused-gate instantiation of the kernel
// contains it, so the plain kernel's registers are not affected.
//
// The work lists' LDS (lds, lds_bytes) is free here.  It holds the
// fixed-point means of all superpixels, then bands of RB block rows of the
// label map (with a halo row above and below) loaded with coalesced bulk
// reads, which the lanes walk in segments, and a window of accumulators for
// the superpixels whose initial grid rows meet the band: runs add to the
// window with LDS atomics, the window goes to global memory once per band.
// A band of a few cells' height touches few grid rows, so this replaces
// most global atomics (which contend on the same lines) with LDS ones.  The
// squared mean distances fit 32 bits (F <= 4).  Falls back to the label
// map in global memory when the LDS is too small.
__device__ __attribute__((noinline)) void gate_point(const Job &J, const int64_t *st, int stage_q, int Bq, int F,
                                                     int fset, const uint16_t *mlp_w, float thresh, char *lds,
                                                     uint32_t lds_bytes, int tid, int nt)
{
    const int K = J.K;
    const int nbxq = (J.W + Bq - 1) / Bq, nbyq = (J.H + Bq - 1) / Bq;
    const int32_t *Lq = J.lab[stage_q & 1];
    const uint32_t *moms = (J.moms && J.moms_stage == stage_q) ? J.moms : nullptr;
    const int spr = (nbxq + FEAT_SEG - 1) / FEAT_SEG;
    // LDS carve-up: means, window, band
    const int64_t fm_bytes = (12 * (int64_t)K + 15) & ~15ll;
    // a band of about one cell height (at least one block row)
    const int cell_rows = max(1, (int)(((int64_t)J.H / J.gy) / Bq));
    int RB = min(cell_rows, nbyq);
    int WR = 0;
    int64_t win_bytes = 0, band_bytes = 0;
    bool staged = false;
    for (; RB >= 1; RB >>= 1) {
        // grid rows met by RB block rows: the rows of their pixel span, one
        // more for the block-centre rule's rounding, two for drift
        WR = min(J.gy, (int)(((int64_t)RB * Bq * J.gy + J.H - 1) / J.H) + 3);
        win_bytes = (int64_t)WR * J.gx * (int64_t)sizeof(WinAcc);
        band_bytes = 4 * (int64_t)(RB + 2) * nbxq;
        if (fm_bytes + win_bytes + band_bytes <= (int64_t)lds_bytes) {
            staged = true;
            break;
        }
    }
    int32_t *fm_l = reinterpret_cast<int32_t *>(lds);
    WinAcc *win = reinterpret_cast<WinAcc *>(lds + fm_bytes);
    int32_t *band = reinterpret_cast<int32_t *>(lds + fm_bytes + win_bytes);
    for (int k = tid; k < K; k += nt) {
        feat_init_sp(st, J.fmean, J.facc, k, F);
        if (staged)
            for (int ch = 0; ch < 3; ch++) fm_l[3 * k + ch] = J.fmean[3 * k + ch];
    }
    if (staged) {
        for (int e = tid; e < WR * J.gx; e += nt) {
            WinAcc &w = win[e];
            w.q[0] = w.q[1] = w.q[2] = w.ed2 = w.nbs = 0;
            w.bl = w.mx = 0;
            w.mn = 0xFFFFFFFFu;
        }
    }
    wg_sync();
    if (staged) {
        for (int by0 = 0; by0 < nbyq; by0 += RB) {
            const int rows = min(RB, nbyq - by0);
            // rows by0 - 1 .. by0 + rows of the label map, -1 outside it:
            // one contiguous range of the map, copied in one pass with
            // OUT_UNROLL loads per lane in flight
            const int64_t nband = (int64_t)(rows + 2) * nbxq, gbase = (int64_t)(by0 - 1) * nbxq;
            const int64_t nbq = (int64_t)nbxq * nbyq;
            for (int64_t e0 = tid; e0 < nband; e0 += OUT_UNROLL * (int64_t)nt) {
                int32_t v[OUT_UNROLL];
#pragma unroll
                for (int u = 0; u < OUT_UNROLL; u++) {
                    const int64_t e = e0 + (int64_t)u * nt, gi = gbase + e;
                    v[u] = (e < nband && gi >= 0 && gi < nbq) ? Lq[gi] : -1;
                }
#pragma unroll
                for (int u = 0; u < OUT_UNROLL; u++) {
                    const int64_t e = e0 + (int64_t)u * nt;
                    if (e < nband) band[e] = v[u];
                }
            }
            // grid rows of the band's first pixel row, minus one
            const int ky0 = (int)(((int64_t)by0 * Bq * J.gy) / J.H) - 1;
            WindowSink sink{win, J.facc, J.gx, ky0, WR};
            wg_sync();
            for (int g = tid; g < rows * spr; g += nt) {
                const int r = g / spr, bx0 = (g - r * spr) * FEAT_SEG;
                const int32_t *row = band + (r + 1) * nbxq;
                feat_segment(J, row, row - nbxq, row + nbxq, Bq, nbxq, by0 + r, bx0, min(bx0 + FEAT_SEG, nbxq), moms,
                             fm_l, sink);
            }
            wg_sync();
            // the window to global memory, then cleared for the next band
            for (int e = tid; e < WR * J.gx; e += nt) {
                WinAcc &w = win[e];
                const int k = (ky0 + e / J.gx) * J.gx + e % J.gx;
                if (w.q[0] | w.q[1] | w.q[2] | w.bl) {
                    FeatAcc v;
                    v.q[0] = (int64_t)w.q[0];
                    v.q[1] = (int64_t)w.q[1];
                    v.q[2] = (int64_t)w.q[2];
                    v.bl = w.bl;
                    v.ed2 = (int64_t)w.ed2;
                    v.nbs = (int64_t)w.nbs;
                    v.mx = w.mx;
                    v.mn = w.mn;
                    feat_flush(J.facc, k, v);
                    w.q[0] = w.q[1] = w.q[2] = w.ed2 = w.nbs = 0;
                    w.bl = w.mx = 0;
                    w.mn = 0xFFFFFFFFu;
                }
            }
            wg_sync();
        }
    } else {
        for (int64_t g = tid; g < (int64_t)spr * nbyq; g += nt) {
            const int by = (int)(g / spr), bx0 = (int)(g % spr) * FEAT_SEG;
            const int32_t *row = Lq + (int64_t)by * nbxq;
            feat_segment(J, row, by > 0 ? row - nbxq : nullptr, by + 1 < nbyq ? row + nbxq : nullptr, Bq, nbxq, by,
                         bx0, min(bx0 + FEAT_SEG, nbxq), moms, J.fmean, GlobalSink{J.facc});
        }
        wg_sync();
    }
    for (int k = tid; k < K; k += nt) feat_final_sp(J, st, J.facc, J.moved, k, F, fset, J.xrow + 16 * (int64_t)k);
    wg_sync();
    const int lane = tid & 63;
    for (int t = tid >> 6; t < (K + 15) / 16; t += nt >> 6) {
        const int n = 16 * t + (lane & 15);
        const float z = mlp_logit(mlp_w, load_x(J.xrow, n, K, lane >> 4), lane);
        if (lane < 16 && n < K) J.gate_out[n] = z >= thresh ? 1 : 0;
    }
    wg_sync();
}

// P1 for one active block bi of the current class (the cooperative
// kernel's; k_refine writes the same steps out in place): the source keeps
// its minimum size (Sec. 3.1), the block is a simple point of its label
// (the topology rule, 3x3 window), then the strict argmin of E' over the
// source and its distinct 4-neighbour labels that stay within the maximum
// size (Eq. (3); ties keep the source or the smaller label).  Reads the
// class-start state only.
template <bool PK>
__device__ __forceinline__ void propose_block(const Job &J, int s, int B, int32_t bi, int nbx, int nby, int W,
                                              int H, const int32_t *L, const int32_t *mn, const uint32_t *s_lut,
                                              const Sched &sc, const GateView &gv, bool use_f64, int32_t &a,
                                              int32_t &best, int64_t &m, uint64_t &Ipk, bool &prop, bool &smin,
                                              bool &stopo, int64_t &na, int64_t &nk)
{
    // PK: mn holds the packed statistics (two words per superpixel) and the
    // means are computed from them
    const unsigned long long *pk = reinterpret_cast<const unsigned long long *>(mn);
    const int bx = bi % nbx, by = bi / nbx;
    const bool hw = bx > 0, he = bx + 1 < nbx, hn = by > 0, hs = by + 1 < nby;
    // every global load of the block at once: its label,
    // its 3x3 ring and its colour sum
    const int32_t *Lc = L + bi;
    a = Lc[0];
    int32_t rl[8];
    rl[0] = (hn && hw) ? Lc[-nbx - 1] : -1;
    rl[1] = hn ? Lc[-nbx] : -1;
    rl[2] = (hn && he) ? Lc[-nbx + 1] : -1;
    rl[3] = hw ? Lc[-1] : -1;
    rl[4] = he ? Lc[1] : -1;
    rl[5] = (hs && hw) ? Lc[nbx - 1] : -1;
    rl[6] = hs ? Lc[nbx] : -1;
    rl[7] = (hs && he) ? Lc[nbx + 1] : -1;
    int64_t I[3];
    block_rgb(J, s, B, bi, bx, by, I);
    Ipk = pack_rgb(I[0], I[1], I[2]);
    Geo g = block_geo(bx, by, B, W, H);
    m = g.m;
    int4 ra;
    int2 rb;
    if (PK) pk_means(pk, a, sc, ra, rb);
    else load_mn(mn, a, ra, rb);
    na = rb.y;
    nk = 0;
    if ((int64_t)rb.y - g.m < sc.min_size) {
        smin = true;
    } else {
        uint32_t mask = 0;
#pragma unroll
        for (int q = 0; q < 8; q++) mask |= (rl[q] == a ? 1u : 0u) << q;
        if (!((s_lut[mask >> 5] >> (mask & 31)) & 1u)) {
            stopo = true;
        } else {
            // 4-neighbours W, E, N, S and their shared edge lengths
            const int32_t nl[4] = {rl[3], rl[4], rl[1], rl[6]};
            const int el[4] = {g.h, g.h, g.w, g.w};
            // candidate labels: distinct, != a, ascending
            // (sorting network; excluded values sink as INT_MAX)
            int32_t q0 = (nl[0] < 0 || nl[0] == a) ? INT32_MAX : nl[0];
            int32_t q1 = (nl[1] < 0 || nl[1] == a) ? INT32_MAX : nl[1];
            int32_t q2 = (nl[2] < 0 || nl[2] == a) ? INT32_MAX : nl[2];
            int32_t q3 = (nl[3] < 0 || nl[3] == a) ? INT32_MAX : nl[3];
            int32_t t0 = min(q0, q1), t1 = max(q0, q1), t2 = min(q2, q3), t3 = max(q2, q3);
            int32_t s0 = min(t0, t2), s2 = max(t0, t2), s1 = min(t1, t3), s3 = max(t1, t3);
            int32_t u1 = min(s1, s2), u2 = max(s1, s2);
            const int32_t cs[4] = {s0, u1, u2, s3};
            int bnd_a = 0;
#pragma unroll
            for (int d = 0; d < 4; d++) bnd_a += (nl[d] >= 0 && nl[d] != a) ? el[d] : 0;
            best = a;
            if (use_f64) {
                const double dm = (double)g.m, dI0 = (double)I[0], dI1 = (double)I[1],
                             dI2 = (double)I[2], dpx = (double)g.px, dpy = (double)g.py;
                double estar = energy_f64(ra, rb, sc, dm, dI0, dI1, dI2, dpx, dpy, sc.d_wb * (double)bnd_a);
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t k = cs[u];
                    if (k == INT32_MAX || (u > 0 && k == cs[u - 1])) continue;
                    int4 ka;
                    int2 kb;
                    if (PK) pk_means(pk, k, sc, ka, kb);
                    else load_mn(mn, k, ka, kb);
                    if ((int64_t)kb.y + g.m > sc.max_size) continue;
                    int bnd = 0;
#pragma unroll
                    for (int d = 0; d < 4; d++) bnd += (nl[d] >= 0 && nl[d] != k) ? el[d] : 0;
                    double ek = energy_f64(ka, kb, sc, dm, dI0, dI1, dI2, dpx, dpy, sc.d_wb * (double)bnd);
                    if (ek < estar) {
                        estar = ek;
                        best = k;
                        nk = kb.y;
                    }
                }
            } else {
                int64_t estar = block_energy(ra, rb, g, I, bnd_a, sc);
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int32_t k = cs[u];
                    if (k == INT32_MAX || (u > 0 && k == cs[u - 1])) continue;
                    int4 ka;
                    int2 kb;
                    if (PK) pk_means(pk, k, sc, ka, kb);
                    else load_mn(mn, k, ka, kb);
                    if ((int64_t)kb.y + g.m > sc.max_size) continue;
                    int bnd = 0;
#pragma unroll
                    for (int d = 0; d < 4; d++) bnd += (nl[d] >= 0 && nl[d] != k) ? el[d] : 0;
                    int64_t ek = block_energy(ka, kb, g, I, bnd, sc);
                    if (ek < estar) {
                        estar = ek;
                        best = k;
                        nk = kb.y;
                    }
                }
            }
            prop = best != a && pair_on(gv, a, best);
        }
    }
}

// SL: where the per-superpixel state lives -- 0 all in global memory, 1
// statistics, means records and flow counters in LDS, 2 the means records
// in LDS (the hot reads of P1) and the rest in global memory, 3 the means
// records and the flow counters in LDS, the statistics in global memory.
template <int SL, int GM, bool MERGE>
__device__ __forceinline__ void refine_job(const Job &J, const Sched &sc, const LdsPlan &lp, int s_begin, int s_end,
                                           int flags, const uint32_t *__restrict__ lut_g)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_lut[8];
    __shared__ int32_t s_cnt[9];
    // proposal counters of the class phases, used by turns: a class with no
    // proposal goes on to the next class's P1 without another barrier, so
    // that phase appends to the other counter while slower waves may still
    // read this one
    __shared__ int32_t s_nprop[2];
    __shared__ int32_t s_nchg, s_nreq, s_merged, s_any;
    __shared__ unsigned long long s_ctr[6];   // active proposals commits skip_min skip_topo merges

    const int tid = threadIdx.x, nt = blockDim.x;
    const int W = J.W, H = J.H, K = J.K;
    int64_t *st;
    int32_t *mn, *fl;
    unsigned long long *pk = nullptr;   // residency 4: packed statistics in LDS
    if (SL == 1) {
        st = reinterpret_cast<int64_t *>(smem);
        mn = reinterpret_cast<int32_t *>(st + 6 * (int64_t)K);   // K records of 16 bytes, 16-byte aligned
        fl = mn + MN_STRIDE * (int64_t)K;
    } else if (SL == 4) {
        // the sums in two words per superpixel, then the flow counters; no
        // means records: the means are computed where they are read
        st = J.stats;
        mn = nullptr;
        pk = reinterpret_cast<unsigned long long *>(smem);
        fl = reinterpret_cast<int32_t *>(pk + 2 * (int64_t)K);
    } else if (SL == 2 || SL == 3) {
        st = J.stats;
        mn = reinterpret_cast<int32_t *>(smem);
        fl = SL == 3 ? mn + MN_STRIDE * (int64_t)K : J.flow;
    } else {
        st = J.stats;
        mn = J.means;
        fl = J.flow;
    }
    int32_t *l_lists = reinterpret_cast<int32_t *>(smem + lp.off_lists);
    Prop *l_props = reinterpret_cast<Prop *>(smem + lp.off_props);
    int32_t *l_chg = reinterpret_cast<int32_t *>(smem + lp.off_chg);
    uint32_t *l_bm = reinterpret_cast<uint32_t *>(smem + lp.off_bm);
    // the bitmap's words as an open-addressing hash set: a power of two
    int ht_cap = 0;
    if (lp.bm_words >= 64) {
        ht_cap = 64;
        while (2 * ht_cap <= lp.bm_words) ht_cap *= 2;
    }
    uint32_t *l_gate = reinterpret_cast<uint32_t *>(smem + lp.off_gate);
    bool gate_loaded = false;
    Prop *g_props = J.props;
    const int capl = lp.capl, capp = lp.capp, capx = lp.capx;
    const int64_t capg = J.capc;

    if (tid < 8) s_lut[tid] = lut_g[tid];
    if (tid == 0) {
        s_nprop[0] = s_nprop[1] = 0;
        s_nchg = 0;
        s_nreq = 0;
    }
    for (int64_t i = tid; i < 2 * (int64_t)K; i += nt) fl[i] = 0;
    if (MERGE) {
        for (int64_t i = tid; i < K; i += nt) {
            J.mpick[i] = -1;
            J.mwin[i] = INT32_MAX;
        }
        for (int i = tid; i < (K + 31) / 32; i += nt) J.mreq[i] = 0;
    }
    if (s_end > s_begin) {
        // visit stamps are unique per (stage, sweep) of this launch: cleared
        // once, for the largest stage whose blocks the LDS bitmap cannot cover
        const int Bf = sc.B[s_end - 1];
        const int64_t nbf = (int64_t)((W + Bf - 1) / Bf) * ((H + Bf - 1) / Bf);
        if ((int64_t)lp.bm_words * 32 < nbf)
            for (int64_t i = tid; i < nbf; i += nt) J.stamp[i] = 0;
    }
    if (GM == GM_FUSED)
        for (int64_t i = tid; i < K; i += nt) J.moved[i] = 0;
    for (int i = tid; i < lp.bm_words; i += nt) l_bm[i] = 0;

    if (flags & FLAG_INIT) {
        // the block-sum pyramid, grid initialisation (Algorithm RAPID,
        // first step) and the statistics, computed once for all levels
        // (Sec. 3.2)
        if (SL == 4)
            for (int64_t i = tid; i < 2 * (int64_t)K; i += nt) pk[i] = 0;
        else
            for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) st[i] = 0;
        if (flags & FLAG_PYRAMID)
            build_pyramid(J, sc, tid, nt, []() {
                __syncthreads();
                return true;
            });
        else wg_sync();
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
            if (SL == 4) {
                pk_add(pk + 2 * (int64_t)k, g.m, I[0], I[1], I[2], g.px, g.py, sc);
            } else {
                int64_t *r = st + 6 * (int64_t)k;
                add64(r + 0, g.m);
                add64(r + 1, I[0]);
                add64(r + 2, I[1]);
                add64(r + 3, I[2]);
                add64(r + 4, g.px);
                add64(r + 5, g.py);
            }
        }
    } else if (SL == 1) {
        for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) st[i] = J.stats[i];
    } else if (SL == 4) {
        for (int k = tid; k < K; k += nt) pk_store(pk, k, J.stats + 6 * (int64_t)k, sc);
    }
    wg_sync();
    if (SL != 4)
        for (int k = tid; k < K; k += nt) refresh_sp(st, mn, k, sc);
    wg_sync();

    int out_stage = s_end - 1;   // stage whose label map the output reads
    for (int s = s_begin; s < s_end; s++) {
        const int B = sc.B[s];
        const int nbx = (W + B - 1) / B, nby = (H + B - 1) / B;
        const int64_t nb = (int64_t)nbx * nby;
        int32_t *L = J.lab[s & 1];
        if (GM == GM_FUSED && s == sc.gate_stage && s > 0) {
            // The gate point may use all the LDS that holds no statistics:
            // the work lists, the gate words (loaded only afterwards) and,
            // when only the means records live in LDS, their region too (it
            // keeps its own means; the records are rebuilt afterwards).  A
            // larger band of the label map per pass means fewer passes.
            const uint32_t gp_off = SL == 1 ? lp.off_lists : 0u;
            if (SL == 4) {
                // the features read the sums from global memory; the gate
                // point then borrows their LDS, and they come back after it
                for (int k = tid; k < K; k += nt) {
                    int64_t r[6];
                    pk_unpack(pk + 2 * (int64_t)k, r, sc);
                    for (int q = 0; q < 6; q++) J.stats[6 * (int64_t)k + q] = r[q];
                }
                wg_sync();
            }
            gate_point(J, st, s - 1, sc.B[s - 1], sc.F, sc.feat_set, sc.mlp_w, sc.mlp_thresh, smem + gp_off,
                       lp.total - gp_off, tid, nt);
            if (SL == 2 || SL == 3)
                for (int k = tid; k < K; k += nt) refresh_sp(st, mn, k, sc);
            if (SL == 4)
                for (int k = tid; k < K; k += nt) pk_store(pk, k, J.stats + 6 * (int64_t)k, sc);
            if (SL == 3 || SL == 4)   // the flow counters are zero between class phases
                for (int64_t i = tid; i < 2 * (int64_t)K; i += nt) fl[i] = 0;
            // the frontier bitmap shares that LDS and must start the stage clear
            for (int i = tid; i < lp.bm_words; i += nt) l_bm[i] = 0;
        }
        // moved pixels feed the gate's features: past the gate point of a
        // fused launch nothing needs them
        int64_t *const mv = (GM == GM_FUSED && s >= sc.gate_stage) ? nullptr : J.moved;
        GateView gv;
        gv.bits = nullptr;
        gv.tt = rule_table(sc.gate_rule);
        if (GM != GM_NONE && J.gate && s >= sc.gate_stage) {
            if (!gate_loaded) {
                // first gated stage of the launch: the gate bits into LDS
                // (the host guarantees 32 * gate_words >= K)
                for (int w = tid; w < (K + 31) / 32; w += nt) {
                    uint32_t v = 0;
                    for (int b = 0; b < 32 && 32 * w + b < K; b++) v |= (J.gate[32 * w + b] != 0 ? 1u : 0u) << b;
                    l_gate[w] = v;
                }
                gate_loaded = true;   // uniform: the workgroup syncs below before any use
            }
            gv.bits = l_gate;
        }
        const bool use_bm = (int64_t)lp.bm_words * 32 >= nb;
        const bool use_f64 = sc.f64[s] != 0;
        if (tid < 9) s_cnt[tid] = 0;
        if (tid < 6) s_ctr[tid] = 0;
        if (tid == 0) s_any = 0;
        wg_sync();
        if (GM != GM_NONE && (flags & FLAG_OUT) && s == s_end - 1 && s > 0 && gv.bits != nullptr) {
            // The last stage of a launch under the gate: when no two adjacent
            // parent blocks form an active pair, no block of the stage is a
            // boundary element, so its one sweep finds nothing.  The stage
            // then writes only its report and the output comes from the
            // parent map, which spares materialising the finest map.  (The
            // pair rules are symmetric: east and south neighbours cover
            // every edge.)
            const int Bp = sc.B[s - 1];
            const int nbxp = (W + Bp - 1) / Bp, nbyp = (H + Bp - 1) / Bp;
            const int32_t *Lp = J.lab[(s - 1) & 1];
            // four parents per lane and pass, their loads issued together
            const int64_t npar = (int64_t)nbxp * nbyp;
            bool any = false;
            for (int64_t p0 = tid; p0 < npar && !any; p0 += 4 * (int64_t)nt) {
                int32_t a[4], e[4], d[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int64_t p = p0 + u * (int64_t)nt;
                    const int pxb = (int)(p % nbxp), pyb = (int)(p / nbxp);
                    const bool in = p < npar;
                    a[u] = in ? Lp[p] : -1;
                    e[u] = in && pxb + 1 < nbxp ? Lp[p + 1] : -1;
                    d[u] = in && pyb + 1 < nbyp ? Lp[p + nbxp] : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    any = any || (e[u] >= 0 && e[u] != a[u] && pair_on(gv, a[u], e[u]));
                    any = any || (d[u] >= 0 && d[u] != a[u] && pair_on(gv, a[u], d[u]));
                }
            }
            if (any) s_any = 1;
            wg_sync();
            if (s_any == 0) {   // uniform
                if (tid == 0) {
                    rapid_stage_report r;
                    r.level = sc.level[s];
                    r.block = B;
                    r.sweeps = 1;
                    r.converged = 1;
                    r.active = r.proposals = r.commits = r.skip_min = r.skip_topo = r.merges = 0;
                    J.rep[s] = r;
                }
                out_stage = s - 1;
                wg_sync();
                continue;
            }
        }
        if (s > 0) {
            // split: each block inherits the label of the block that holds it.
            // A child is a boundary block only on a side where its parent
            // borders a parent of another (active) label, so the boundary
            // scan runs over the parents.
            const int Bp = sc.B[s - 1];
            const int nbxp = (W + Bp - 1) / Bp, nbyp = (H + Bp - 1) / Bp;
            const int64_t nbp = (int64_t)nbxp * nbyp;
            const int32_t *Lp = J.lab[(s - 1) & 1];
            const int r = Bp / B;
            // SPLIT_UNROLL parents per lane and pass: the five labels of
            // each (itself and its 4-neighbours) are loaded together
            for (int64_t p0 = 0; p0 < nbp; p0 += SPLIT_UNROLL * (int64_t)nt) {
                int32_t a[SPLIT_UNROLL], nw[SPLIT_UNROLL], ne[SPLIT_UNROLL], nn[SPLIT_UNROLL], ns[SPLIT_UNROLL];
                int pxb[SPLIT_UNROLL], pyb[SPLIT_UNROLL];
#pragma unroll
                for (int u = 0; u < SPLIT_UNROLL; u++) {
                    const int64_t p = p0 + (int64_t)u * nt + tid;
                    pxb[u] = (int)((uint32_t)p % (uint32_t)nbxp);
                    pyb[u] = (int)((uint32_t)p / (uint32_t)nbxp);
                    const bool in = p < nbp;
                    a[u] = in ? Lp[p] : 0;
                    nw[u] = in ? lab_at(Lp, pxb[u] - 1, pyb[u], nbxp, nbyp) : -1;
                    ne[u] = in ? lab_at(Lp, pxb[u] + 1, pyb[u], nbxp, nbyp) : -1;
                    nn[u] = in ? lab_at(Lp, pxb[u], pyb[u] - 1, nbxp, nbyp) : -1;
                    ns[u] = in ? lab_at(Lp, pxb[u], pyb[u] + 1, nbxp, nbyp) : -1;
                }
#pragma unroll
                for (int u = 0; u < SPLIT_UNROLL; u++) {
                    const bool in = p0 + (int64_t)u * nt + tid < nbp;
                    const bool sw = nw[u] >= 0 && nw[u] != a[u] && pair_on(gv, a[u], nw[u]);
                    const bool se = ne[u] >= 0 && ne[u] != a[u] && pair_on(gv, a[u], ne[u]);
                    const bool sn = nn[u] >= 0 && nn[u] != a[u] && pair_on(gv, a[u], nn[u]);
                    const bool ss = ns[u] >= 0 && ns[u] != a[u] && pair_on(gv, a[u], ns[u]);
#pragma unroll 1
                    for (int ch = 0; ch < r * r; ch++) {
                        int cx = pxb[u] * r + ch % r, cy = pyb[u] * r + ch / r;
                        bool valid = in && cx < nbx && cy < nby;
                        if (valid) L[(int64_t)cy * nbx + cx] = a[u];
                        bool e = valid && ((sw && ch % r == 0) || (se && ch % r == r - 1) ||
                                           (sn && ch / r == 0) || (ss && ch / r == r - 1));
                        if (e) class_push(s_cnt, l_lists, capl, J.lists, capg, 3 * (cy % 3) + (cx % 3),
                                          cy * nbx + cx);
                    }
                }
            }
        } else {
            // boundary blocks of the grid (Eq. (2); Eq. (7) under the gate)
            for (int64_t i0 = 0; i0 < nb; i0 += nt) {
                int64_t i = i0 + tid;
                bool e = false;
                int cls = 0;
                if (i < nb) {
                    int bx = (int)(i % nbx), by = (int)(i / nbx);
                    e = eligible(L, bx, by, nbx, nby, gv);
                    cls = 3 * (by % 3) + (bx % 3);
                }
                if (e) class_push(s_cnt, l_lists, capl, J.lists, capg, cls, (int32_t)i);
            }
        }
        wg_sync();

        int sweeps = 0, converged = 0;
        int n_smin = 0, n_stopo = 0;   // this thread's skip counts of the stage
        for (int t = 0; t < sc.max_sweeps; t++) {
            if (tid == 0) {
                int64_t tot = 0;
                for (int c = 0; c < 9; c++) tot += s_cnt[c];
                s_ctr[0] += (unsigned long long)tot;
            }
            wg_sync();
            int turn = 0;   // alternates with every class phase that runs P1
            for (int c = 0; c < 9; c++) {
                const int ncls = s_cnt[c];
                if (ncls == 0) continue;
                int32_t *const nprop = &s_nprop[turn];
                turn ^= 1;
                const int32_t *llst = l_lists + c * capl;
                // ---- P1: propose from the class-start state
                for (int e0 = 0; e0 < ncls; e0 += nt) {
                    int e = e0 + tid;
                    bool prop = false, smin = false, stopo = false;
                    int32_t bi = 0, a = 0, best = 0;
                    int64_t m = 0;
                    uint64_t Ipk = 0;
                    if (e < ncls) {
                        bi = list_get(llst, capl, J.lists, c * capg, e);
                        // the steps of propose_block written out in place:
                        // the call cost this kernel 1 % in instruction
                        // scheduling (both are checked against the oracle)
                        const int bx = bi % nbx, by = bi / nbx;
                        const bool hw = bx > 0, he = bx + 1 < nbx, hn = by > 0, hs = by + 1 < nby;
                        // every global load of the block at once: its label,
                        // its 3x3 ring and its colour sum
                        const int32_t *Lc = L + bi;
                        a = Lc[0];
                        int32_t rl[8];
                        rl[0] = (hn && hw) ? Lc[-nbx - 1] : -1;
                        rl[1] = hn ? Lc[-nbx] : -1;
                        rl[2] = (hn && he) ? Lc[-nbx + 1] : -1;
                        rl[3] = hw ? Lc[-1] : -1;
                        rl[4] = he ? Lc[1] : -1;
                        rl[5] = (hs && hw) ? Lc[nbx - 1] : -1;
                        rl[6] = hs ? Lc[nbx] : -1;
                        rl[7] = (hs && he) ? Lc[nbx + 1] : -1;
                        int64_t I[3];
                        block_rgb(J, s, B, bi, bx, by, I);
                        Ipk = pack_rgb(I[0], I[1], I[2]);
                        Geo g = block_geo(bx, by, B, W, H);
                        m = g.m;
                        int4 ra;
                        int2 rb;
                        if (SL == 4) pk_means(pk, a, sc, ra, rb);
                        else load_mn(mn, a, ra, rb);
                        if ((int64_t)rb.y - g.m < sc.min_size) {
                            smin = true;
                            if (MERGE) merge_ask(J, a, &s_nreq);
                        } else {
                            uint32_t mask = 0;
#pragma unroll
                            for (int q = 0; q < 8; q++) mask |= (rl[q] == a ? 1u : 0u) << q;
                            if (!((s_lut[mask >> 5] >> (mask & 31)) & 1u)) {
                                stopo = true;
                            } else {
                                // 4-neighbours W, E, N, S and their shared edge lengths
                                const int32_t nl[4] = {rl[3], rl[4], rl[1], rl[6]};
                                const int el[4] = {g.h, g.h, g.w, g.w};
                                // candidate labels: distinct, != a, ascending
                                // (sorting network; excluded values sink as INT_MAX)
                                int32_t q0 = (nl[0] < 0 || nl[0] == a) ? INT32_MAX : nl[0];
                                int32_t q1 = (nl[1] < 0 || nl[1] == a) ? INT32_MAX : nl[1];
                                int32_t q2 = (nl[2] < 0 || nl[2] == a) ? INT32_MAX : nl[2];
                                int32_t q3 = (nl[3] < 0 || nl[3] == a) ? INT32_MAX : nl[3];
                                int32_t t0 = min(q0, q1), t1 = max(q0, q1), t2 = min(q2, q3), t3 = max(q2, q3);
                                int32_t s0 = min(t0, t2), s2 = max(t0, t2), s1 = min(t1, t3), s3 = max(t1, t3);
                                int32_t u1 = min(s1, s2), u2 = max(s1, s2);
                                const int32_t cs[4] = {s0, u1, u2, s3};
                                int bnd_a = 0;
#pragma unroll
                                for (int d = 0; d < 4; d++) bnd_a += (nl[d] >= 0 && nl[d] != a) ? el[d] : 0;
                                best = a;
                                if (use_f64) {
                                    const double dm = (double)g.m, dI0 = (double)I[0], dI1 = (double)I[1],
                                                 dI2 = (double)I[2], dpx = (double)g.px, dpy = (double)g.py;
                                    double estar = energy_f64(ra, rb, sc, dm, dI0, dI1, dI2, dpx, dpy, sc.d_wb * (double)bnd_a);
#pragma unroll
                                    for (int u = 0; u < 4; u++) {
                                        const int32_t k = cs[u];
                                        if (k == INT32_MAX || (u > 0 && k == cs[u - 1])) continue;
                                        int4 ka;
                                        int2 kb;
                                        if (SL == 4) pk_means(pk, k, sc, ka, kb);
                                        else load_mn(mn, k, ka, kb);
                                        if ((int64_t)kb.y + g.m > sc.max_size) continue;
                                        int bnd = 0;
#pragma unroll
                                        for (int d = 0; d < 4; d++) bnd += (nl[d] >= 0 && nl[d] != k) ? el[d] : 0;
                                        double ek = energy_f64(ka, kb, sc, dm, dI0, dI1, dI2, dpx, dpy, sc.d_wb * (double)bnd);
                                        if (ek < estar) {
                                            estar = ek;
                                            best = k;
                                        }
                                    }
                                } else {
                                    int64_t estar = block_energy(ra, rb, g, I, bnd_a, sc);
#pragma unroll
                                    for (int u = 0; u < 4; u++) {
                                        const int32_t k = cs[u];
                                        if (k == INT32_MAX || (u > 0 && k == cs[u - 1])) continue;
                                        int4 ka;
                                        int2 kb;
                                        if (SL == 4) pk_means(pk, k, sc, ka, kb);
                                        else load_mn(mn, k, ka, kb);
                                        if ((int64_t)kb.y + g.m > sc.max_size) continue;
                                        int bnd = 0;
#pragma unroll
                                        for (int d = 0; d < 4; d++) bnd += (nl[d] >= 0 && nl[d] != k) ? el[d] : 0;
                                        int64_t ek = block_energy(ka, kb, g, I, bnd, sc);
                                        if (ek < estar) {
                                            estar = ek;
                                            best = k;
                                        }
                                    }
                                }
                                prop = best != a && pair_on(gv, a, best);
                            }
                        }
                    }
                    n_smin += smin;
                    n_stopo += stopo;
                    if (prop && J.involved && s >= J.involve_stage) {
                        J.involved[a] = 1;
                        J.involved[best] = 1;
                    }
                    int slot = wave_append(nprop, prop);
                    if (slot >= 0) {
                        Prop rec;
                        rec.bi = bi;
                        rec.a = a;
                        rec.k = best;
                        rec.pad = 0;
                        rec.I = Ipk;
                        if (slot < capp) l_props[slot] = rec;
                        else g_props[slot] = rec;
                        atomicAdd(&fl[2 * (int64_t)a], (int32_t)m);
                        atomicAdd(&fl[2 * (int64_t)best + 1], (int32_t)m);
                    }
                }
                wg_sync();
                const int np = *nprop;
                if (np == 0) continue;   // uniform: nothing proposed in this class
                // ---- P2: class-wide size filter, commit, stat moves.  Two
                // lanes per proposal: lane 0 moves the block's sums out of the
                // source a (and writes the label), lane 1 into the target k.
                if (SL == 4) {
                    // packed statistics: every decision first, on the sizes
                    // at class start (the moves below change them), kept in
                    // the record's pad; the moves and the flow counters'
                    // clearing follow, so no refresh pass is needed
                    for (int e = tid; e < np; e += nt) {
                        Prop *rp = e < capp ? l_props + e : g_props + e;
                        const int32_t a = rp->a, k = rp->k;
                        rp->pad = (pk_size(pk, a, sc) - fl[2 * a] >= sc.min_size &&
                                   pk_size(pk, k, sc) + fl[2 * k + 1] <= sc.max_size)
                                      ? 1
                                      : 0;
                    }
                    wg_sync();
                    for (int e0 = 0; e0 < 2 * np; e0 += nt) {
                        const int e = (e0 + tid) >> 1, side = (e0 + tid) & 1;
                        bool com = false;
                        int32_t bi = 0;
                        if (e < np) {
                            const Prop rec = e < capp ? l_props[e] : g_props[e];
                            bi = rec.bi;
                            const int32_t sp = side ? rec.k : rec.a;
                            com = rec.pad != 0;
                            if (com) {
                                const int bx = bi % nbx, by = bi / nbx;
                                const Geo g = block_geo(bx, by, B, W, H);
                                const int64_t sg = side ? 1 : -1;
                                pk_add(pk + 2 * (int64_t)sp, sg * g.m, sg * (int64_t)(rec.I & 0x1FFFFFull),
                                       sg * (int64_t)((rec.I >> 21) & 0x1FFFFFull), sg * (int64_t)(rec.I >> 42),
                                       sg * g.px, sg * g.py, sc);
                                if (mv)
                                    atomicAdd(reinterpret_cast<unsigned long long *>(mv + sp), (unsigned long long)g.m);
                                if (side == 0) L[bi] = rec.k;
                            }
                            fl[2 * sp + side] = 0;
                        }
                        int slot = wave_append(&s_nchg, com && side == 0);
                        if (slot >= 0) list_put(l_chg, capx, J.changed, 0, slot, bi);
                    }
                }
                for (int e0 = 0; SL != 4 && e0 < 2 * np; e0 += nt) {
                    const int e = (e0 + tid) >> 1, side = (e0 + tid) & 1;
                    bool com = false;
                    int32_t bi = 0;
                    if (e < np) {
                        const Prop rec = e < capp ? l_props[e] : g_props[e];
                        bi = rec.bi;
                        const int32_t a = rec.a, k = rec.k;
                        // sizes from the class-start snapshot: the atomics of
                        // this phase are already moving the live counts
                        com = mn_size(mn, a) - fl[2 * a] >= sc.min_size &&
                              mn_size(mn, k) + fl[2 * k + 1] <= sc.max_size;
                        if (com) {
                            const int bx = bi % nbx, by = bi / nbx;
                            const Geo g = block_geo(bx, by, B, W, H);
                            const int64_t sg = side ? 1 : -1;
                            int64_t *rr = st + 6 * (int64_t)(side ? k : a);
                            add64(rr + 0, sg * g.m);
                            add64(rr + 1, sg * (int64_t)(rec.I & 0x1FFFFFull));
                            add64(rr + 2, sg * (int64_t)((rec.I >> 21) & 0x1FFFFFull));
                            add64(rr + 3, sg * (int64_t)(rec.I >> 42));
                            add64(rr + 4, sg * g.px);
                            add64(rr + 5, sg * g.py);
                            if (mv)
                                atomicAdd(reinterpret_cast<unsigned long long *>(mv + (side ? k : a)),
                                          (unsigned long long)g.m);
                            if (side == 0) {
                                L[bi] = k;
                                // P3 refreshes the superpixels of committed moves
                                if (e < capp) l_props[e].pad = 1;
                                else g_props[e].pad = 1;
                            }
                        }
                    }
                    // the changed list doubles as the sweep's commit count
                    int slot = wave_append(&s_nchg, com && side == 0);
                    if (slot >= 0) list_put(l_chg, capx, J.changed, 0, slot, bi);
                }
                wg_sync();
                // ---- P3: refresh the superpixels of committed moves (lane 0 of
                // a proposal its source, lane 1 its target; a superpixel in
                // several moves is refreshed several times with identical
                // values) and clear the flow counters
                for (int q = tid; SL != 4 && q < 2 * np; q += nt) {
                    const int e = q >> 1, side = q & 1;
                    const Prop rec = e < capp ? l_props[e] : g_props[e];
                    const int32_t sp = side ? rec.k : rec.a;
                    fl[2 * sp + side] = 0;
                    if (rec.pad) refresh_sp(st, mn, sp, sc);
                }
                // every thread read np before the P2 barrier: safe to reset
                // (the other counter is zero: its phase either proposed
                // nothing or was reset the same way)
                if (tid == 0) {
                    s_ctr[1] += (unsigned long long)np;
                    *nprop = 0;
                }
                wg_sync();
            }
            wg_sync();
            sweeps = t + 1;
            const int commits = s_nchg;
            if (tid == 0) s_ctr[2] += (unsigned long long)commits;
            if (commits == 0) {
                // a quiet sweep: pending merges go now, and the merged
                // blocks seed the next sweep like committed moves
                int merged = 0;
                if (MERGE && s_nreq > 0)
                    merged = merge_pass(J, st, mn, L, B, nbx, nby, sc, gv, &s_nreq, &s_nchg, &s_merged, l_chg, capx,
                                        tid, nt);
                if (merged == 0) {
                    converged = 1;
                    break;
                }
                if (tid == 0) s_ctr[5] += (unsigned long long)merged;
            }
            // next boundary set: eligible blocks within one block of a change
            const int nchg = s_nchg;
            wg_sync();
            if (tid < 9) s_cnt[tid] = 0;
            wg_sync();
            // nine lanes per changed block, one per block of its 3x3
            // neighbourhood; the first visitor of a block checks eligibility.
            // First visits are found with the LDS bitmap when it covers the
            // stage, else with an LDS hash set in the same words when the
            // visits fit it at half load, else with the global stamps.
            const int32_t stamp = s * (sc.max_sweeps + 1) + t + 1;
            const bool use_hash = !use_bm && 9 * nchg <= ht_cap / 2;
            // FRONT_UNROLL neighbourhood blocks per lane and pass: their
            // first-visit tests (global stamps: atomics that return) and
            // then their eligibility loads are issued together
            for (int q0 = tid; q0 < 9 * nchg; q0 += FRONT_UNROLL * nt) {
                int32_t ni[FRONT_UNROLL];
                int bxs[FRONT_UNROLL], bys[FRONT_UNROLL];
                bool ok[FRONT_UNROLL];
#pragma unroll
                for (int u = 0; u < FRONT_UNROLL; u++) {
                    const int q = q0 + u * nt;
                    ok[u] = q < 9 * nchg;
                    const int32_t bi = ok[u] ? list_get(l_chg, capx, J.changed, 0, q / 9) : 0;
                    const int d = q % 9;
                    bxs[u] = bi % nbx + (d % 3) - 1;
                    bys[u] = bi / nbx + (d / 3) - 1;
                    ok[u] = ok[u] && bxs[u] >= 0 && bys[u] >= 0 && bxs[u] < nbx && bys[u] < nby;
                    ni[u] = bys[u] * nbx + bxs[u];
                }
#pragma unroll
                for (int u = 0; u < FRONT_UNROLL; u++) {
                    if (!ok[u]) continue;
                    if (use_bm) {
                        const uint32_t bit = 1u << (ni[u] & 31);
                        ok[u] = (atomicOr(&l_bm[ni[u] >> 5], bit) & bit) == 0;
                    } else if (use_hash) {
                        ok[u] = hash_insert(l_bm, ht_cap - 1, ni[u]);
                    } else {
                        ok[u] = atomicExch(&J.stamp[ni[u]], stamp) != stamp;
                    }
                }
                bool el[FRONT_UNROLL];
#pragma unroll
                for (int u = 0; u < FRONT_UNROLL; u++) el[u] = ok[u] && eligible(L, bxs[u], bys[u], nbx, nby, gv);
#pragma unroll
                for (int u = 0; u < FRONT_UNROLL; u++)
                    if (el[u]) class_push(s_cnt, l_lists, capl, J.lists, capg, 3 * (bys[u] % 3) + (bxs[u] % 3), ni[u]);
            }
            wg_sync();
            if (use_bm)
                for (int i = tid; i < (int)((nb + 31) >> 5); i += nt) l_bm[i] = 0;
            else if (use_hash)
                for (int i = tid; i < ht_cap; i += nt) l_bm[i] = 0;
            if (tid == 0) s_nchg = 0;
            wg_sync();
        }
        if (n_smin) atomicAdd(&s_ctr[3], (unsigned long long)n_smin);
        if (n_stopo) atomicAdd(&s_ctr[4], (unsigned long long)n_stopo);
        if (MERGE) {
            // asks do not outlive the stage
            const int nreq = s_nreq;
            for (int r = tid; r < nreq; r += nt) {
                const int32_t m = J.mlist[r];
                atomicAnd(&J.mreq[m >> 5], ~(1u << (m & 31)));
            }
        }
        wg_sync();
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
            r.merges = (int64_t)s_ctr[5];
            J.rep[s] = r;
            s_nchg = 0;
            s_nreq = 0;
        }
        wg_sync();
    }
    if (SL == 1)
        for (int64_t i = tid; i < 6 * (int64_t)K; i += nt) J.stats[i] = st[i];
    if (SL == 4)
        for (int k = tid; k < K; k += nt) {
            int64_t r[6];
            pk_unpack(pk + 2 * (int64_t)k, r, sc);
            for (int q = 0; q < 6; q++) J.stats[6 * (int64_t)k + q] = r[q];
        }
    if ((flags & FLAG_OUT) && s_end > 0 && J.tile) {
        // slide tile: core pixels only, labels as slide-wide cell ids
        const int B = sc.B[out_stage];
        const int nbx = (W + B - 1) / B;
        const int32_t *L = J.lab[out_stage & 1];
        const uint32_t cw = (uint32_t)J.core_w, ncore = cw * (uint32_t)J.core_h;
        const int32_t gx = J.gx;
        // OUT_UNROLL pixels per lane and pass, every label load issued
        // before the first store (W, H <= 8192: 32-bit pixel indices)
        for (uint32_t i0 = (uint32_t)tid; i0 < ncore; i0 += OUT_UNROLL * (uint32_t)nt) {
            int32_t k[OUT_UNROLL];
            int x[OUT_UNROLL], y[OUT_UNROLL];
#pragma unroll
            for (int u = 0; u < OUT_UNROLL; u++) {
                const uint32_t i = i0 + (uint32_t)u * (uint32_t)nt;
                x[u] = J.core_x0 + (int)(i % cw);
                y[u] = J.core_y0 + (int)(i / cw);
                k[u] = i < ncore ? L[(y[u] / B) * nbx + x[u] / B] : -1;
            }
#pragma unroll
            for (int u = 0; u < OUT_UNROLL; u++)
                if (k[u] >= 0)
                    J.out[(int64_t)y[u] * J.out_stride + x[u]] =
                        (int32_t)((J.gid_y0 + k[u] / gx) * J.gid_w + J.gid_x0 + k[u] % gx);
        }
    } else if ((flags & FLAG_OUT) && s_end > 0) {
        const int B = sc.B[out_stage];
        const int nbx = (W + B - 1) / B;
        const int32_t *L = J.lab[out_stage & 1];
        if (!(B == 1 && L == J.out)) {
            const uint32_t npx = (uint32_t)W * (uint32_t)H;
            for (uint32_t i0 = (uint32_t)tid; i0 < npx; i0 += OUT_UNROLL * (uint32_t)nt) {
                int32_t k[OUT_UNROLL];
                int x[OUT_UNROLL], y[OUT_UNROLL];
#pragma unroll
                for (int u = 0; u < OUT_UNROLL; u++) {
                    const uint32_t i = i0 + (uint32_t)u * (uint32_t)nt;
                    x[u] = (int)(i % (uint32_t)W);
                    y[u] = (int)(i / (uint32_t)W);
                    k[u] = i < npx ? L[(y[u] / B) * nbx + x[u] / B] : -1;
                }
#pragma unroll
                for (int u = 0; u < OUT_UNROLL; u++)
                    if (k[u] >= 0) J.out[(int64_t)y[u] * J.out_stride + x[u]] = k[u];
            }
        }
    }
}

// The refinement launch over n_jobs images or tiles.  queue == nullptr: one
// workgroup per job (workgroup b refines job b).  Otherwise a persistent
// launch over a work queue: every workgroup takes its next job from the
// queue counter (zeroed before the launch) until the jobs run out, so the
// grid can be sized to what the chip holds at once and the host's job order
// (largest first) is the order in which they start.  Every workgroup leaves
// once the counter has passed n_jobs.
template <int SL, int GM, bool MERGE>
__global__ __launch_bounds__(1024) void k_refine(const Job *__restrict__ jobs, int n_jobs, uint32_t *queue, Sched sc,
                                                  LdsPlan lp, int s_begin, int s_end, int flags,
                                                  const uint32_t *__restrict__ lut_g)
{
    __shared__ int32_t s_job;
    int job = blockIdx.x;
    for (;;) {
        if (queue) {
            if (threadIdx.x == 0) s_job = (int32_t)atomicAdd(queue, 1u);
            __syncthreads();
            job = s_job;
        }
        if (job >= n_jobs) break;
        refine_job<SL, GM, MERGE>(jobs[job], sc, lp, s_begin, s_end, flags, lut_g);
        if (!queue) break;
        // every lane is done with this job's LDS (and has read s_job)
        __syncthreads();
    }
}

// ------------------------------------------- one image on many workgroups
// k_refine_mc: the same stage loop, class phases and counters as k_refine,
// for a single image whose class phases hold thousands of blocks.  G
// workgroups of one cooperative launch share the image: every pass is split
// over all G * nt lanes, and the phases are separated by grid barriers
// instead of workgroup barriers.  The per-superpixel state, the work lists
// and their counters live in global memory (the control words J.ctl, zeroed
// by the host before the launch); device-scope integer atomics keep every
// sum exact, so the labels equal those of k_refine bit for bit.

// Grid barrier over the workgroups of a cooperative launch.  The arrival
// counter only grows (the n-th barrier waits for n * G arrivals); thread 0
// publishes the workgroup's writes before it arrives (agent-scope release:
// L2 writeback) and invalidates its caches after the wait (agent-scope
// acquire: L2 invalidation), one of each per barrier.  The wait is bounded: past
// the spin limit, or when another workgroup gave up, it raises the abort
// word and returns false, and the caller leaves the kernel, so that every
// workgroup exits.
constexpr uint32_t GRID_SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ bool grid_sync(uint32_t *ctl, uint32_t &target, int32_t *s_ok)
{
    __syncthreads();
    target += gridDim.x;
    if (threadIdx.x == 0) {
        int ok = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomicAdd(&ctl[CTL_BAR], 1u);
        uint32_t spins = 0;
        while (__hip_atomic_load(&ctl[CTL_BAR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&ctl[CTL_ABORT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                ++spins > GRID_SPIN_LIMIT) {
                atomicExch(&ctl[CTL_ABORT], 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// A word of the control block that other workgroups update, read after a
// grid barrier (an atomic load: never served from a stale cache).
__device__ __forceinline__ int32_t ctl_read(const uint32_t *ctl, int w)
{
    return (int32_t)__hip_atomic_load(&ctl[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Class-list append aggregated per workgroup and pass: slots are taken with
// LDS atomics, then one global atomic per class reserves the workgroup's
// range.  Every thread of the workgroup calls it once per pass.
__device__ __forceinline__ void class_push_wg(bool e, int cls, int32_t v, int32_t *l_cnt, int32_t *l_base,
                                              uint32_t *g_cnt, int32_t *glob, int64_t capg)
{
    const int slot = e ? atomicAdd(&l_cnt[cls], 1) : 0;
    __syncthreads();
    if (threadIdx.x < 9) {
        const int n = l_cnt[threadIdx.x];
        l_base[threadIdx.x] = n ? (int32_t)atomicAdd(&g_cnt[threadIdx.x], (uint32_t)n) : 0;
        l_cnt[threadIdx.x] = 0;
    }
    __syncthreads();
    if (e) glob[cls * capg + l_base[cls] + slot] = v;
}

// The gate point of a cooperative launch (one image on G workgroups,
// Algorithm RAPID's prediction step before the gated level): the features of
// every superpixel on the labels of stage stage_q (the statistics in their
// six-word layout in J.stats), then the network's decision (Eq. (6)) into
// J.gate_out, each pass spread over the grid and closed by a grid barrier.
// Returns false when a barrier gave up (the caller leaves the kernel).
// Kept out of line so that the sweep's registers do not carry it.
__device__ __forceinline__ bool gate_point_mc(const Job &J, const Sched &sc, int stage_q, int64_t gt,
                                                         int64_t gn, uint32_t *ctl, uint32_t &bar, int32_t *s_ok)
{
    const int K = J.K, F = sc.F;
    const int Bq = sc.B[stage_q];
    const int nbxq = (J.W + Bq - 1) / Bq, nbyq = (J.H + Bq - 1) / Bq;
    const int32_t *Lq = J.lab[stage_q & 1];
    const uint32_t *moms = (J.moms && J.moms_stage == stage_q) ? J.moms : nullptr;
    for (int64_t k = gt; k < K; k += gn) feat_init_sp(J.stats, J.fmean, J.facc, (int)k, F);
    if (!grid_sync(ctl, bar, s_ok)) return false;
    const int spr = (nbxq + FEAT_SEG - 1) / FEAT_SEG;
    for (int64_t g = gt; g < (int64_t)spr * nbyq; g += gn) {
        const int by = (int)(g / spr), bx0 = (int)(g % spr) * FEAT_SEG;
        const int32_t *row = Lq + (int64_t)by * nbxq;
        feat_segment(J, row, by > 0 ? row - nbxq : nullptr, by + 1 < nbyq ? row + nbxq : nullptr, Bq, nbxq, by, bx0,
                     min(bx0 + FEAT_SEG, nbxq), moms, J.fmean, GlobalSink{J.facc});
    }
    if (!grid_sync(ctl, bar, s_ok)) return false;
    for (int64_t k = gt; k < K; k += gn)
        feat_final_sp(J, J.stats, J.facc, J.moved, (int)k, F, sc.feat_set, J.xrow + 16 * k);
    if (!grid_sync(ctl, bar, s_ok)) return false;
    // one wave per 16 superpixels (the wave index is uniform in a wave)
    const int lane = (int)(threadIdx.x & 63);
    for (int64_t t = gt >> 6; t < ((int64_t)K + 15) / 16; t += gn >> 6) {
        const int64_t n = 16 * t + (lane & 15);
        const float z = mlp_logit(sc.mlp_w, load_x(J.xrow, n, K, lane >> 4), lane);
        if (lane < 16 && n < K) J.gate_out[n] = z >= sc.mlp_thresh ? 1 : 0;
    }
    return grid_sync(ctl, bar, s_ok);
}

#define MC_SYNC()                                  \
    do {                                           \
        if (!grid_sync(ctl, bar, &s_ok)) return;   \
    } while (0)

// PK: packed statistics (two words per superpixel in J.means, updated with
// device-scope atomics; the means are computed where they are read), the
// flow counters and the proposal counter double-buffered by class phase, so
// that a class fitting one pass needs two grid barriers instead of three
// and no refresh pass.
template <int GM, bool PK>
__global__ __launch_bounds__(1024) void k_refine_mc(const Job *__restrict__ jobs, Sched sc, int s_begin, int s_end,
                                                    int flags, const uint32_t *__restrict__ lut_g, int64_t solo_max)
{
    // GM_BITS: the gate bits of all superpixels, loaded into LDS (dynamic,
    // (K + 31) / 32 words) at the first gated stage
    extern __shared__ uint32_t l_gate[];
    __shared__ uint32_t s_lut[8];
    __shared__ int32_t s_ok;
    __shared__ int32_t l_cnt[9], l_base[9];
    __shared__ unsigned long long s_skip[2];

    const Job &J = jobs[0];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t gt = (int64_t)blockIdx.x * nt + tid, gn = (int64_t)gridDim.x * nt;
    const int64_t wg0 = (int64_t)blockIdx.x * nt;   // first lane of this workgroup
    const int W = J.W, H = J.H, K = J.K;
    int64_t *const st = J.stats;
    int32_t *const mn = J.means, *const fl = J.flow;
    unsigned long long *const pk = reinterpret_cast<unsigned long long *>(J.means);
    uint32_t *const ctl = J.ctl;
    unsigned long long *const ctr = reinterpret_cast<unsigned long long *>(ctl + CTL_CTR);
    Prop *const props = J.props;
    const int64_t capg = J.capc;
    uint32_t bar = 0;
    GateView gv;
    gv.bits = nullptr;
    gv.tt = rule_table(sc.gate_rule);
    bool gate_loaded = false;

    if (tid < 8) s_lut[tid] = lut_g[tid];
    if (tid < 9) l_cnt[tid] = 0;
    if (tid < 2) s_skip[tid] = 0;
    for (int64_t i = gt; i < (PK ? 4 : 2) * (int64_t)K; i += gn) fl[i] = 0;
    if (GM == GM_FUSED)   // pixels moved before the gate point, a feature
        for (int64_t i = gt; i < K; i += gn) J.moved[i] = 0;
    if (s_end > s_begin) {
        // visit stamps are unique per (stage, sweep) of this launch
        const int Bf = sc.B[s_end - 1];
        const int64_t nbf = (int64_t)((W + Bf - 1) / Bf) * ((H + Bf - 1) / Bf);
        for (int64_t i = gt; i < nbf; i += gn) J.stamp[i] = 0;
    }
    if (flags & FLAG_INIT) {
        // grid initialisation and statistics (Algorithm RAPID, first step)
        if (PK)
            for (int64_t i = gt; i < 2 * (int64_t)K; i += gn) pk[i] = 0;
        else
            for (int64_t i = gt; i < 6 * (int64_t)K; i += gn) st[i] = 0;
        // the block-sum pyramid over the whole grid, its levels separated
        // by grid barriers, so that the image takes this one launch
        if (flags & FLAG_PYRAMID) {
            if (!build_pyramid(J, sc, (int)gt, (int)gn, [&]() { return grid_sync(ctl, bar, &s_ok); })) return;
        } else {
            MC_SYNC();
        }
        const int B0 = sc.B[0];
        const int nbx = (W + B0 - 1) / B0, nby = (H + B0 - 1) / B0;
        int32_t *L = J.lab[0];
        for (int64_t i = gt; i < (int64_t)nbx * nby; i += gn) {
            int bx = (int)(i % nbx), by = (int)(i / nbx);
            Geo g = block_geo(bx, by, B0, W, H);
            int64_t row = ((2 * (int64_t)by * B0 + g.h) * J.gy) / (2 * (int64_t)H);
            int64_t col = ((2 * (int64_t)bx * B0 + g.w) * J.gx) / (2 * (int64_t)W);
            int32_t k = (int32_t)(row * J.gx + col);
            L[i] = k;
            int64_t I[3];
            block_rgb(J, 0, B0, i, bx, by, I);
            if (PK) {
                pk_add(pk + 2 * (int64_t)k, g.m, I[0], I[1], I[2], g.px, g.py, sc);
            } else {
                int64_t *r = st + 6 * (int64_t)k;
                add64(r + 0, g.m);
                add64(r + 1, I[0]);
                add64(r + 2, I[1]);
                add64(r + 3, I[2]);
                add64(r + 4, g.px);
                add64(r + 5, g.py);
            }
        }
    } else if (PK) {
        for (int64_t k = gt; k < K; k += gn) pk_store(pk, (int)k, st + 6 * k, sc);
    }
    MC_SYNC();
    if (!PK) {
        for (int64_t k = gt; k < K; k += gn) refresh_sp(st, mn, (int)k, sc);
        MC_SYNC();
    }
    // PK: the phases of a sweep alternate between two flow buffers and two
    // proposal counters; a lane clears the flows of its last one-pass
    // proposal at the start of the next phase that runs, or at the sweep's
    // end
    int32_t pend_a = -1, pend_k = -1;

    // Class counts are double-buffered: the sweep reads cnt[par] while the
    // frontier rebuild fills cnt[par ^ 1]; the changed-block counter of a
    // sweep is nchg[par].
    int par = 0;
    for (int s = s_begin; s < s_end; s++) {
        const int B = sc.B[s];
        const int nbx = (W + B - 1) / B, nby = (H + B - 1) / B;
        const int64_t nb = (int64_t)nbx * nby;
        int32_t *L = J.lab[s & 1];
        const bool use_f64 = sc.f64[s] != 0;
        int64_t *const mv = (GM == GM_FUSED && s >= sc.gate_stage) ? nullptr : J.moved;
        if (GM == GM_FUSED && s == sc.gate_stage && s > 0) {
            // the prediction step inside the launch: features on the
            // previous stage's labels, then the network's gate bits
            if (PK) {
                for (int64_t k = gt; k < K; k += gn) {
                    int64_t r[6];
                    pk_unpack(pk + 2 * k, r, sc);
                    for (int q = 0; q < 6; q++) st[6 * k + q] = r[q];
                }
                MC_SYNC();
            }
            if (!gate_point_mc(J, sc, s - 1, gt, gn, ctl, bar, &s_ok)) return;
        }
        if (GM != GM_NONE && J.gate && s >= sc.gate_stage) {
            if (!gate_loaded) {
                // first gated stage: every workgroup its own copy of the bits
                // (read-only; the grid barrier below orders it before use)
                for (int w = tid; w < (K + 31) / 32; w += nt) {
                    uint32_t v = 0;
                    for (int b = 0; b < 32 && 32 * w + b < K; b++) v |= (J.gate[32 * w + b] != 0 ? 1u : 0u) << b;
                    l_gate[w] = v;
                }
                gate_loaded = true;
            }
            gv.bits = l_gate;
        }
        if (gt < 9) ctl[CTL_CNT + 9 * par + gt] = 0;
        if (gt == 0) {
            ctl[CTL_NCHG] = 0;
            ctl[CTL_NCHG + 1] = 0;
        }
        MC_SYNC();
        uint32_t *cnt = ctl + CTL_CNT + 9 * par;
        if (s > 0) {
            // split: each block inherits its parent's label; a child is a
            // boundary block only on a side where its parent borders another
            // (active) label
            const int Bp = sc.B[s - 1];
            const int nbxp = (W + Bp - 1) / Bp, nbyp = (H + Bp - 1) / Bp;
            const int64_t nbp = (int64_t)nbxp * nbyp;
            const int32_t *Lp = J.lab[(s - 1) & 1];
            const int r = Bp / B;
            for (int64_t p0 = wg0; p0 < nbp; p0 += gn) {
                const int64_t p = p0 + tid;
                int32_t a = 0;
                bool sw = false, se = false, sn = false, ss = false;
                int pxb = 0, pyb = 0;
                if (p < nbp) {
                    pxb = (int)(p % nbxp);
                    pyb = (int)(p / nbxp);
                    a = Lp[p];
                    int32_t k;
                    k = lab_at(Lp, pxb - 1, pyb, nbxp, nbyp);
                    sw = k >= 0 && k != a && pair_on(gv, a, k);
                    k = lab_at(Lp, pxb + 1, pyb, nbxp, nbyp);
                    se = k >= 0 && k != a && pair_on(gv, a, k);
                    k = lab_at(Lp, pxb, pyb - 1, nbxp, nbyp);
                    sn = k >= 0 && k != a && pair_on(gv, a, k);
                    k = lab_at(Lp, pxb, pyb + 1, nbxp, nbyp);
                    ss = k >= 0 && k != a && pair_on(gv, a, k);
                }
                for (int ch = 0; ch < r * r; ch++) {
                    const int cx = pxb * r + ch % r, cy = pyb * r + ch / r;
                    const bool valid = p < nbp && cx < nbx && cy < nby;
                    if (valid) L[(int64_t)cy * nbx + cx] = a;
                    const bool e = valid && ((sw && ch % r == 0) || (se && ch % r == r - 1) ||
                                             (sn && ch / r == 0) || (ss && ch / r == r - 1));
                    class_push_wg(e, 3 * (cy % 3) + (cx % 3), cy * nbx + cx, l_cnt, l_base, cnt, J.lists, capg);
                }
            }
        } else {
            // boundary blocks of the grid (Eq. (2); Eq. (7) under the gate)
            for (int64_t i0 = wg0; i0 < nb; i0 += gn) {
                const int64_t i = i0 + tid;
                bool e = false;
                int cls = 0;
                if (i < nb) {
                    const int bx = (int)(i % nbx), by = (int)(i / nbx);
                    e = eligible(L, bx, by, nbx, nby, gv);
                    cls = 3 * (by % 3) + (bx % 3);
                }
                class_push_wg(e, cls, (int32_t)i, l_cnt, l_base, cnt, J.lists, capg);
            }
        }
        MC_SYNC();

        int sweeps = 0, converged = 0;
        int n_smin = 0, n_stopo = 0;
        for (int t = 0; t < sc.max_sweeps; t++) {
            cnt = ctl + CTL_CNT + 9 * par;
            int64_t tot = 0;
            for (int c = 0; c < 9; c++) tot += ctl_read(cnt, c);
            // A sweep with few active blocks runs on workgroup 0 alone, with
            // workgroup barriers; the other workgroups wait at its end.
            const bool solo = tot <= solo_max;
            const int64_t first = solo ? 0 : wg0, step = solo ? (int64_t)nt : gn;
            uint32_t cph = 0;   // class phases run so far in this sweep
#define SW_SYNC()              \
    do {                       \
        if (solo)              \
            __syncthreads();   \
        else                   \
            MC_SYNC();         \
    } while (0)
            // the other buffers start the sweep clear (their last readers
            // passed at least one grid barrier ago)
            if (gt < 9) ctl[CTL_CNT + 9 * (par ^ 1) + gt] = 0;
            if (gt == 0) {
                ctr[0] += (unsigned long long)tot;
                ctl[CTL_NCHG + par] = 0;
            }
            int32_t *const nchg = reinterpret_cast<int32_t *>(ctl + CTL_NCHG + par);
            if (!solo || blockIdx.x == 0) {
                for (int c = 0; c < 9; c++) {
                    const int ncls = ctl_read(cnt, c);   // stable during the sweep
                    if (ncls == 0) continue;
                    const int32_t *llst = J.lists + c * capg;
                    // This phase's proposal counter (and, PK, flow buffer);
                    // the previous phase's counter (and this lane's flows in
                    // the other buffer) are cleared: their readers passed a
                    // barrier since, or read a counter that stayed 0 and went
                    // on without one, and their next writers come after this
                    // phase's first barrier.  A phase that proposes nothing
                    // is followed by the next phase's P1 without a barrier,
                    // so the two must not share a counter.
                    const uint32_t pb = cph & 1;
                    int32_t *const flc = PK ? fl + 2 * (int64_t)K * pb : fl;
                    const int nprop_w = CTL_NPROP + (int)pb;
                    if (cph > 0 && gt == 0) ctl[CTL_NPROP + (pb ^ 1)] = 0;
                    cph++;
                    if (PK) {
                        if (pend_a >= 0) {
                            int32_t *const flo = fl + 2 * (int64_t)K * (pb ^ 1);
                            flo[2 * (int64_t)pend_a] = 0;
                            flo[2 * (int64_t)pend_k + 1] = 0;
                            pend_a = -1;
                        }
                    }
                    if (ncls <= step) {
                        // One pass: every lane keeps its block's proposal in
                        // registers through P2 and P3 (no proposal records;
                        // the proposal counter only counts).
                        const int64_t e = first + tid;
                        bool prop = false, smin = false, stopo = false;
                        int32_t bi = 0, a = 0, best = 0;
                        int64_t m = 0;
                        uint64_t Ipk = 0;
                        int64_t na = 0, nk = 0;   // class-start sizes of a and best
                        if (e < ncls) {
                            bi = llst[e];
                            propose_block<PK>(J, s, B, bi, nbx, nby, W, H, L, mn, s_lut, sc, gv, use_f64, a, best, m,
                                              Ipk, prop, smin, stopo, na, nk);
                        }
                        n_smin += smin;
                        n_stopo += stopo;
                        if (prop && J.involved && s >= J.involve_stage) {
                            J.involved[a] = 1;
                            J.involved[best] = 1;
                        }
                        const uint64_t pm = __ballot(prop);
                        if (pm != 0 && lane_id() == __ffsll((unsigned long long)pm) - 1)
                            atomicAdd(&ctl[nprop_w], (uint32_t)__popcll(pm));
                        if (prop) {
                            atomicAdd(&flc[2 * (int64_t)a], (int32_t)m);
                            atomicAdd(&flc[2 * (int64_t)best + 1], (int32_t)m);
                        }
                        SW_SYNC();
                        const int np = ctl_read(ctl, nprop_w);
                        if (np == 0) continue;   // uniform
                        // ---- P2: size filter on the class-wide flows, commit
                        // (both sides of the move in one lane)
                        bool com = false;
                        if (prop) {
                            com = PK ? (na - flc[2 * (int64_t)a] >= sc.min_size &&
                                        nk + flc[2 * (int64_t)best + 1] <= sc.max_size)
                                     : (mn_size(mn, a) - fl[2 * (int64_t)a] >= sc.min_size &&
                                        mn_size(mn, best) + fl[2 * (int64_t)best + 1] <= sc.max_size);
                            if (com) {
                                const Geo g = block_geo(bi % nbx, bi / nbx, B, W, H);
                                const int64_t d[6] = {g.m, (int64_t)(Ipk & 0x1FFFFFull),
                                                      (int64_t)((Ipk >> 21) & 0x1FFFFFull), (int64_t)(Ipk >> 42),
                                                      g.px, g.py};
                                if (PK) {
                                    pk_add(pk + 2 * (int64_t)a, -d[0], -d[1], -d[2], -d[3], -d[4], -d[5], sc);
                                    pk_add(pk + 2 * (int64_t)best, d[0], d[1], d[2], d[3], d[4], d[5], sc);
                                } else {
                                    int64_t *ra = st + 6 * (int64_t)a, *rk = st + 6 * (int64_t)best;
#pragma unroll
                                    for (int q = 0; q < 6; q++) {
                                        add64(ra + q, -d[q]);
                                        add64(rk + q, d[q]);
                                    }
                                }
                                if (mv) {
                                    atomicAdd(reinterpret_cast<unsigned long long *>(mv + a), (unsigned long long)g.m);
                                    atomicAdd(reinterpret_cast<unsigned long long *>(mv + best),
                                              (unsigned long long)g.m);
                                }
                                L[bi] = best;
                            }
                        }
                        const int slot = wave_append(nchg, com);
                        if (slot >= 0) J.changed[slot] = bi;
                        if (PK) {
                            // no refresh: the next phase computes the means
                            if (prop) {
                                pend_a = a;
                                pend_k = best;
                            }
                            if (gt == 0) ctr[1] += (unsigned long long)np;
                            SW_SYNC();
                            continue;
                        }
                        SW_SYNC();
                        // ---- P3: refresh the moved superpixels, clear the
                        // flow counters
                        if (prop) {
                            fl[2 * (int64_t)a] = 0;
                            fl[2 * (int64_t)best + 1] = 0;
                            if (com) {
                                refresh_sp(st, mn, a, sc);
                                refresh_sp(st, mn, best, sc);
                            }
                        }
                        // every lane read np before the P2 barrier: safe to reset
                        if (gt == 0) {
                            ctr[1] += (unsigned long long)np;
                            ctl[nprop_w] = 0;
                        }
                        SW_SYNC();
                        continue;
                    }
                    // ---- P1: propose from the class-start state
                    for (int64_t e0 = first; e0 < ncls; e0 += step) {
                        const int e = (int)(e0 + tid);
                        bool prop = false, smin = false, stopo = false;
                        int32_t bi = 0, a = 0, best = 0;
                        int64_t m = 0;
                        uint64_t Ipk = 0;
                        int64_t na = 0, nk = 0;
                        if (e < ncls) {
                            bi = llst[e];
                            propose_block<PK>(J, s, B, bi, nbx, nby, W, H, L, mn, s_lut, sc, gv, use_f64, a, best, m,
                                              Ipk, prop, smin, stopo, na, nk);
                        }
                        n_smin += smin;
                        n_stopo += stopo;
                        if (prop && J.involved && s >= J.involve_stage) {
                            J.involved[a] = 1;
                            J.involved[best] = 1;
                        }
                        const int slot = wave_append(reinterpret_cast<int32_t *>(ctl + nprop_w), prop);
                        if (slot >= 0) {
                            Prop rec;
                            rec.bi = bi;
                            rec.a = a;
                            rec.k = best;
                            rec.pad = 0;
                            rec.I = Ipk;
                            props[slot] = rec;
                            atomicAdd(&flc[2 * (int64_t)a], (int32_t)m);
                            atomicAdd(&flc[2 * (int64_t)best + 1], (int32_t)m);
                        }
                    }
                    SW_SYNC();
                    const int np = ctl_read(ctl, nprop_w);
                    if (np == 0) continue;   // uniform
                    if (PK) {
                        // every decision on the class-start sizes first, then
                        // the moves (packed, device-scope atomics), the label
                        // writes and the flows' clearing
                        for (int64_t e = first + tid; e < np; e += step) {
                            const int32_t a = props[e].a, k = props[e].k;
                            props[e].pad = (pk_size(pk, a, sc) - flc[2 * (int64_t)a] >= sc.min_size &&
                                            pk_size(pk, k, sc) + flc[2 * (int64_t)k + 1] <= sc.max_size)
                                               ? 1
                                               : 0;
                        }
                        SW_SYNC();
                        for (int64_t e0 = first; e0 < 2 * (int64_t)np; e0 += step) {
                            const int64_t q = e0 + tid;
                            const int e = (int)(q >> 1), side = (int)(q & 1);
                            bool com = false;
                            int32_t bi = 0;
                            if (e < np) {
                                const Prop rec = props[e];
                                bi = rec.bi;
                                const int32_t sp = side ? rec.k : rec.a;
                                com = rec.pad != 0;
                                if (com) {
                                    const Geo g = block_geo(bi % nbx, bi / nbx, B, W, H);
                                    const int64_t sg = side ? 1 : -1;
                                    pk_add(pk + 2 * (int64_t)sp, sg * g.m, sg * (int64_t)(rec.I & 0x1FFFFFull),
                                           sg * (int64_t)((rec.I >> 21) & 0x1FFFFFull), sg * (int64_t)(rec.I >> 42),
                                           sg * g.px, sg * g.py, sc);
                                    if (mv)
                                        atomicAdd(reinterpret_cast<unsigned long long *>(mv + sp),
                                                  (unsigned long long)g.m);
                                    if (side == 0) L[bi] = rec.k;
                                }
                                flc[2 * (int64_t)sp + side] = 0;
                            }
                            const int slot = wave_append(nchg, com && side == 0);
                            if (slot >= 0) J.changed[slot] = bi;
                        }
                        if (gt == 0) ctr[1] += (unsigned long long)np;
                        SW_SYNC();
                        continue;
                    }
                    // ---- P2: class-wide size filter, commit, statistic
                    // moves (lane 0 of a proposal: source side and label
                    // write, lane 1 target side)
                    for (int64_t e0 = first; e0 < 2 * (int64_t)np; e0 += step) {
                        const int64_t q = e0 + tid;
                        const int e = (int)(q >> 1), side = (int)(q & 1);
                        bool com = false;
                        int32_t bi = 0;
                        if (e < np) {
                            const Prop rec = props[e];
                            bi = rec.bi;
                            const int32_t a = rec.a, k = rec.k;
                            com = mn_size(mn, a) - fl[2 * a] >= sc.min_size &&
                                  mn_size(mn, k) + fl[2 * k + 1] <= sc.max_size;
                            if (com) {
                                const int bx = bi % nbx, by = bi / nbx;
                                const Geo g = block_geo(bx, by, B, W, H);
                                const int64_t sg = side ? 1 : -1;
                                int64_t *rr = st + 6 * (int64_t)(side ? k : a);
                                add64(rr + 0, sg * g.m);
                                add64(rr + 1, sg * (int64_t)(rec.I & 0x1FFFFFull));
                                add64(rr + 2, sg * (int64_t)((rec.I >> 21) & 0x1FFFFFull));
                                add64(rr + 3, sg * (int64_t)(rec.I >> 42));
                                add64(rr + 4, sg * g.px);
                                add64(rr + 5, sg * g.py);
                                if (mv)
                                    atomicAdd(reinterpret_cast<unsigned long long *>(mv + (side ? k : a)),
                                              (unsigned long long)g.m);
                                if (side == 0) {
                                    L[bi] = k;
                                    props[e].pad = 1;
                                }
                            }
                        }
                        const int slot = wave_append(nchg, com && side == 0);
                        if (slot >= 0) J.changed[slot] = bi;
                    }
                    SW_SYNC();
                    // ---- P3: refresh the superpixels of committed moves,
                    // clear the flow counters
                    for (int64_t q = first + tid; q < 2 * (int64_t)np; q += step) {
                        const int e = (int)(q >> 1), side = (int)(q & 1);
                        const Prop rec = props[e];
                        const int32_t sp = side ? rec.k : rec.a;
                        fl[2 * sp + side] = 0;
                        if (rec.pad) refresh_sp(st, mn, sp, sc);
                    }
                    // every lane read np before the P2 barrier: safe to reset
                    if (gt == 0) {
                        ctr[1] += (unsigned long long)np;
                        ctl[nprop_w] = 0;
                    }
                    SW_SYNC();
                }
                // the sweep's last phase: its counters (and, PK, flows) clear
                // before the next sweep (the barrier below orders them)
                if (PK && pend_a >= 0) {
                    int32_t *const flo = fl + 2 * (int64_t)K * ((cph - 1) & 1);
                    flo[2 * (int64_t)pend_a] = 0;
                    flo[2 * (int64_t)pend_k + 1] = 0;
                    pend_a = -1;
                }
                if (gt == 0) {
                    ctl[CTL_NPROP] = 0;
                    ctl[CTL_NPROP + 1] = 0;
                }
                SW_SYNC();
                const int commits = ctl_read(ctl, CTL_NCHG + par);
                if (gt == 0) ctr[2] += (unsigned long long)commits;
                if (commits > 0) {
                    // next boundary set: eligible blocks within one block of
                    // a change, first visits found with the global stamps
                    const int32_t stamp = s * (sc.max_sweeps + 1) + t + 1;
                    uint32_t *const ncnt = ctl + CTL_CNT + 9 * (par ^ 1);
                    for (int64_t q0 = first; q0 < 9 * (int64_t)commits; q0 += step) {
                        const int64_t q = q0 + tid;
                        bool e = false;
                        int cls = 0;
                        int32_t ni = 0;
                        if (q < 9 * (int64_t)commits) {
                            const int32_t bi = J.changed[q / 9];
                            const int d = (int)(q % 9);
                            const int bx = bi % nbx + (d % 3) - 1, by = bi / nbx + (d / 3) - 1;
                            if (bx >= 0 && by >= 0 && bx < nbx && by < nby) {
                                ni = by * nbx + bx;
                                e = atomicExch(&J.stamp[ni], stamp) != stamp && eligible(L, bx, by, nbx, nby, gv);
                                cls = 3 * (by % 3) + (bx % 3);
                            }
                        }
                        class_push_wg(e, cls, ni, l_cnt, l_base, ncnt, J.lists, capg);
                    }
                }
            }
#undef SW_SYNC
            MC_SYNC();
            sweeps = t + 1;
            if (ctl_read(ctl, CTL_NCHG + par) == 0) {
                converged = 1;
                break;
            }
            par ^= 1;
        }
        // skip counts: one LDS sum per workgroup, one global atomic each
        if (n_smin) atomicAdd(&s_skip[0], (unsigned long long)n_smin);
        if (n_stopo) atomicAdd(&s_skip[1], (unsigned long long)n_stopo);
        __syncthreads();
        if (tid == 0) {
            if (s_skip[0]) atomicAdd(&ctr[3], s_skip[0]);
            if (s_skip[1]) atomicAdd(&ctr[4], s_skip[1]);
            s_skip[0] = 0;
            s_skip[1] = 0;
        }
        MC_SYNC();
        if (gt == 0) {
            rapid_stage_report rp;
            rp.level = sc.level[s];
            rp.block = B;
            rp.sweeps = sweeps;
            rp.converged = converged;
            rp.active = (int64_t)ctr[0];
            rp.proposals = (int64_t)ctr[1];
            rp.commits = (int64_t)ctr[2];
            rp.skip_min = (int64_t)ctr[3];
            rp.skip_topo = (int64_t)ctr[4];
            rp.merges = 0;
            J.rep[s] = rp;
            for (int i = 0; i < 6; i++) ctr[i] = 0;
        }
    }
    if (PK)   // the statistics out in their six-word layout
        for (int64_t k = gt; k < K; k += gn) {
            int64_t r[6];
            pk_unpack(pk + 2 * k, r, sc);
            for (int q = 0; q < 6; q++) st[6 * k + q] = r[q];
        }
    if ((flags & FLAG_OUT) && s_end > 0) {
        const int B = sc.B[s_end - 1];
        const int nbx = (W + B - 1) / B;
        const int32_t *L = J.lab[(s_end - 1) & 1];
        if (!(B == 1 && L == J.out)) {
            for (int64_t i = gt; i < (int64_t)W * H; i += gn) {
                const int x = (int)(i % W), y = (int)(i / W);
                J.out[(int64_t)y * J.out_stride + x] = L[(int64_t)(y / B) * nbx + x / B];
            }
        }
    }
}
#undef MC_SYNC

// ------------------------------------------------------------ launchers

hipError_t launch_block_sums(const Job *jobs_dev, int n_jobs, int s, int B, int64_t max_nb, hipStream_t stream)
{
    int64_t blocks = (max_nb + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)blocks, (unsigned)n_jobs), dim3(256), 0, stream, jobs_dev, s,
                       B);
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

hipError_t launch_refine(const Job *jobs_dev, int n_jobs, uint32_t *queue, int wgs, const Sched &sc,
                         const LdsPlan &lp, int s_begin, int s_end, int flags, const uint32_t *lut_dev, int threads,
                         hipStream_t stream)
{
    typedef void (*Kern)(const Job *, int, uint32_t *, Sched, LdsPlan, int, int, int, const uint32_t *);
    // instantiations: where the per-superpixel state lives, gate mode, merge
    // on underflow
#define RAPID_K(sl, gm) {k_refine<sl, gm, false>, k_refine<sl, gm, true>}
    // residency 4 (packed statistics) has no merge on underflow
#define RAPID_K4(gm) {k_refine<4, gm, false>, nullptr}
    static const Kern table[5][3][2] = {
        {RAPID_K(0, GM_NONE), RAPID_K(0, GM_BITS), RAPID_K(0, GM_FUSED)},
        {RAPID_K(1, GM_NONE), RAPID_K(1, GM_BITS), RAPID_K(1, GM_FUSED)},
        {RAPID_K(2, GM_NONE), RAPID_K(2, GM_BITS), RAPID_K(2, GM_FUSED)},
        {RAPID_K(3, GM_NONE), RAPID_K(3, GM_BITS), RAPID_K(3, GM_FUSED)},
        {RAPID_K4(GM_NONE), RAPID_K4(GM_BITS), RAPID_K4(GM_FUSED)}};
#undef RAPID_K
#undef RAPID_K4
    const int gm = (flags & FLAG_GATE) ? GM_FUSED : lp.gate_words > 0 ? GM_BITS : GM_NONE;
    const Kern fn = table[lp.stats_lds][gm][sc.merge ? 1 : 0];
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lp.total);
    if (e != hipSuccess) return e;
    // the persistent launch: wgs workgroups, or (wgs == 0) as many as the
    // chip holds at once, when that is fewer than the jobs
    int grid = n_jobs;
    if (queue) {
        if (wgs <= 0) {
            // at least one workgroup per CU is resident; fewer jobs than CUs
            // never need the queue, so only larger launches ask how many fit
            int dev = 0, cus = 0;
            if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
            if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
            wgs = std::max(1, cus);
            if (n_jobs > wgs) {
                int per_cu = 0;
                if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, threads,
                                                                      lp.total)) != hipSuccess)
                    return e;
                wgs *= std::max(1, per_cu);
            }
        }
        grid = std::min(n_jobs, wgs);
        if (grid == n_jobs) queue = nullptr;   // one workgroup per job: no queue
        else if ((e = hipMemsetAsync(queue, 0, sizeof(uint32_t), stream)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(threads), lp.total, stream, jobs_dev, n_jobs, queue, sc, lp,
                       s_begin, s_end, flags, lut_dev);
    return hipGetLastError();
}

hipError_t launch_refine_mc(const Job *jobs_dev, int groups, const Sched &sc, int s_begin, int s_end, int flags,
                            const uint32_t *lut_dev, int threads, int64_t solo_max, int gate_words,
                            hipStream_t stream)
{
    Sched sc_arg = sc;
    void *args[] = {(void *)&jobs_dev, (void *)&sc_arg, (void *)&s_begin, (void *)&s_end, (void *)&flags,
                    (void *)&lut_dev, (void *)&solo_max};
    const bool pk = sc.pk_bn > 0;
    typedef void (*Kern)(const Job *, Sched, int, int, int, const uint32_t *, int64_t);
    static const Kern table[3][2] = {{k_refine_mc<GM_NONE, false>, k_refine_mc<GM_NONE, true>},
                                     {k_refine_mc<GM_BITS, false>, k_refine_mc<GM_BITS, true>},
                                     {k_refine_mc<GM_FUSED, false>, k_refine_mc<GM_FUSED, true>}};
    const int gm = (flags & FLAG_GATE) ? GM_FUSED : gate_words > 0 ? GM_BITS : GM_NONE;
    const void *fn = (const void *)table[gm][pk ? 1 : 0];
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)groups), dim3((unsigned)threads), args,
                                      4 * (size_t)gate_words, stream);
}

hipError_t max_coop_groups(int threads, int *out)
{
    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess && !coop) {
        *out = 0;   // no cooperative launches on this device: one workgroup per image
        return hipSuccess;
    }
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the instantiation that holds the most registers and LDS sets the bound
    const void *fns[4] = {(const void *)k_refine_mc<GM_BITS, false>, (const void *)k_refine_mc<GM_BITS, true>,
                          (const void *)k_refine_mc<GM_FUSED, false>, (const void *)k_refine_mc<GM_FUSED, true>};
    per_cu = 1 << 30;
    for (int i = 0; i < 4 && e == hipSuccess; i++) {
        int pc = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, fns[i], threads, 4 * MAX_GATE_WORDS);
        per_cu = std::min(per_cu, pc);
    }
    *out = e == hipSuccess ? cus * per_cu : 0;
    return e;
}

}  // namespace rapid
