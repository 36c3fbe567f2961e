// rapid_host.cpp -- host side of the C-ABI: validation, schedule, scratch
// planning, launches.  Every step of the segmentation runs in the kernels of
// rapid_kernels.hip; this file only marshals.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rapid_internal.h"
#include "rapid_state_kernels.h"

using namespace rapid;

// Launch shape of the refinement: workgroup size, statistics in LDS (when
// they fit) or in global memory, block-sum pyramid inside the launch or in
// separate launches.  The labels never depend on it.
struct LaunchShape {
    int threads = 1024;
    int stats_lds = 1;
    int pyramid = 1;
    int groups = 1;    // workgroups per job: > 1 spreads a single image over
                       // a cooperative launch (state global, pyramid apart)
    int solo = -1;     // cooperative launch: sweeps with at most this many
                       // active blocks run on one workgroup (-1: never)
    int wgs = 0;       // several jobs: workgroups of the persistent launch
                       // over the job queue (0: as many as the chip holds)
    float ms = 0.0f;   // autotuner: time of the choice
};

struct rapid_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t *lut_dev = nullptr;
    size_t lds_limit = 0;
    int threads = 1024;
    bool threads_forced = false;   // RAPID_THREADS fixes the workgroup size
    bool verbose = false;
    // autotuner: chosen shape per problem shape, optional cache file
    bool autotune = false;
    std::string cache_path, arch;
    std::map<std::string, LaunchShape> tuned;
    hipEvent_t tev[2] = {nullptr, nullptr};
    LaunchShape last;              // shape of the last refinement launch
    int last_tuned = 0;
    bool shape_forced = false;     // RAPID_SHAPE=threads,stats_lds,pyramid[,groups,solo,wgs] fixes the shape
    LaunchShape forced;
    // scratch pool for rapid_segment / rapid_segment_batch
    char *pool = nullptr;
    size_t pool_size = 0;
    Job *jobs_dev = nullptr;
    size_t jobs_cap = 0;
    Job *jobs_pinned = nullptr;
    std::vector<int32_t> order;    // the job table's order (largest job first)
    hipEvent_t jobs_copied = nullptr;
    bool timing = false;
    bool timed = false;
    bool test_abort = false;   // RAPID_CFG_TEST_ABORT: cooperative launches start aborted
    // timed calls use the event triples of a ring in turn, so that the
    // kernel durations of up to TIMING_RING calls queued back to back can be
    // read after one synchronisation; ev points at the current triple
    static constexpr int TIMING_RING = 128;
    hipEvent_t ring[TIMING_RING][3] = {};
    int ring_pos = 0;
    int64_t ring_count = 0;
    hipEvent_t *ev = ring[0];
    float *part = nullptr;   // per-wave partial gradients of the gate network
    char *scratch = nullptr; // this device's copy of the fixed scratch (rapid_segment_noalloc)
    std::mutex mu;
};

struct rapid_state {
    rapid_ctx *ctx = nullptr;
    Job job{};
    Job *job_dev = nullptr;
    int64_t *zero_dev = nullptr;   // a device 0 (row offset of the state's features)
    uint32_t *err_dev = nullptr;   // import: violation flag
    float *xbuf = nullptr;         // rapid_gate: feature rows when the caller passes none
    bool imported = false;         // statistics or labels came from rapid_state_import
    char *mem = nullptr;
    Sched sc{};
    int32_t level_first[RAPID_MAX_LEVELS + 1] = {};
    int32_t n_levels = 0;
    int32_t next_level = 0;  // -1: a failed import left the labels undefined
    int32_t map_stage = 0;   // stage whose block size the current label map uses
    int32_t W = 0, H = 0;
};

namespace {

// ------------------------------------------------------------ topology LUT

// (4,8) simple-point table of the topology term: bit m is set when a block
// whose 3x3 ring has same-label mask m may leave its label.  Ring bit r is the
// neighbour (dx, dy) in row-major order with the centre skipped.  Built with
// union-find over the ring cells.
struct UF {
    int p[8];
    UF() { for (int i = 0; i < 8; i++) p[i] = i; }
    int f(int x) { while (p[x] != x) x = p[x] = p[p[x]]; return x; }
    void u(int a, int b) { p[f(a)] = f(b); }
};

void build_simple_lut(uint32_t lut[8])
{
    static const int DX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
    static const int DY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
    std::memset(lut, 0, 8 * sizeof(uint32_t));
    for (int m = 0; m < 256; m++) {
        UF fg, bg;
        for (int a = 0; a < 8; a++)
            for (int b = a + 1; b < 8; b++) {
                int ddx = std::abs(DX[a] - DX[b]), ddy = std::abs(DY[a] - DY[b]);
                bool in_a = (m >> a) & 1, in_b = (m >> b) & 1;
                if (in_a && in_b && ddx + ddy == 1) fg.u(a, b);           // 4-adjacent
                if (!in_a && !in_b && ddx <= 1 && ddy <= 1) bg.u(a, b);   // 8-adjacent
            }
        // foreground components 4-adjacent to the centre
        int roots_fg[8], nfg = 0, nbg = 0, roots_bg[8];
        for (int a = 0; a < 8; a++) {
            bool in_a = (m >> a) & 1;
            if (in_a && (DX[a] == 0 || DY[a] == 0)) {
                int r = fg.f(a);
                bool seen = false;
                for (int q = 0; q < nfg; q++) seen |= roots_fg[q] == r;
                if (!seen) roots_fg[nfg++] = r;
            }
            if (!in_a) {
                int r = bg.f(a);
                bool seen = false;
                for (int q = 0; q < nbg; q++) seen |= roots_bg[q] == r;
                if (!seen) roots_bg[nbg++] = r;
            }
        }
        if (nfg == 1 && nbg == 1) lut[m >> 5] |= 1u << (m & 31);
    }
}

// ------------------------------------------------------------------ grid

rapid_status grid_of(int32_t W, int32_t H, int32_t K, int32_t *gx, int32_t *gy)
{
    if (W < 1 || H < 1 || K < 1) return RAPID_EINVAL;
    // gy: nearest integer to sqrt(K H / W), ties down
    int64_t lo = 0, hi = (int64_t)K * H + 1;
    while (lo + 1 < hi) {   // largest g with g^2 W <= K H
        int64_t mid = (lo + hi) / 2;
        if ((__int128)mid * mid * W <= (__int128)K * H) lo = mid; else hi = mid;
    }
    int64_t g = lo;
    if ((__int128)4 * K * H > (__int128)(2 * g + 1) * (2 * g + 1) * W) g++;
    if (g < 1) g = 1;
    int64_t q = K / g;
    if (2 * (K % g) > g) q++;
    if (q < 1) q = 1;
    *gy = (int32_t)g;
    *gx = (int32_t)q;
    return RAPID_OK;
}

// --------------------------------------------------------------- validate

rapid_status make_sched(const rapid_params *p, Sched *sc, int32_t level_first[RAPID_MAX_LEVELS + 1])
{
    if (!p) return RAPID_EINVAL;
    if (p->n_levels < 1 || p->n_levels > RAPID_MAX_LEVELS) return RAPID_EINVAL;
    std::memset(sc, 0, sizeof *sc);
    int n = 0, prev = 0;
    for (int l = 0; l < p->n_levels; l++) {
        if (p->factor[l] < 1 || p->n_stages[l] < 1 || p->n_stages[l] > RAPID_MAX_STAGES)
            return RAPID_EINVAL;
        if (level_first) level_first[l] = n;
        for (int s = 0; s < p->n_stages[l]; s++) {
            int64_t B = (int64_t)p->stages[l][s] * p->factor[l];
            if (B < 1 || B > 64) return RAPID_EINVAL;
            if (prev && (B > prev || prev % B)) return RAPID_EINVAL;
            prev = (int)B;
            sc->B[n] = (int32_t)B;
            sc->level[n] = l;
            n++;
        }
    }
    if (level_first) level_first[p->n_levels] = n;
    sc->n_stages = n;
    sc->gate_stage = n;
    if (p->gate_level >= 0 && p->gate_level < p->n_levels) {
        int first = 0;
        for (int l = 0; l < p->gate_level; l++) first += p->n_stages[l];
        sc->gate_stage = first;
    }
    if (p->frac_bits < 0 || p->frac_bits > 4 || p->max_sweeps < 1 || p->max_sweeps > (1 << 20)) return RAPID_EINVAL;
    if (p->gate_rule < RAPID_GATE_EITHER || p->gate_rule > RAPID_GATE_DIFFER) return RAPID_EINVAL;
    sc->gate_rule = p->gate_rule;
    if ((p->merge != 0 && p->merge != 1)) return RAPID_EINVAL;
    sc->merge = p->merge;
    if (p->gate_features != RAPID_FEATURES_LEARNED && p->gate_features != RAPID_FEATURES_ROI) return RAPID_EINVAL;
    sc->feat_set = p->gate_features;
    if (p->w_col < 0 || p->w_pos < 0 || p->w_bnd < 0 || p->min_size < 0 || p->max_size < 1)
        return RAPID_EINVAL;
    sc->F = p->frac_bits;
    sc->max_sweeps = p->max_sweeps;
    sc->min_size = p->min_size;
    sc->max_size = p->max_size;
    sc->w_col = p->w_col;
    sc->w_pos = p->w_pos;
    sc->w_bnd = p->w_bnd;
    return RAPID_OK;
}

// Largest intermediate magnitude of E' for blocks of size B (see
// block_energy / energy_md): every product and partial sum is bounded
// by the sum of the three weighted terms' worst cases.
__int128 energy_bound(const Sched &sc, int B, int32_t W, int32_t H)
{
    typedef __int128 i128;
    i128 m = (i128)B * B;
    i128 cmax = (i128)255 << sc.F;
    i128 dim = std::max(W, H);
    i128 mumax = (dim - 1) << sc.F;
    i128 e_col = m * 3 * cmax * cmax + ((i128)2 << sc.F) * 3 * cmax * m * 255;
    i128 e_pos = m * 2 * mumax * mumax + ((i128)2 << sc.F) * 2 * mumax * m * (dim - 1);
    i128 e_bnd = (4 * (i128)B) << (2 * sc.F);
    return sc.w_col * e_col + sc.w_pos * e_pos + sc.w_bnd * e_bnd;
}

// Per stage: can fp64 evaluate E' exactly (all intermediates < 2^53)?
void set_exactness(Sched &sc, int32_t W, int32_t H)
{
    const __int128 lim53 = (__int128)1 << 53;
    for (int s = 0; s < sc.n_stages; s++) sc.f64[s] = energy_bound(sc, sc.B[s], W, H) < lim53;
    sc.d_wc = (double)sc.w_col;
    sc.d_wp = (double)sc.w_pos;
    sc.d_wb = std::ldexp((double)sc.w_bnd, 2 * sc.F);
    sc.d_fs = std::ldexp(1.0, sc.F + 1);
    sc.d_wcfs = sc.d_wc * sc.d_fs;
    sc.d_wpfs = sc.d_wp * sc.d_fs;
}

// Worst-case |E'| of a block must stay below 2^62 so that the int64 block
// energy of the kernels is exact.
bool energy_fits(const Sched &sc, int32_t W, int32_t H)
{
    typedef __int128 i128;
    const i128 lim = (i128)1 << 62;
    i128 Bm = sc.B[0];
    i128 m = Bm * Bm;
    i128 cmax = (i128)255 << sc.F;
    i128 dim = std::max(W, H);
    i128 mumax = (dim - 1) << sc.F;
    i128 e_col = m * 3 * cmax * cmax + ((i128)2 << sc.F) * 3 * cmax * m * 255;
    i128 e_pos = m * 2 * mumax * mumax + ((i128)2 << sc.F) * 2 * mumax * m * (dim - 1);
    i128 e_bnd = (4 * Bm) << (2 * sc.F);
    if (sc.w_col > 0 && e_col > lim / sc.w_col) return false;
    if (sc.w_pos > 0 && e_pos > lim / sc.w_pos) return false;
    if (sc.w_bnd > 0 && e_bnd > lim / sc.w_bnd) return false;
    i128 tot = sc.w_col * e_col + sc.w_pos * e_pos + sc.w_bnd * e_bnd;
    return tot < lim;
}

rapid_status check_image(const rapid_image *img, bool need_labels)
{
    if (!img || !img->rgb_dev) return RAPID_EINVAL;
    if (img->W < 1 || img->H < 1 || img->W > RAPID_MAX_DIM || img->H > RAPID_MAX_DIM) return RAPID_EINVAL;
    if (img->row_stride_bytes < 3 * (int64_t)img->W) return RAPID_EINVAL;
    if (need_labels && (!img->labels_dev || img->label_stride < img->W)) return RAPID_EINVAL;
    return RAPID_OK;
}

rapid_status image_grid(const rapid_image *img, const rapid_params *p, const Sched &sc,
                        int32_t *gx, int32_t *gy)
{
    rapid_status r;
    if (p->K > 0) {
        if ((r = grid_of(img->W, img->H, p->K, gx, gy))) return r;
    } else {
        *gx = p->gx;
        *gy = p->gy;
    }
    if (*gx < 1 || *gy < 1) return RAPID_EINVAL;
    if ((int64_t)*gx * sc.B[0] > img->W || (int64_t)*gy * sc.B[0] > img->H) return RAPID_EINVAL;
    if (!energy_fits(sc, img->W, img->H)) return RAPID_EINVAL;
    return RAPID_OK;
}

// ------------------------------------------------------- scratch planning

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t bytes = 0;
    size_t off_lab[2], off_sums[MAXST], off_lists, off_props, off_changed, off_stamp;
    size_t off_stats, off_means, off_flow, off_rep;
    size_t off_fmean, off_facc, off_moved, off_moms;
    size_t off_merge[8];   // merge on: mreq mlist mbox mkey mlen mstate mpick mwin
    size_t off_ctl;
    int64_t capc = 0;
};

// moms_stage: stage whose per-block second moments the gate reads (-1: none)
Layout plan(int32_t W, int32_t H, int32_t K, const Sched &sc, int moms_stage = -1)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t n) { size_t r = o; o = align256(o + n); return r; };
    int Bmin = sc.B[sc.n_stages - 1];
    int64_t nbxF = (W + Bmin - 1) / Bmin, nbyF = (H + Bmin - 1) / Bmin;
    int64_t nbF = nbxF * nbyF;
    L.capc = ((nbxF + 2) / 3) * ((nbyF + 2) / 3);
    L.off_lab[0] = take(4 * nbF);
    L.off_lab[1] = take(4 * nbF);
    for (int s = 0; s < MAXST; s++) {
        L.off_sums[s] = (size_t)-1;
        if (s < sc.n_stages && sc.B[s] >= 2) {
            int64_t nb = (int64_t)((W + sc.B[s] - 1) / sc.B[s]) * ((H + sc.B[s] - 1) / sc.B[s]);
            L.off_sums[s] = take(8 * nb);
        }
    }
    L.off_lists = take(4 * 9 * L.capc);
    L.off_props = take(sizeof(Prop) * L.capc);
    L.off_changed = take(4 * nbF);
    L.off_stamp = take(4 * nbF);
    L.off_stats = take(8 * 6 * (size_t)K);
    L.off_means = take(4 * MN_STRIDE * (size_t)K);
    L.off_flow = take(4 * 4 * (size_t)K);
    L.off_rep = take(sizeof(rapid_stage_report) * MAXST);
    L.off_ctl = take(4 * (size_t)CTL_WORDS);
    L.off_fmean = take(4 * 3 * (size_t)K);
    L.off_facc = take(8 * FACC * (size_t)K);
    L.off_moved = take(8 * (size_t)K);
    L.off_moms = (size_t)-1;
    if (moms_stage >= 0) {
        const int B = sc.B[moms_stage];
        L.off_moms = take(12 * (size_t)((W + B - 1) / B) * ((H + B - 1) / B));
    }
    for (int i = 0; i < 8; i++) L.off_merge[i] = (size_t)-1;
    if (sc.merge) {
        const size_t Kz = (size_t)K;
        const size_t bytes[8] = {4 * ((Kz + 31) / 32), 4 * Kz, 16 * Kz, 4 * MERGE_NB * Kz,
                                 4 * MERGE_NB * Kz, 4 * Kz, 4 * Kz, 4 * Kz};
        for (int i = 0; i < 8; i++) L.off_merge[i] = take(bytes[i]);
    }
    L.bytes = o;
    return L;
}

void fill_job(Job &J, char *base, const Layout &L, const rapid_image *img, int32_t gx, int32_t gy,
              const uint8_t *gate)
{
    std::memset(&J, 0, sizeof J);
    J.rgb = img->rgb_dev;
    J.rgb_stride = img->row_stride_bytes;
    J.W = img->W;
    J.H = img->H;
    J.gx = gx;
    J.gy = gy;
    J.K = gx * gy;
    J.out = img->labels_dev;
    J.out_stride = img->label_stride;
    J.lab[0] = reinterpret_cast<int32_t *>(base + L.off_lab[0]);
    J.lab[1] = reinterpret_cast<int32_t *>(base + L.off_lab[1]);
    for (int s = 0; s < MAXST; s++)
        J.sums[s] = L.off_sums[s] == (size_t)-1 ? nullptr : reinterpret_cast<uint64_t *>(base + L.off_sums[s]);
    J.lists = reinterpret_cast<int32_t *>(base + L.off_lists);
    J.capc = L.capc;
    J.props = reinterpret_cast<Prop *>(base + L.off_props);
    J.changed = reinterpret_cast<int32_t *>(base + L.off_changed);
    J.stamp = reinterpret_cast<int32_t *>(base + L.off_stamp);
    J.stats = reinterpret_cast<int64_t *>(base + L.off_stats);
    J.means = reinterpret_cast<int32_t *>(base + L.off_means);
    J.flow = reinterpret_cast<int32_t *>(base + L.off_flow);
    J.rep = reinterpret_cast<rapid_stage_report *>(base + L.off_rep);
    J.ctl = reinterpret_cast<uint32_t *>(base + L.off_ctl);
    J.gate = gate;
    J.fmean = reinterpret_cast<int32_t *>(base + L.off_fmean);
    J.facc = reinterpret_cast<int64_t *>(base + L.off_facc);
    J.moms = L.off_moms == (size_t)-1 ? nullptr : reinterpret_cast<uint32_t *>(base + L.off_moms);
    J.moms_stage = -1;
    if (L.off_merge[0] != (size_t)-1) {
        J.mreq = reinterpret_cast<uint32_t *>(base + L.off_merge[0]);
        J.mlist = reinterpret_cast<int32_t *>(base + L.off_merge[1]);
        J.mbox = reinterpret_cast<int4 *>(base + L.off_merge[2]);
        J.mkey = reinterpret_cast<int32_t *>(base + L.off_merge[3]);
        J.mlen = reinterpret_cast<int32_t *>(base + L.off_merge[4]);
        J.mstate = reinterpret_cast<int32_t *>(base + L.off_merge[5]);
        J.mpick = reinterpret_cast<int32_t *>(base + L.off_merge[6]);
        J.mwin = reinterpret_cast<int32_t *>(base + L.off_merge[7]);
    }
}

rapid_status dev_err(hipError_t e) { return e == hipSuccess ? RAPID_OK : RAPID_EDEVICE; }

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return RAPID_EDEVICE; \
    } while (0)

// Carve the LDS of the refinement kernel: statistics first (when they fit
// with room to spare), then the class lists, proposals, the frontier visit
// bitmap and the changed list, each within a share of what remains.
// Residency of the per-superpixel state that fits LDS beside the work
// space, given the one asked for, falling back in the order 1 (statistics,
// means, flow), 4 (packed statistics and flow, where the launch allows the
// packing), 3 (means and flow), 2 (means), 0 (all in global memory).
int lds_residency(size_t limit, int32_t Kmax, bool gated, int want, bool packable)
{
    const size_t gwords = gated ? ((size_t)Kmax + 31) / 32 : 0;
    const size_t base = 48 * 1024 + 4 * gwords;
    if (want == 1 && (size_t)Kmax * LDS_PER_SP + base <= limit) return 1;
    if ((want == 1 || want == 4) && packable && (size_t)Kmax * LDS_PACKED_FLOW_PER_SP + base <= limit) return 4;
    if ((want == 1 || want == 3 || want == 4) && (size_t)Kmax * LDS_MEANS_FLOW_PER_SP + base <= limit) return 3;
    if (want >= 1 && (size_t)Kmax * LDS_MEANS_PER_SP + base <= limit) return 2;
    return 0;
}

inline int bit_length(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// Packed statistics (residency 4) for a launch that starts from the grid:
// n stays below nmax = the larger of max_size and the largest initial cell
// (the size filter never lets a superpixel grow past max_size), so the
// colour sums need 255 nmax < 2^21 and n, T_x <= nmax (W - 1) and
// T_y <= nmax (H - 1) must share 64 bits.  Sets sc.pk_bn, sc.pk_bx and
// returns true when every job allows it.
bool set_packing(Sched &sc, const Job *jobs, size_t n, int flags)
{
    sc.pk_bn = sc.pk_bx = 0;
    if (!(flags & (FLAG_INIT | FLAG_OWN_STATS)) || sc.merge) return false;
    int bn = 1, bx = 1, by = 1;
    const int B0 = sc.B[0];
    for (size_t j = 0; j < n; j++) {
        const Job &J = jobs[j];
        // the widest cell column and tallest cell row of the block-centre
        // rule (a block's cell index never decreases along an axis)
        auto widest = [B0](int64_t len, int64_t cells) {
            int64_t best = 0, run = 0, cur = -1;
            for (int64_t x0 = 0; x0 < len; x0 += B0) {
                const int64_t w = std::min<int64_t>(B0, len - x0);
                const int64_t c = ((2 * x0 + w) * cells) / (2 * len);
                if (c != cur) {
                    cur = c;
                    run = 0;
                }
                run += w;
                best = std::max(best, run);
            }
            return best;
        };
        const int64_t cell = widest(J.W, J.gx) * widest(J.H, J.gy);
        const int64_t nmax = std::max<int64_t>(sc.max_size, cell);
        if (nmax <= 0 || nmax >= ((int64_t)1 << 30) || 255 * nmax >= ((int64_t)1 << 21)) return false;
        bn = std::max(bn, bit_length((uint64_t)nmax));
        bx = std::max(bx, bit_length((uint64_t)nmax * (uint64_t)(J.W - 1)));
        by = std::max(by, bit_length((uint64_t)nmax * (uint64_t)(J.H - 1)));
    }
    if (bn + bx + by > 64) return false;
    sc.pk_bn = bn;
    sc.pk_bx = bx;
    return true;
}

LdsPlan plan_lds(size_t limit, int32_t Kmax, int64_t nbF, bool gated, int want, bool packable)
{
    LdsPlan p;
    std::memset(&p, 0, sizeof p);
    auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    size_t off = 0;
    const size_t gwords = gated ? ((size_t)Kmax + 31) / 32 : 0;   // at most MAX_GATE_WORDS (run_jobs)
    p.stats_lds = lds_residency(limit, Kmax, gated, want, packable);
    if (p.stats_lds == 1) off = a16((size_t)Kmax * LDS_PER_SP);
    else if (p.stats_lds == 4) off = a16((size_t)Kmax * LDS_PACKED_FLOW_PER_SP);
    else if (p.stats_lds == 3) off = a16((size_t)Kmax * LDS_MEANS_FLOW_PER_SP);
    else if (p.stats_lds == 2) off = a16((size_t)Kmax * LDS_MEANS_PER_SP);
    p.gate_words = (int32_t)gwords;
    p.off_gate = (uint32_t)off;
    off = a16(off + 4 * gwords);
    size_t rem = limit > off ? limit - off : 0;
    p.capl = (int)std::min<size_t>(1024, rem * 35 / 100 / (9 * 4));
    p.capp = (int)std::min<size_t>(1024, rem * 25 / 100 / sizeof(Prop));
    p.bm_words = (int)std::min<size_t>((size_t)((nbF + 31) / 32), rem * 25 / 100 / 4);
    p.off_lists = (uint32_t)off;
    off = a16(off + (size_t)9 * 4 * p.capl);
    p.off_props = (uint32_t)off;
    off = a16(off + sizeof(Prop) * p.capp);
    p.off_bm = (uint32_t)off;
    off = a16(off + 4 * (size_t)p.bm_words);
    p.off_chg = (uint32_t)off;
    size_t left = limit > off ? limit - off : 0;
    p.capx = (int)std::min<size_t>(4096, left / 4);
    off = a16(off + 4 * (size_t)p.capx);
    p.total = (uint32_t)off;
    return p;
}

// ---------------------------------------------------------- autotuner

// Problem shape: jobs, largest image and superpixel count, schedule, gate
// and merge modes, which stages run.
std::string shape_key(const std::vector<Job> &jobs, const Sched &sc, int s_begin, int s_end, int flags,
                      int32_t Kmax, bool gated)
{
    int Wm = 0, Hm = 0;
    for (const Job &J : jobs) {
        Wm = std::max(Wm, J.W);
        Hm = std::max(Hm, J.H);
    }
    std::string k = "n" + std::to_string(jobs.size()) + "_W" + std::to_string(Wm) + "_H" + std::to_string(Hm) +
                    "_K" + std::to_string(Kmax) + "_B";
    for (int s = 0; s < sc.n_stages; s++) k += (s ? "." : "") + std::to_string(sc.B[s]);
    k += "_s" + std::to_string(s_begin) + "-" + std::to_string(s_end) + "_f" + std::to_string(flags) + "_g" +
         std::to_string(gated ? 1 : 0) + "_m" + std::to_string(sc.merge) + "_r" + std::to_string(sc.gate_rule);
    return k;
}

// Cache file: one JSON object, one entry per line:
//   {"rapid_autotune": 1, "arch": "<gcnArchName>", "entries": {
//   "<key>": [threads, stats_lds, pyramid, groups, solo, ms],
//   ...
//   }}
void cache_load(rapid_ctx *ctx)
{
    if (ctx->cache_path.empty()) return;
    FILE *f = std::fopen(ctx->cache_path.c_str(), "r");
    if (!f) return;
    char line[2048];
    bool arch_ok = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strstr(line, "\"rapid_autotune\"")) {
            const char *a = std::strstr(line, "\"arch\": \"");
            arch_ok = a && std::strncmp(a + 9, ctx->arch.c_str(), ctx->arch.size()) == 0 &&
                      a[9 + ctx->arch.size()] == '"';
            continue;
        }
        if (!arch_ok) break;
        char key[1024];
        LaunchShape sh;
        // entries without the cooperative fields (one workgroup per job) are
        // read too
        const int got = std::sscanf(line, " \"%1023[^\"]\": [%d, %d, %d, %d, %d, %f]", key, &sh.threads,
                                    &sh.stats_lds, &sh.pyramid, &sh.groups, &sh.solo, &sh.ms);
        if (got != 7) {
            sh.groups = 1;
            sh.solo = -1;
            if (std::sscanf(line, " \"%1023[^\"]\": [%d, %d, %d, %f]", key, &sh.threads, &sh.stats_lds, &sh.pyramid,
                            &sh.ms) != 5)
                continue;
        }
        if (sh.threads >= 64 && sh.threads <= 1024 && sh.threads % 64 == 0 && sh.groups >= 1 && sh.groups <= 4096)
            ctx->tuned[key] = sh;
    }
    std::fclose(f);
}

void cache_save(const rapid_ctx *ctx)
{
    if (ctx->cache_path.empty()) return;
    const std::string tmp = ctx->cache_path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\"rapid_autotune\": 1, \"arch\": \"%s\", \"entries\": {\n", ctx->arch.c_str());
    size_t i = 0;
    for (const auto &e : ctx->tuned)
        std::fprintf(f, "\"%s\": [%d, %d, %d, %d, %d, %.4f]%s\n", e.first.c_str(), e.second.threads,
                     e.second.stats_lds, e.second.pyramid, e.second.groups, e.second.solo, e.second.ms,
                     ++i < ctx->tuned.size() ? "," : "");
    std::fprintf(f, "}}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), ctx->cache_path.c_str());
}

// The next event triple of the timing ring for a timed call.
void timing_next(rapid_ctx *ctx)
{
    if (ctx->ring_count > 0) ctx->ring_pos = (ctx->ring_pos + 1) % rapid_ctx::TIMING_RING;
    ctx->ring_count++;
    ctx->ev = ctx->ring[ctx->ring_pos];
}

// A cooperative launch whose grid barrier gave up left its workgroups
// early, so its labels and statistics are not the method's: wait for it
// and read its abort word (before a later launch clears it).
rapid_status coop_status(rapid_ctx *ctx, const Job &J)
{
    HIPCHK(hipStreamSynchronize(ctx->stream));
    uint32_t abort_w = 0;
    HIPCHK(hipMemcpy(&abort_w, J.ctl + CTL_ABORT, 4, hipMemcpyDeviceToHost));
    return abort_w ? RAPID_EDEVICE : RAPID_OK;
}

// Block sums (when the launch does not build the pyramid) and the
// refinement launch with shape sh; jobs are on the device already.
rapid_status launch_shape(rapid_ctx *ctx, const Job *jobs, size_t n, const Job *jobs_dev, const Sched &sc,
                          int s_begin, int s_end, int flags, int32_t Kmax, int64_t nbF_max, bool gated,
                          const LaunchShape &sh, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2)
{
    if (e0) HIPCHK(hipEventRecord(e0, ctx->stream));
    if (flags & FLAG_INIT) {
        // a cooperative launch always builds its pyramid over its grid
        if (sh.pyramid || sh.groups > 1) {
            flags |= FLAG_PYRAMID;
        } else {
            // chip-wide launches, one per stage with B >= 2
            for (int s = 0; s < sc.n_stages; s++) {
                const int B = sc.B[s];
                if (B < 2) continue;
                int64_t nb = 0;
                for (size_t j = 0; j < n; j++)
                    nb = std::max<int64_t>(nb, (int64_t)((jobs[j].W + B - 1) / B) * ((jobs[j].H + B - 1) / B));
                HIPCHK(launch_block_sums(jobs_dev, (int)n, s, B, nb, ctx->stream));
            }
        }
    }
    LdsPlan lp = plan_lds(ctx->lds_limit, Kmax, nbF_max, gated, sh.stats_lds, sc.pk_bn > 0);
    if (ctx->verbose)
        std::fprintf(stderr,
                     "rapid: threads %d, lds limit %zu, stats_lds %d, capl %d capp %d capx %d bm_words %d "
                     "gate_words %d total %u\n",
                     sh.threads, ctx->lds_limit, lp.stats_lds, lp.capl, lp.capp, lp.capx, lp.bm_words,
                     lp.gate_words, lp.total);
    if (sh.groups > 1) {
        // one image on many workgroups: its control words start at zero
        // (the test hook raises the abort word of a launch that refines
        // stages, so that every workgroup leaves at its first grid barrier)
        HIPCHK(hipMemsetAsync(jobs[0].ctl, 0, 4 * (size_t)CTL_WORDS, ctx->stream));
        if (ctx->test_abort && s_end > s_begin)
            HIPCHK(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(jobs[0].ctl + CTL_ABORT), 1, 1, ctx->stream));
        if (e1) HIPCHK(hipEventRecord(e1, ctx->stream));
        HIPCHK(launch_refine_mc(jobs_dev, sh.groups, sc, s_begin, s_end, flags, ctx->lut_dev, sh.threads,
                                sh.solo, lp.gate_words, ctx->stream));
        if (e2) HIPCHK(hipEventRecord(e2, ctx->stream));
        return RAPID_OK;
    }
    if (e1) HIPCHK(hipEventRecord(e1, ctx->stream));
    // several jobs: a persistent launch over the job queue that follows the
    // job table (a word past its last entry)
    uint32_t *queue = n > 1 ? reinterpret_cast<uint32_t *>(const_cast<Job *>(jobs_dev) + n) : nullptr;
    HIPCHK(launch_refine(jobs_dev, (int)n, queue, sh.wgs, sc, lp, s_begin, s_end, flags, ctx->lut_dev, sh.threads,
                         ctx->stream));
    if (e2) HIPCHK(hipEventRecord(e2, ctx->stream));
    return RAPID_OK;
}

// follow: when the shape of an earlier launch spread the image over many
// workgroups, this launch does too (where it may)
rapid_status run_jobs(rapid_ctx *ctx, const std::vector<Job> &jobs, const Sched &sc_in, int s_begin,
                      int s_end, int flags, int32_t Kmax, int64_t nbF_max, const LaunchShape *follow = nullptr)
{
    size_t n = jobs.size();
    Sched sc = sc_in;
    const bool packable = set_packing(sc, jobs.data(), n, flags);
    if (n > ctx->jobs_cap) {
        if (ctx->jobs_dev) {
            HIPCHK(hipStreamSynchronize(ctx->stream));
            HIPCHK(hipFree(ctx->jobs_dev));
            HIPCHK(hipHostFree(ctx->jobs_pinned));
            ctx->jobs_dev = nullptr;
            ctx->jobs_pinned = nullptr;
            ctx->jobs_cap = 0;
        }
        size_t cap = std::max<size_t>(n, 64);
        // the job table, then the work queue's counter
        if (hipMalloc(&ctx->jobs_dev, cap * sizeof(Job) + 256) != hipSuccess) return RAPID_ENOMEM;
        if (hipHostMalloc(&ctx->jobs_pinned, cap * sizeof(Job)) != hipSuccess) return RAPID_ENOMEM;
        ctx->jobs_cap = cap;
    }
    // the gate bits live in LDS during the gated stages
    bool gated = (flags & FLAG_GATE) != 0;
    if (s_end > sc.gate_stage)
        for (const Job &J : jobs) gated |= J.gate != nullptr;
    if (gated && ((int64_t)Kmax + 31) / 32 > MAX_GATE_WORDS) return RAPID_EINVAL;
    // the previous upload from the staging buffer must have completed
    HIPCHK(hipEventSynchronize(ctx->jobs_copied));
    if (n > 1) {
        // the queue hands the jobs out largest first (pixels, then index), so
        // that the last ones to start are short
        ctx->order.resize(n);
        for (size_t j = 0; j < n; j++) ctx->order[j] = (int32_t)j;
        std::stable_sort(ctx->order.begin(), ctx->order.end(), [&](int32_t x, int32_t y) {
            return (int64_t)jobs[x].W * jobs[x].H > (int64_t)jobs[y].W * jobs[y].H;
        });
        for (size_t j = 0; j < n; j++) ctx->jobs_pinned[j] = jobs[ctx->order[j]];
    } else {
        std::memcpy(ctx->jobs_pinned, jobs.data(), n * sizeof(Job));
    }
    HIPCHK(hipMemcpyAsync(ctx->jobs_dev, ctx->jobs_pinned, n * sizeof(Job), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipEventRecord(ctx->jobs_copied, ctx->stream));

    // launch shape: the tuned one for this problem shape, else the default
    // (enough jobs to fill the chip: the pyramid inside the launch)
    // a single image may spread over the workgroups of a cooperative launch
    // (no merge, not a slide tile)
    int coop_max = 0;
    if (n == 1 && !sc.merge && !jobs[0].tile) HIPCHK(max_coop_groups(1024, &coop_max));
    LaunchShape sh;
    sh.threads = ctx->threads;
    sh.stats_lds = lds_residency(ctx->lds_limit, Kmax, gated, 1, packable);
    sh.pyramid = (int)n >= PYRAMID_MIN_JOBS ? 1 : 0;
    if (coop_max > 1 && nbF_max >= ((int64_t)1 << 20) && (!ctx->threads_forced || ctx->threads == 1024)) {
        // untuned default for a single image of a million finest blocks or
        // more: the cooperative shape that measured fastest on such images
        sh.threads = 1024;
        sh.groups = std::min(64, coop_max);
        sh.solo = 16384;
    }
    const std::string key = shape_key(jobs, sc, s_begin, s_end, flags, Kmax, gated);
    auto it = ctx->tuned.find(key);
    ctx->last_tuned = 0;
    if (ctx->shape_forced) {
        sh = ctx->forced;
    } else if (follow && follow->groups > 1 && coop_max > 1) {
        sh = *follow;
    } else if (it != ctx->tuned.end()) {
        sh = it->second;
        if (ctx->threads_forced) sh.threads = ctx->threads;
    } else if (ctx->autotune && (flags & FLAG_INIT)) {
        // a call that starts from the image can be repeated: time it once
        // per candidate shape (the labels are the same for all of them)
        for (int i = 0; i < 2; i++)
            if (!ctx->tev[i]) HIPCHK(hipEventCreate(&ctx->tev[i]));
        // candidates: for a single image first the cooperative shapes (8 ..
        // 128 workgroups of 1024 lanes; more pay more for each grid barrier
        // than they gain; small sweeps on the whole grid or on one
        // workgroup), then the one-workgroup shapes, the default first
        std::vector<LaunchShape> cand;
        const int solo_all[3] = {-1, 4096, 16384};
        if (!ctx->threads_forced || ctx->threads == 1024)
            for (int g = 8; g <= std::min(coop_max, 128); g *= 2)
                for (int so = 0; so < 3; so++) {
                    LaunchShape c;
                    c.threads = 1024;
                    c.stats_lds = 0;
                    c.pyramid = 1;
                    c.groups = g;
                    c.solo = solo_all[so];
                    cand.push_back(c);
                }
        const size_t n_coop = cand.size();
        LaunchShape dflt;   // the default one-workgroup shape
        dflt.threads = ctx->threads;
        dflt.stats_lds = lds_residency(ctx->lds_limit, Kmax, gated, 1, packable);
        dflt.pyramid = (int)n >= PYRAMID_MIN_JOBS ? 1 : 0;
        cand.push_back(dflt);
        const int thr_all[3] = {256, 512, 1024};
        const int res_all[5] = {1, 4, 3, 2, 0};
        for (int t = 0; t < 3; t++) {
            if (ctx->threads_forced && thr_all[t] != ctx->threads) continue;
            for (int li = 0; li < 5; li++) {
                const int l = res_all[li];
                if (lds_residency(ctx->lds_limit, Kmax, gated, l, packable) != l) continue;   // does not fit
                for (int py = 1; py >= 0; py--) {
                    LaunchShape c;
                    c.threads = thr_all[t];
                    c.stats_lds = l;
                    c.pyramid = py;
                    if (c.threads == dflt.threads && c.stats_lds == dflt.stats_lds && c.pyramid == dflt.pyramid)
                        continue;
                    cand.push_back(c);
                }
            }
        }
        LaunchShape best;
        best.ms = -1.0f;
        for (size_t ci = 0; ci < cand.size(); ci++) {
            LaunchShape c = cand[ci];
            // the faster of two runs (the first of a shape may pay for cold
            // caches and code loading)
            bool aborted = false;
            for (int rep = 0; rep < 2 && !aborted; rep++) {
                rapid_status r = launch_shape(ctx, jobs.data(), n, ctx->jobs_dev, sc, s_begin, s_end, flags, Kmax,
                                              nbF_max, gated, c, ctx->tev[0], nullptr, ctx->tev[1]);
                if (r) return r;
                HIPCHK(hipEventSynchronize(ctx->tev[1]));
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, ctx->tev[0], ctx->tev[1]));
                c.ms = rep == 0 ? ms : std::min(c.ms, ms);
                // an aborted cooperative candidate is not a shape that works
                if (c.groups > 1) {
                    r = coop_status(ctx, jobs[0]);
                    if (r == RAPID_EDEVICE) aborted = true;
                    else if (r) return r;
                }
            }
            if (aborted) continue;
            if (best.ms < 0.0f || c.ms < best.ms) best = c;
            // a default one-workgroup launch more than twice as slow as the
            // best cooperative one: the other one-workgroup shapes (which
            // differ from it by far less) are not timed
            if (ci == n_coop && n_coop > 0 && c.ms > 2.0f * best.ms) break;
        }
        if (best.ms < 0.0f) return RAPID_EDEVICE;   // every candidate aborted
        sh = best;
        ctx->tuned[key] = best;
        ctx->last_tuned = 1;
        cache_save(ctx);
        if (ctx->verbose)
            std::fprintf(stderr, "rapid: tuned %s -> threads %d stats_lds %d pyramid %d groups %d solo %d (%.3f ms)\n",
                         key.c_str(), best.threads, best.stats_lds, best.pyramid, best.groups, best.solo, best.ms);
    }
    if (sh.groups > 1) {
        // the cooperative shape where this call allows it (state global,
        // pyramid inside the launch), else one workgroup per job
        sh.groups = std::min(sh.groups, coop_max);
        if (sh.groups > 1) {
            sh.stats_lds = 0;
            sh.pyramid = 1;
        } else {
            sh.groups = 1;
        }
    }
    sh.stats_lds = lds_residency(ctx->lds_limit, Kmax, gated, sh.stats_lds, packable);
    ctx->last = sh;
    if (ctx->timing) timing_next(ctx);
    rapid_status r = launch_shape(ctx, jobs.data(), n, ctx->jobs_dev, sc, s_begin, s_end, flags, Kmax, nbF_max,
                                  gated, sh,
                                  ctx->timing ? ctx->ev[0] : nullptr, ctx->timing ? ctx->ev[1] : nullptr,
                                  ctx->timing ? ctx->ev[2] : nullptr);
    if (r) return r;
    if (ctx->timing) ctx->timed = true;
    // a cooperative launch returns only once it is known not to have
    // aborted, reports asked for or not
    if (sh.groups > 1) return coop_status(ctx, jobs[0]);
    return RAPID_OK;
}

rapid_status fetch_reports(rapid_ctx *ctx, const std::vector<Job> &jobs, const Sched &sc, int s_begin,
                           int s_end, rapid_report *reports)
{
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->last.groups > 1 && jobs.size() == 1) {
        // a cooperative launch whose grid barrier gave up left its workgroups
        // early: its labels are not the method's
        uint32_t abort_w = 0;
        HIPCHK(hipMemcpy(&abort_w, jobs[0].ctl + CTL_ABORT, 4, hipMemcpyDeviceToHost));
        if (abort_w) return RAPID_EDEVICE;
    }
    for (size_t j = 0; j < jobs.size(); j++) {
        rapid_report &R = reports[j];
        std::memset(&R, 0, sizeof R);
        R.K = jobs[j].K;
        R.n_stages = s_end - s_begin;
        if (s_end > s_begin)
            HIPCHK(hipMemcpy(R.stage, jobs[j].rep + s_begin, sizeof(rapid_stage_report) * (s_end - s_begin),
                             hipMemcpyDeviceToHost));
    }
    (void)sc;
    return RAPID_OK;
}

}  // namespace

// ================================================================= C-ABI

extern "C" {

const char *rapid_status_str(rapid_status s)
{
    switch (s) {
    case RAPID_OK: return "ok";
    case RAPID_EINVAL: return "invalid argument";
    case RAPID_ENOMEM: return "out of memory";
    case RAPID_EDEVICE: return "device error";
    case RAPID_ESTATE: return "state used out of order";
    case RAPID_EGATE: return "gate model unusable";
    }
    return "unknown status";
}

rapid_status rapid_grid(int32_t W, int32_t H, int32_t K, int32_t *gx, int32_t *gy)
{
    if (!gx || !gy) return RAPID_EINVAL;
    return grid_of(W, H, K, gx, gy);
}

// Host-only helpers (no device needed): the topology table and the
// parameter check, exposed for tests of the host logic.
rapid_status rapid_simple_lut(uint32_t out[8])
{
    if (!out) return RAPID_EINVAL;
    build_simple_lut(out);
    return RAPID_OK;
}

rapid_status rapid_check_params(int32_t W, int32_t H, const rapid_params *params, int32_t *K_out)
{
    Sched sc;
    rapid_status r = make_sched(params, &sc, nullptr);
    if (r) return r;
    rapid_image img{};
    img.rgb_dev = reinterpret_cast<const uint8_t *>(1);
    img.W = W;
    img.H = H;
    img.row_stride_bytes = 3 * (int64_t)W;
    if ((r = check_image(&img, false))) return r;
    int32_t gx, gy;
    if ((r = image_grid(&img, params, sc, &gx, &gy))) return r;
    if (K_out) *K_out = gx * gy;
    return RAPID_OK;
}

rapid_status rapid_init(const rapid_config *cfg, rapid_ctx **out)
{
    if (!cfg || !out || cfg->abi_version != RAPID_ABI_VERSION) return RAPID_EINVAL;
    rapid_ctx *ctx = new (std::nothrow) rapid_ctx();
    if (!ctx) return RAPID_ENOMEM;
    ctx->device = cfg->device;
    ctx->stream = reinterpret_cast<hipStream_t>(cfg->hip_stream);
    if (hipSetDevice(ctx->device) != hipSuccess) { delete ctx; return RAPID_EDEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) { delete ctx; return RAPID_EDEVICE; }
    // leave room for the kernel's static LDS
    size_t lim = prop.sharedMemPerBlock;
    ctx->lds_limit = lim > 1024 ? lim - 1024 : 0;
    ctx->verbose = std::getenv("RAPID_VERBOSE") != nullptr;
    if (const char *t = std::getenv("RAPID_THREADS")) {
        int v = std::atoi(t);
        if (v >= 64 && v <= 1024 && v % 64 == 0) {
            ctx->threads = v;
            ctx->threads_forced = true;
        }
    }
    if (const char *t = std::getenv("RAPID_SHAPE")) {
        LaunchShape f;
        const int got = std::sscanf(t, "%d,%d,%d,%d,%d,%d", &f.threads, &f.stats_lds, &f.pyramid, &f.groups, &f.solo,
                                    &f.wgs);
        if (got >= 3 && f.threads >= 64 && f.threads <= 1024 && f.threads % 64 == 0 && f.groups >= 1 &&
            f.groups <= 4096 && f.wgs >= 0) {
            ctx->forced = f;
            ctx->shape_forced = true;
        }
    }
    ctx->timing = (cfg->flags & RAPID_CFG_TIMING) != 0;
    ctx->test_abort = (cfg->flags & RAPID_CFG_TEST_ABORT) != 0;
    ctx->autotune = (cfg->flags & RAPID_CFG_AUTOTUNE) != 0;
    ctx->arch = prop.gcnArchName;
    if (cfg->autotune_cache) {
        ctx->cache_path = cfg->autotune_cache;
        cache_load(ctx);
    }
    if (ctx->timing)
        for (int j = 0; j < rapid_ctx::TIMING_RING; j++)
            for (int i = 0; i < 3; i++)
                if (hipEventCreate(&ctx->ring[j][i]) != hipSuccess) {
                    rapid_destroy(ctx);
                    return RAPID_EDEVICE;
                }
    uint32_t lut[8];
    build_simple_lut(lut);
    if (hipMalloc(&ctx->lut_dev, sizeof lut) != hipSuccess) { delete ctx; return RAPID_ENOMEM; }
    if (hipMemcpy(ctx->lut_dev, lut, sizeof lut, hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->jobs_copied, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(ctx->lut_dev);
        delete ctx;
        return RAPID_EDEVICE;
    }
    // the fixed scratch of rapid_segment_noalloc on this device (its address
    // only; a failed lookup leaves that entry point unusable, not the others)
    if (noalloc_scratch(ctx->device, &ctx->scratch) != hipSuccess) ctx->scratch = nullptr;
    *out = ctx;
    return RAPID_OK;
}

void rapid_destroy(rapid_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->lut_dev);
    (void)hipFree(ctx->pool);
    (void)hipFree(ctx->jobs_dev);
    (void)hipFree(ctx->part);
    if (ctx->jobs_pinned) (void)hipHostFree(ctx->jobs_pinned);
    if (ctx->jobs_copied) (void)hipEventDestroy(ctx->jobs_copied);
    for (int j = 0; j < rapid_ctx::TIMING_RING; j++)
        for (int i = 0; i < 3; i++)
            if (ctx->ring[j][i]) (void)hipEventDestroy(ctx->ring[j][i]);
    for (int i = 0; i < 2; i++)
        if (ctx->tev[i]) (void)hipEventDestroy(ctx->tev[i]);
    delete ctx;
}

rapid_status rapid_last_timings(rapid_ctx *ctx, rapid_timings *out)
{
    if (!ctx || !out) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (!ctx->timing || !ctx->timed) return RAPID_ESTATE;
    HIPCHK(hipEventSynchronize(ctx->ev[2]));
    HIPCHK(hipEventElapsedTime(&out->block_sums_ms, ctx->ev[0], ctx->ev[1]));
    HIPCHK(hipEventElapsedTime(&out->refine_ms, ctx->ev[1], ctx->ev[2]));
    out->threads = ctx->last.threads;
    out->stats_lds = ctx->last.stats_lds;
    out->pyramid = ctx->last.pyramid;
    out->tuned = ctx->last_tuned;
    out->workgroups = ctx->last.groups;
    return RAPID_OK;
}

rapid_status rapid_timing_history(rapid_ctx *ctx, float *refine_ms, int32_t max_n, int32_t *n_out)
{
    if (!ctx || !refine_ms || max_n < 0 || !n_out) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (!ctx->timing || !ctx->timed) return RAPID_ESTATE;
    const int64_t n = std::min<int64_t>({(int64_t)max_n, ctx->ring_count, (int64_t)rapid_ctx::TIMING_RING});
    HIPCHK(hipEventSynchronize(ctx->ev[2]));
    for (int64_t i = 0; i < n; i++) {
        const int slot = (int)((ctx->ring_pos - (n - 1 - i) + rapid_ctx::TIMING_RING) % rapid_ctx::TIMING_RING);
        HIPCHK(hipEventElapsedTime(&refine_ms[i], ctx->ring[slot][1], ctx->ring[slot][2]));
    }
    *n_out = (int32_t)n;
    return RAPID_OK;
}

}  // extern "C"

namespace {

// A batch of images laid out in the context's scratch pool: per image its
// Job scratch, then (for the gate) the feature rows and the gate bits of
// all superpixels, image after image.
struct Batch {
    std::vector<Job> jobs;
    std::vector<int64_t> xoff;
    Sched sc;
    int32_t Kmax = 0;
    int64_t Ktot = 0, nbF_max = 0;
    int64_t max_nb[MAXST] = {};
    float *X = nullptr;
    uint8_t *gates = nullptr;
    int64_t *xoff_dev = nullptr;   // gated: feature row offset of each image
};

struct TileInfo {
    int32_t gx, gy, core_x0, core_y0, core_w, core_h;
    int64_t gid_x0, gid_y0, gid_w;
};

rapid_status prepare_batch(rapid_ctx *ctx, const rapid_image *imgs, int32_t n, const rapid_params *params,
                           const uint8_t *gate_dev, bool gated, Batch &b,
                           const TileInfo *tiles = nullptr)
{
    rapid_status r = make_sched(params, &b.sc, nullptr);
    if (r) return r;
    Sched &sc = b.sc;
    if (gated) {
        if (params->gate_level < 1 || params->gate_level >= params->n_levels) return RAPID_EINVAL;
    } else if (!gate_dev) {
        sc.gate_stage = sc.n_stages;
    }
    std::vector<Layout> lay(n);
    std::vector<int32_t> gxs(n), gys(n);
    size_t total = 0;
    int32_t Wmax = 0, Hmax = 0;
    b.xoff.assign(n, 0);
    for (int i = 0; i < n; i++) {
        if ((r = check_image(&imgs[i], true))) return r;
        if (tiles) {
            rapid_params pt = *params;
            pt.K = 0;
            pt.gx = tiles[i].gx;
            pt.gy = tiles[i].gy;
            if ((r = image_grid(&imgs[i], &pt, sc, &gxs[i], &gys[i]))) return r;
        } else if ((r = image_grid(&imgs[i], params, sc, &gxs[i], &gys[i]))) {
            return r;
        }
        // the gate's features read second moments of the stage before it
        const int ms = (gated && sc.B[sc.gate_stage - 1] >= 2) ? sc.gate_stage - 1 : -1;
        lay[i] = plan(imgs[i].W, imgs[i].H, gxs[i] * gys[i], sc, ms);
        total += lay[i].bytes;
        b.Kmax = std::max(b.Kmax, gxs[i] * gys[i]);
        b.xoff[i] = b.Ktot;
        b.Ktot += gxs[i] * gys[i];
        for (int s = 0; s < sc.n_stages; s++) {
            int64_t nb = (int64_t)((imgs[i].W + sc.B[s] - 1) / sc.B[s]) * ((imgs[i].H + sc.B[s] - 1) / sc.B[s]);
            b.max_nb[s] = std::max(b.max_nb[s], nb);
        }
        b.nbF_max = std::max(b.nbF_max, b.max_nb[sc.n_stages - 1]);
        Wmax = std::max(Wmax, imgs[i].W);
        Hmax = std::max(Hmax, imgs[i].H);
    }
    size_t off_x = total, off_g = 0, off_xo = 0;
    if (gated) {
        off_x = align256(total);
        off_g = align256(off_x + 4 * 16 * (size_t)b.Ktot);
        off_xo = align256(off_g + (size_t)b.Ktot);
        total = align256(off_xo + 8 * (size_t)n);
    }
    if (total > ctx->pool_size) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (ctx->pool) HIPCHK(hipFree(ctx->pool));
        ctx->pool = nullptr;
        ctx->pool_size = 0;
        if (hipMalloc(&ctx->pool, total) != hipSuccess) return RAPID_ENOMEM;
        ctx->pool_size = total;
    }
    b.jobs.resize(n);
    size_t off = 0;
    for (int i = 0; i < n; i++) {
        fill_job(b.jobs[i], ctx->pool + off, lay[i], &imgs[i], gxs[i], gys[i], gate_dev);
        if (gated) b.jobs[i].moved = reinterpret_cast<int64_t *>(ctx->pool + off + lay[i].off_moved);
        off += lay[i].bytes;
        if (tiles) {
            Job &J = b.jobs[i];
            J.tile = 1;
            J.core_x0 = tiles[i].core_x0;
            J.core_y0 = tiles[i].core_y0;
            J.core_w = tiles[i].core_w;
            J.core_h = tiles[i].core_h;
            J.gid_x0 = tiles[i].gid_x0;
            J.gid_y0 = tiles[i].gid_y0;
            J.gid_w = tiles[i].gid_w;
        } else if (sc.B[sc.n_stages - 1] == 1 && imgs[i].label_stride == imgs[i].W) {
            // a final stage of single pixels writes its label map straight
            // into the caller's contiguous label buffer
            b.jobs[i].lab[(sc.n_stages - 1) & 1] = imgs[i].labels_dev;
        }
    }
    if (gated) {
        b.X = reinterpret_cast<float *>(ctx->pool + off_x);
        b.gates = reinterpret_cast<uint8_t *>(ctx->pool + off_g);
        b.xoff_dev = reinterpret_cast<int64_t *>(ctx->pool + off_xo);
        // the gate is evaluated inside the refinement launch (FLAG_GATE),
        // which also clears the moved counters
        for (int i = 0; i < n; i++) {
            Job &J = b.jobs[i];
            J.xrow = b.X + 16 * b.xoff[i];
            J.gate_out = b.gates + b.xoff[i];
            J.gate = J.gate_out;
            if (J.moms) J.moms_stage = sc.gate_stage - 1;
        }
    }
    set_exactness(sc, Wmax, Hmax);
    return RAPID_OK;
}

// The gate model's weights: 1 when every bf16 weight is finite, 0 when one
// has an all-ones exponent (Inf or NaN), -1 when they could not be read.
int model_check(rapid_ctx *ctx, const uint16_t *w_dev)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return -1;
    std::vector<uint16_t> h(MLP_PARAMS);
    if (hipMemcpyAsync(h.data(), w_dev, 2 * MLP_PARAMS, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess) return -1;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return -1;
    for (uint16_t v : h)
        if ((v & 0x7F80) == 0x7F80) return 0;
    return 1;
}

}  // namespace

extern "C" {

static rapid_status segment_impl(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                                 const rapid_params *params, const uint8_t *gate_dev,
                                 rapid_report *reports, const TileInfo *tiles = nullptr)
{
    if (!ctx || !imgs || n < 1 || !params) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    Batch b;
    rapid_status r = prepare_batch(ctx, imgs, n, params, gate_dev, false, b, tiles);
    if (r) return r;
    if ((r = run_jobs(ctx, b.jobs, b.sc, 0, b.sc.n_stages, FLAG_INIT | FLAG_OUT, b.Kmax, b.nbF_max)))
        return r;
    if (reports) return fetch_reports(ctx, b.jobs, b.sc, 0, b.sc.n_stages, reports);
    return RAPID_OK;
}

rapid_status rapid_segment(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                           const uint8_t *gate_dev, rapid_report *report)
{
    return segment_impl(ctx, img, 1, params, gate_dev, report);
}

rapid_status rapid_segment_batch(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                                 const rapid_params *params, rapid_report *reports)
{
    return segment_impl(ctx, imgs, n, params, nullptr, reports);
}

rapid_status rapid_segment_noalloc(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                                   const uint8_t *gate_dev, rapid_report *report)
{
    if (!ctx || !img || !params) return RAPID_EINVAL;
    rapid_status r;
    if ((r = check_image(img, true))) return r;
    Sched sc;
    if ((r = make_sched(params, &sc, nullptr))) return r;
    if (!gate_dev) sc.gate_stage = sc.n_stages;
    int32_t gx, gy;
    if ((r = image_grid(img, params, sc, &gx, &gy))) return r;
    const int32_t K = gx * gy;
    const bool gated = gate_dev != nullptr && sc.gate_stage < sc.n_stages;
    if (gated && ((int64_t)K + 31) / 32 > MAX_GATE_WORDS) return RAPID_EINVAL;
    const Layout L = plan(img->W, img->H, K, sc);
    if (L.bytes > NOALLOC_SCRATCH_BYTES - NOALLOC_JOB_BYTES) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (!ctx->scratch) return RAPID_EDEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    Job J;
    fill_job(J, ctx->scratch + NOALLOC_JOB_BYTES, L, img, gx, gy, gate_dev);
    if (sc.B[sc.n_stages - 1] == 1 && img->label_stride == img->W) J.lab[(sc.n_stages - 1) & 1] = img->labels_dev;
    set_exactness(sc, img->W, img->H);
    Job *jd = reinterpret_cast<Job *>(ctx->scratch);
    HIPCHK(launch_store_job(J, jd, ctx->stream));
    // the default one-workgroup shape; the block sums in their own launches
    LaunchShape sh;
    sh.threads = ctx->threads;
    const bool packable = set_packing(sc, &J, 1, FLAG_INIT);
    sh.stats_lds = lds_residency(ctx->lds_limit, K, gated, 1, packable);
    sh.pyramid = 0;
    sh.groups = 1;
    const int Bf = sc.B[sc.n_stages - 1];
    const int64_t nbF = (int64_t)((img->W + Bf - 1) / Bf) * ((img->H + Bf - 1) / Bf);
    ctx->last = sh;
    ctx->last_tuned = 0;
    if (ctx->timing) timing_next(ctx);
    if ((r = launch_shape(ctx, &J, 1, jd, sc, 0, sc.n_stages, FLAG_INIT | FLAG_OUT, K, nbF, gated, sh,
                          ctx->timing ? ctx->ev[0] : nullptr, ctx->timing ? ctx->ev[1] : nullptr,
                          ctx->timing ? ctx->ev[2] : nullptr)))
        return r;
    if (ctx->timing) ctx->timed = true;
    if (report) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        std::memset(report, 0, sizeof *report);
        report->K = K;
        report->n_stages = sc.n_stages;
        HIPCHK(hipMemcpy(report->stage, J.rep, sizeof(rapid_stage_report) * sc.n_stages, hipMemcpyDeviceToHost));
    }
    return RAPID_OK;
}

static rapid_status gated_impl(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                               const rapid_params *params, const rapid_gate_model *model,
                               float *features_dev, uint8_t *gate_dev, rapid_report *reports,
                               const TileInfo *tiles = nullptr)
{
    if (!ctx || !imgs || n < 1 || !params || !model || !model->w_bf16_dev) return RAPID_EINVAL;
    const int mc = model_check(ctx, model->w_bf16_dev);
    if (mc < 0) return RAPID_EDEVICE;
    if (mc == 0) {
        rapid_status r = segment_impl(ctx, imgs, n, params, nullptr, reports, tiles);
        return r ? r : RAPID_EGATE;
    }
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    Batch b;
    rapid_status r = prepare_batch(ctx, imgs, n, params, nullptr, true, b, tiles);
    if (r) return r;
    b.sc.mlp_w = model->w_bf16_dev;
    b.sc.mlp_thresh = model->thresh;
    // one launch: the levels before the gate, then the features of the
    // superpixels and the network's decision (Eq. (6)), then the finer levels
    // under the gate (Eq. (7)); a single image may spread over the workgroups
    // of a cooperative launch, which runs the gate point across them
    if ((r = run_jobs(ctx, b.jobs, b.sc, 0, b.sc.n_stages, FLAG_INIT | FLAG_OUT | FLAG_GATE, b.Kmax, b.nbF_max)))
        return r;
    if (features_dev)
        HIPCHK(hipMemcpyAsync(features_dev, b.X, 4 * 16 * (size_t)b.Ktot, hipMemcpyDeviceToDevice, ctx->stream));
    if (gate_dev)
        HIPCHK(hipMemcpyAsync(gate_dev, b.gates, (size_t)b.Ktot, hipMemcpyDeviceToDevice, ctx->stream));
    if (reports) {
        // one report per image over all stages
        HIPCHK(hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < n; i++) {
            rapid_report &R = reports[i];
            std::memset(&R, 0, sizeof R);
            R.K = b.jobs[i].K;
            R.n_stages = b.sc.n_stages;
            HIPCHK(hipMemcpy(R.stage, b.jobs[i].rep, sizeof(rapid_stage_report) * b.sc.n_stages,
                             hipMemcpyDeviceToHost));
        }
    }
    return RAPID_OK;
}

rapid_status rapid_segment_gated(rapid_ctx *ctx, const rapid_image *imgs, int32_t n,
                                 const rapid_params *params, const rapid_gate_model *model,
                                 float *features_dev, uint8_t *gate_dev, rapid_report *reports)
{
    return gated_impl(ctx, imgs, n, params, model, features_dev, gate_dev, reports);
}

rapid_status rapid_slide_tiles(const rapid_slide *sl, int32_t *n_tiles)
{
    if (!sl || !n_tiles) return RAPID_EINVAL;
    if (sl->W < 1 || sl->H < 1 || sl->tile < 1 || sl->halo < 0 || sl->cell < 1) return RAPID_EINVAL;
    if (sl->tile % sl->cell || sl->halo % sl->cell) return RAPID_EINVAL;
    if (sl->tile + 2 * (int64_t)sl->halo > RAPID_MAX_DIM) return RAPID_EINVAL;
    int64_t nt = ((sl->W + sl->tile - 1) / sl->tile) * ((sl->H + sl->tile - 1) / sl->tile);
    if (nt > (1 << 20)) return RAPID_EINVAL;
    *n_tiles = (int32_t)nt;
    return RAPID_OK;
}

static rapid_status slide_impl(rapid_ctx *ctx, const rapid_slide *sl, const rapid_params *params,
                               const rapid_gate_model *model, float *features_dev, uint8_t *gate_dev,
                               rapid_report *reports)
{
    int32_t nt;
    rapid_status r = rapid_slide_tiles(sl, &nt);
    if (r) return r;
    if (!ctx || !params || !sl->rgb_dev || !sl->labels_dev || sl->row_stride_bytes < 3 * sl->W ||
        sl->label_stride < sl->W)
        return RAPID_EINVAL;
    const int64_t T = sl->tile, h = sl->halo, c = sl->cell;
    const int64_t ntx = (sl->W + T - 1) / T;
    const int64_t gid_w = (sl->W + c - 1) / c;
    std::vector<rapid_image> imgs(nt);
    std::vector<TileInfo> info(nt);
    for (int32_t t = 0; t < nt; t++) {
        const int64_t tx = t % ntx, ty = t / ntx;
        const int64_t cx0 = tx * T, cy0 = ty * T;
        const int64_t cx1 = std::min<int64_t>(cx0 + T, sl->W), cy1 = std::min<int64_t>(cy0 + T, sl->H);
        const int64_t ex0 = std::max<int64_t>(0, cx0 - h), ey0 = std::max<int64_t>(0, cy0 - h);
        const int64_t ex1 = std::min<int64_t>(sl->W, cx1 + h), ey1 = std::min<int64_t>(sl->H, cy1 + h);
        rapid_image &im = imgs[t];
        im.rgb_dev = sl->rgb_dev + ey0 * sl->row_stride_bytes + 3 * ex0;
        im.W = (int32_t)(ex1 - ex0);
        im.H = (int32_t)(ey1 - ey0);
        im.row_stride_bytes = sl->row_stride_bytes;
        im.labels_dev = sl->labels_dev + ey0 * sl->label_stride + ex0;
        im.label_stride = sl->label_stride;
        TileInfo &ti = info[t];
        // cells of the slide-wide grid (the last one per axis absorbs a
        // ragged remainder narrower than a cell)
        ti.gx = (int32_t)std::max<int64_t>(1, im.W / c);
        ti.gy = (int32_t)std::max<int64_t>(1, im.H / c);
        ti.core_x0 = (int32_t)(cx0 - ex0);
        ti.core_y0 = (int32_t)(cy0 - ey0);
        ti.core_w = (int32_t)(cx1 - cx0);
        ti.core_h = (int32_t)(cy1 - cy0);
        ti.gid_x0 = ex0 / c;
        ti.gid_y0 = ey0 / c;
        ti.gid_w = gid_w;
    }
    if (model) return gated_impl(ctx, imgs.data(), nt, params, model, features_dev, gate_dev, reports, info.data());
    return segment_impl(ctx, imgs.data(), nt, params, nullptr, reports, info.data());
}

rapid_status rapid_segment_slide(rapid_ctx *ctx, const rapid_slide *sl, const rapid_params *params,
                                 const rapid_gate_model *model, rapid_report *reports)
{
    return slide_impl(ctx, sl, params, model, nullptr, nullptr, reports);
}

rapid_status rapid_segment_slide_gated(rapid_ctx *ctx, const rapid_slide *sl, const rapid_params *params,
                                       const rapid_gate_model *model, float *features_dev, uint8_t *gate_dev,
                                       rapid_report *reports)
{
    if (!model) return RAPID_EINVAL;
    return slide_impl(ctx, sl, params, model, features_dev, gate_dev, reports);
}

rapid_status rapid_state_create(rapid_ctx *ctx, const rapid_image *img, const rapid_params *params,
                                rapid_state **out)
{
    if (!ctx || !out) return RAPID_EINVAL;
    rapid_status r;
    if ((r = check_image(img, false))) return r;
    rapid_state *st = new (std::nothrow) rapid_state();
    if (!st) return RAPID_ENOMEM;
    if ((r = make_sched(params, &st->sc, st->level_first))) { delete st; return r; }
    int32_t gx, gy;
    if ((r = image_grid(img, params, st->sc, &gx, &gy))) { delete st; return r; }
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) { delete st; return RAPID_EDEVICE; }
    st->ctx = ctx;
    st->W = img->W;
    st->H = img->H;
    set_exactness(st->sc, img->W, img->H);
    Layout L = plan(img->W, img->H, gx * gy, st->sc);
    if (hipMalloc(&st->mem, L.bytes) != hipSuccess) { delete st; return RAPID_ENOMEM; }
    if (hipMalloc(&st->job_dev, sizeof(Job)) != hipSuccess) {
        (void)hipFree(st->mem);
        delete st;
        return RAPID_ENOMEM;
    }
    rapid_image im = *img;
    im.labels_dev = nullptr;
    im.label_stride = img->W;
    fill_job(st->job, st->mem, L, &im, gx, gy, nullptr);
    std::vector<Job> jobs(1, st->job);
    const int Bf = st->sc.B[st->sc.n_stages - 1];
    const int64_t nbF = (int64_t)((img->W + Bf - 1) / Bf) * ((img->H + Bf - 1) / Bf);
    // block-sum pyramid, grid labels and statistics, no stage yet
    Sched sc = st->sc;
    sc.gate_stage = sc.n_stages;
    r = run_jobs(ctx, jobs, sc, 0, 0, FLAG_INIT, gx * gy, nbF);
    if (r == RAPID_OK) r = dev_err(hipStreamSynchronize(ctx->stream));
    if (r) {
        (void)hipFree(st->mem);
        (void)hipFree(st->job_dev);
        delete st;
        return r;
    }
    st->n_levels = params->n_levels;
    st->next_level = 0;
    st->map_stage = 0;
    *out = st;
    return RAPID_OK;
}

rapid_status rapid_refine_level(rapid_ctx *ctx, rapid_state *st, int32_t level, const uint8_t *gate_dev,
                                rapid_report *report)
{
    if (!ctx || !st || st->ctx != ctx) return RAPID_EINVAL;
    if (level != st->next_level || level >= RAPID_MAX_LEVELS) return RAPID_ESTATE;
    int s0 = st->level_first[level], s1 = st->level_first[level + 1];
    if (s1 <= s0) return RAPID_ESTATE;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    Sched sc = st->sc;
    sc.gate_stage = gate_dev ? s0 : sc.n_stages;
    st->job.gate = gate_dev;
    std::vector<Job> jobs(1, st->job);
    int Bf = sc.B[sc.n_stages - 1];
    int64_t nbF = (int64_t)((st->W + Bf - 1) / Bf) * ((st->H + Bf - 1) / Bf);
    // statistics this library made from the grid keep the grid's bounds
    // (packed statistics allowed); imported ones need not
    rapid_status r = run_jobs(ctx, jobs, sc, s0, s1, st->imported ? 0 : FLAG_OWN_STATS, st->job.K, nbF);
    if (r) return r;
    st->next_level = level + 1;
    st->map_stage = s1 - 1;
    if (report) return fetch_reports(ctx, jobs, sc, s0, s1, report);
    return RAPID_OK;
}

rapid_status rapid_state_export(rapid_ctx *ctx, rapid_state *st, int32_t *labels_dev, int64_t *stats_dev)
{
    if (!ctx || !st || st->ctx != ctx) return RAPID_EINVAL;
    if (st->next_level < 0) return RAPID_ESTATE;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    if (labels_dev) {
        int s = st->map_stage;
        HIPCHK(launch_expand(st->job.lab[s & 1], st->W, st->H, st->sc.B[s], labels_dev, st->W, ctx->stream));
    }
    if (stats_dev)
        HIPCHK(hipMemcpyAsync(stats_dev, st->job.stats, sizeof(int64_t) * 6 * st->job.K,
                              hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RAPID_OK;
}

void rapid_state_destroy(rapid_state *st)
{
    if (!st) return;
    if (st->ctx) {
        (void)hipSetDevice(st->ctx->device);
        (void)hipStreamSynchronize(st->ctx->stream);
    }
    (void)hipFree(st->mem);
    (void)hipFree(st->job_dev);
    (void)hipFree(st->zero_dev);
    (void)hipFree(st->err_dev);
    (void)hipFree(st->xbuf);
    delete st;
}

rapid_status rapid_state_track(rapid_state *st, uint8_t *involved_dev, int64_t *moved_dev)
{
    if (!st) return RAPID_EINVAL;
    st->job.involved = involved_dev;
    st->job.moved = moved_dev;
    st->job.involve_stage = 0;
    return RAPID_OK;
}

rapid_status rapid_state_features(rapid_ctx *ctx, rapid_state *st, float *X_dev)
{
    if (!ctx || !st || st->ctx != ctx || !X_dev) return RAPID_EINVAL;
    if (st->next_level < 0) return RAPID_ESTATE;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    if (!st->zero_dev) {
        if (hipMalloc(&st->zero_dev, 8) != hipSuccess) return RAPID_ENOMEM;
        HIPCHK(hipMemsetAsync(st->zero_dev, 0, 8, ctx->stream));
    }
    HIPCHK(hipMemcpyAsync(st->job_dev, &st->job, sizeof(Job), hipMemcpyHostToDevice, ctx->stream));
    const int s = st->map_stage, B = st->sc.B[s];
    const int64_t nb = (int64_t)((st->W + B - 1) / B) * ((st->H + B - 1) / B);
    HIPCHK(launch_features(st->job_dev, 1, B, s & 1, st->sc.F, st->sc.feat_set, st->job.K, nb, st->zero_dev, X_dev,
                           ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RAPID_OK;
}

rapid_status rapid_state_import(rapid_ctx *ctx, rapid_state *st, int32_t next_level, const int32_t *labels_dev,
                                const int64_t *stats_dev)
{
    if (!ctx || !st || st->ctx != ctx || !labels_dev || next_level < 0 || next_level > st->n_levels)
        return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    if (!st->err_dev && hipMalloc(&st->err_dev, 4) != hipSuccess) return RAPID_ENOMEM;
    // the label map of a state that has refined next_level levels: the last
    // stage's block size (the first stage's before any level)
    const int s = next_level == 0 ? 0 : st->level_first[next_level] - 1;
    const int B = st->sc.B[s];
    int32_t *L = st->job.lab[s & 1];
    st->imported = true;
    HIPCHK(hipMemsetAsync(st->err_dev, 0, 4, ctx->stream));
    HIPCHK(launch_import_labels(labels_dev, st->W, st->W, st->H, B, st->job.K, L, st->err_dev, ctx->stream));
    if (stats_dev) {
        HIPCHK(hipMemcpyAsync(st->job.stats, stats_dev, sizeof(int64_t) * 6 * st->job.K, hipMemcpyDeviceToDevice,
                              ctx->stream));
    } else {
        HIPCHK(hipMemsetAsync(st->job.stats, 0, sizeof(int64_t) * 6 * st->job.K, ctx->stream));
        HIPCHK(launch_import_stats(st->job.rgb, st->job.rgb_stride, st->W, st->H, B, L, st->job.stats,
                                   ctx->stream));
    }
    uint32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, st->err_dev, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (err) {
        st->next_level = -1;
        return RAPID_EINVAL;
    }
    st->next_level = next_level;
    st->map_stage = s;
    return RAPID_OK;
}

rapid_status rapid_gate(rapid_ctx *ctx, rapid_state *st, const rapid_gate_model *model, float *features_dev,
                        uint8_t *gate_dev)
{
    if (!ctx || !st || st->ctx != ctx || !model || !model->w_bf16_dev || !gate_dev) return RAPID_EINVAL;
    if (st->next_level < 0) return RAPID_ESTATE;
    const int64_t K = st->job.K;
    const int mc = model_check(ctx, model->w_bf16_dev);
    if (mc < 0) return RAPID_EDEVICE;
    if (mc == 0) {
        // refuse the model: every superpixel stays marked (refine all)
        std::lock_guard<std::mutex> lock(ctx->mu);
        if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
        HIPCHK(hipMemsetAsync(gate_dev, 1, (size_t)K, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return RAPID_EGATE;
    }
    float *X = features_dev;
    if (!X) {
        std::lock_guard<std::mutex> lock(ctx->mu);
        if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
        if (!st->xbuf && hipMalloc(&st->xbuf, sizeof(float) * 16 * (size_t)K) != hipSuccess) return RAPID_ENOMEM;
        X = st->xbuf;
    }
    rapid_status r = rapid_state_features(ctx, st, X);
    if (r) return r;
    return rapid_mlp_forward(ctx, X, K, model->w_bf16_dev, model->thresh, nullptr, gate_dev);
}

rapid_status rapid_boundary_miss(rapid_ctx *ctx, const int32_t *ref_dev, const int32_t *test_dev, int32_t W,
                                 int32_t H, int64_t stride, int32_t radius, int32_t K, int32_t *miss_dev,
                                 int64_t *totals_dev)
{
    if (!ctx || !ref_dev || !test_dev || W < 1 || H < 1 || W > (1 << 22) || H > (1 << 20) || stride < W ||
        radius < 0 || radius > BOUNDARY_MISS_RMAX || (!miss_dev && !totals_dev) || (miss_dev && K < 1))
        return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    HIPCHK(launch_boundary_miss(ref_dev, test_dev, W, H, stride, radius, K, miss_dev, totals_dev, ctx->stream));
    return RAPID_OK;
}

rapid_status rapid_mlp_forward(rapid_ctx *ctx, const float *X_dev, int64_t n, const uint16_t *w_bf16_dev,
                               float thresh, float *logits_dev, uint8_t *gate_dev)
{
    if (!ctx || !X_dev || n < 0 || !w_bf16_dev || (!logits_dev && !gate_dev)) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    if (n == 0) return RAPID_OK;
    HIPCHK(launch_mlp_fwd(X_dev, n, w_bf16_dev, thresh, logits_dev, gate_dev, ctx->stream));
    return RAPID_OK;
}

}  // extern "C"

namespace {
constexpr int GRAD_WAVES = 64;

rapid_status ensure_train_scratch(rapid_ctx *ctx)
{
    if (ctx->part) return RAPID_OK;
    if (hipMalloc(&ctx->part, sizeof(float) * (size_t)GRAD_WAVES * MLP_PARAMS) != hipSuccess) return RAPID_ENOMEM;
    return RAPID_OK;
}
}  // namespace

extern "C" {

rapid_status rapid_mlp_grad(rapid_ctx *ctx, const float *X_dev, const uint8_t *t_dev, const int32_t *idx_dev,
                            int32_t nb, const uint16_t *w_bf16_dev, float *grads_dev, float *logits_dev)
{
    if (!ctx || !X_dev || !t_dev || !idx_dev || nb < 1 || !w_bf16_dev || !grads_dev) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    rapid_status r = ensure_train_scratch(ctx);
    if (r) return r;
    HIPCHK(launch_mlp_grad(X_dev, t_dev, idx_dev, nb, 1.0f / (float)nb, w_bf16_dev, ctx->part, GRAD_WAVES,
                           grads_dev, logits_dev, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RAPID_OK;
}

rapid_status rapid_gate_train(rapid_ctx *ctx, const float *X_dev, const uint8_t *t_dev, int64_t n,
                              const rapid_train_cfg *cfg, float *master_dev, uint16_t *w_bf16_dev)
{
    if (!ctx || !X_dev || !t_dev || n < 1 || n > INT32_MAX || !cfg || !master_dev || !w_bf16_dev)
        return RAPID_EINVAL;
    if (cfg->epochs < 0 || cfg->batch < 2 || cfg->batch % 2 || !(cfg->lr > 0.f)) return RAPID_EINVAL;
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return RAPID_EDEVICE;
    rapid_status r = ensure_train_scratch(ctx);
    if (r) return r;
    // class index lists (balanced batches: half positive, half negative)
    std::vector<uint8_t> t(n);
    HIPCHK(hipMemcpy(t.data(), t_dev, (size_t)n, hipMemcpyDeviceToHost));
    std::vector<int32_t> pos, neg;
    for (int64_t i = 0; i < n; i++) (t[i] ? pos : neg).push_back((int32_t)i);
    const int32_t bs = cfg->batch;
    const int64_t per_epoch = std::max<int64_t>(1, n / bs);
    float *m = nullptr, *v = nullptr, *g = nullptr;
    int32_t *idx = nullptr;
    size_t idx_n = (size_t)per_epoch * bs;
    if (hipMalloc(&m, 4 * MLP_PARAMS) != hipSuccess || hipMalloc(&v, 4 * MLP_PARAMS) != hipSuccess ||
        hipMalloc(&g, 4 * MLP_PARAMS) != hipSuccess || hipMalloc(&idx, 4 * idx_n) != hipSuccess) {
        (void)hipFree(m); (void)hipFree(v); (void)hipFree(g); (void)hipFree(idx);
        return RAPID_ENOMEM;
    }
    rapid_status rc = RAPID_OK;
    std::vector<int32_t> hidx(idx_n);
    uint64_t rs = cfg->seed * 0x9E3779B97F4A7C15ull + 1;
    auto rnd = [&rs]() {   // SplitMix64
        uint64_t z = (rs += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto shuffle = [&rnd](std::vector<int32_t> &a) {
        for (size_t i = a.size(); i > 1; i--) std::swap(a[i - 1], a[rnd() % i]);
    };
    int step = 0;
    if (hipMemsetAsync(m, 0, 4 * MLP_PARAMS, ctx->stream) != hipSuccess ||
        hipMemsetAsync(v, 0, 4 * MLP_PARAMS, ctx->stream) != hipSuccess ||
        launch_to_bf16(master_dev, w_bf16_dev, MLP_PARAMS, ctx->stream) != hipSuccess)
        rc = RAPID_EDEVICE;
    for (int ep = 0; rc == RAPID_OK && ep < cfg->epochs; ep++) {
        shuffle(pos);
        shuffle(neg);
        size_t ip = 0, in = 0;
        for (int64_t bi = 0; bi < per_epoch; bi++)
            for (int32_t j = 0; j < bs; j++) {
                const bool want_pos = (j & 1) ? !neg.empty() && pos.empty() : !pos.empty();
                std::vector<int32_t> &src = (want_pos || neg.empty()) ? pos : neg;
                size_t &cur = (&src == &pos) ? ip : in;
                if (cur == src.size()) { shuffle(src); cur = 0; }
                hidx[(size_t)bi * bs + j] = src[cur++];
            }
        if (hipStreamSynchronize(ctx->stream) != hipSuccess ||
            hipMemcpy(idx, hidx.data(), 4 * idx_n, hipMemcpyHostToDevice) != hipSuccess) {
            rc = RAPID_EDEVICE;
            break;
        }
        for (int64_t bi = 0; bi < per_epoch; bi++) {
            step++;
            if (launch_mlp_grad(X_dev, t_dev, idx + bi * bs, bs, 1.0f / (float)bs, w_bf16_dev, ctx->part,
                                GRAD_WAVES, g, nullptr, ctx->stream) != hipSuccess ||
                launch_adam(master_dev, m, v, g, w_bf16_dev, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, step,
                            ctx->stream) != hipSuccess) {
                rc = RAPID_EDEVICE;
                break;
            }
        }
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == RAPID_OK) rc = RAPID_EDEVICE;
    (void)hipFree(m); (void)hipFree(v); (void)hipFree(g); (void)hipFree(idx);
    return rc;
}

}  // extern "C"
