/* Plain single-threaded CPU oracle of the RAPID refinement sweep.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the product path never does.  It shares no code
 * with the GPU library.
 *
 * What it computes (paper: Sulimowicz & Ahmad, "RAPID: Regions-of-Interest
 * Detection in Big Histopathological Images", ICME 2017):
 *   - the CTFTPS energy of Eq. (1): colour coherence to the superpixel mean,
 *     lambda_pos times shape regularity to the centroid, the topology term,
 *     lambda_b times the boundary length of Eq. (2), and the size term;
 *   - the block move of Eq. (3): a boundary block takes the label, among its
 *     own and those of its 4-neighbours, that minimises the energy; only the
 *     energy difference that involves the block is evaluated (Sec. 3.1, last
 *     paragraph);
 *   - the size regularity of Sec. 3.1 read as a hard lower/upper bound on
 *     superpixel size (Eqs. (4)-(5) supply the upper bound); with merge on,
 *     a superpixel that a block could not leave without falling below the
 *     lower bound is instead merged into the neighbour of least merged
 *     energy (Eq. (4)) whose merged size stays within the upper bound
 *     (Eq. (5)), which lowers the label count;
 *   - the stage loop of Algorithm RAPID: grid initialisation, blocks that
 *     shrink stage by stage, a boundary set that is processed until no block
 *     changes, statistics kept up to date after moves;
 *   - the prediction gate of Eqs. (6)-(7): past the gate level only some
 *     pairs of superpixels take part: those with at least one marked side
 *     (rule "either"), with both sides marked ("both"), or whose predicted
 *     classes differ (rule "differ", the paper's boundary superpixels);
 *   - the adaptive multi-level framework of Sec. 3.2 (Eq. (8)): statistics
 *     are computed once, at the first level, and carried to finer levels.
 *     Levels are exact integer box sums of the fine image, so a level-l block
 *     of b level pixels is the fine block of b*f_l pixels and every sum is
 *     kept in fine-pixel units (Eq. (8) then holds by construction).
 *
 * Readings where the paper is silent (all integer so the result is unique):
 *   - colour is RGB, 3 channels; means are fixed point with F fraction bits,
 *     rounded half up: c = floor((2^(F+1) S + n) / (2 n));
 *   - energy weights are integers w_col, w_pos, w_bnd;
 *   - the topology term is the (4,8) simple-point test of the source label on
 *     the 3x3 ring of blocks, out-of-image counting as another label;
 *   - the boundary queue is replaced by synchronous sweeps over the 9 classes
 *     (i mod 3, j mod 3) of blocks: within a class every block proposes from
 *     the state at class start, a class-wide size filter then admits moves,
 *     and the means are refreshed after the class;  after a sweep only
 *     eligible blocks within one block of a changed block stay active;
 *   - the grid of K superpixels follows a block-centre rule (orc_grid and
 *     orc_init_labels);
 *   - merges are collected and applied in a synchronous pass too (see
 *     merge_pass): the energy of a merge is Eq. (1) after minus before, with
 *     the fixed-point means of the union.
 */
#include "rapid_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* ------------------------------------------------------------------ grid */

/* Grid of superpixels for a target count K (the regular-grid initialisation
 * of Algorithm RAPID).  gy is the integer nearest sqrt(K H / W), gx the
 * integer nearest K / gy, ties to the smaller value, both at least 1. */
int orc_grid(int32_t W, int32_t H, int32_t K, int32_t *gx, int32_t *gy)
{
    if (W < 1 || H < 1 || K < 1) return ORC_EINVAL;
    int64_t g = 0;
    /* largest g with g*g*W <= K*H */
    while ((g + 1) * (g + 1) * (int64_t)W <= (int64_t)K * H) g++;
    /* nearest: g+1 when sqrt(KH/W) > g + 1/2, i.e. 4KH > (2g+1)^2 W */
    if (4 * (int64_t)K * H > (2 * g + 1) * (2 * g + 1) * (int64_t)W) g++;
    if (g < 1) g = 1;
    int64_t q = K / g, r = K % g;
    if (2 * r > g) q++;
    if (q < 1) q = 1;
    *gy = (int32_t)g;
    *gx = (int32_t)q;
    return ORC_OK;
}

/* Initial labels: block (i, j) of size B0 (clipped to w x h at the image
 * edge) takes the cell that contains its centre,
 *   row = floor((2 j B0 + h) gy / (2 H)),  col = floor((2 i B0 + w) gx / (2 W)),
 * label = row * gx + col. */
int orc_init_labels(int32_t W, int32_t H, int32_t B0, int32_t gx, int32_t gy,
                    int32_t *labels)
{
    if (B0 < 1 || (int64_t)gx * B0 > W || (int64_t)gy * B0 > H) return ORC_EINVAL;
    for (int32_t y = 0; y < H; y++) {
        int32_t j = y / B0;
        int32_t y0 = j * B0, y1 = y0 + B0 < H ? y0 + B0 : H;
        int64_t row = ((2 * (int64_t)y0 + (y1 - y0)) * gy) / (2 * (int64_t)H);
        for (int32_t x = 0; x < W; x++) {
            int32_t i = x / B0;
            int32_t x0 = i * B0, x1 = x0 + B0 < W ? x0 + B0 : W;
            int64_t col = ((2 * (int64_t)x0 + (x1 - x0)) * gx) / (2 * (int64_t)W);
            labels[(int64_t)y * W + x] = (int32_t)(row * gx + col);
        }
    }
    return ORC_OK;
}

/* -------------------------------------------------------------- topology */

/* Ring bit order: bit r is the neighbour at (dx, dy) = RING[r], row-major
 * over the 3x3 window with the centre left out. */
static const int RING_DX[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
static const int RING_DY[8] = {-1, -1, -1, 0, 0, 1, 1, 1};

/* The topology term E_topo of Eq. (1) forbids moves that break the
 * connectivity of a superpixel.  A block may leave its label a when it is a
 * (4,8) simple point of a: the a-blocks of its 3x3 ring that are 4-connected
 * (inside the ring) to one of its four edge neighbours form exactly one
 * component, and the other ring blocks form exactly one 8-connected
 * component.  Computed here by flood fill on the 3x3 window each time. */
int orc_simple(int32_t mask)
{
    int fg[3][3], seen[3][3];
    memset(fg, 0, sizeof fg);
    for (int r = 0; r < 8; r++)
        fg[RING_DY[r] + 1][RING_DX[r] + 1] = (mask >> r) & 1;
    /* T4 of the foreground */
    memset(seen, 0, sizeof seen);
    int t4 = 0;
    for (int sy = 0; sy < 3; sy++)
        for (int sx = 0; sx < 3; sx++) {
            if ((sx == 1 && sy == 1) || !fg[sy][sx] || seen[sy][sx]) continue;
            int stk[9][2], top = 0, touches_centre = 0;
            stk[top][0] = sx; stk[top][1] = sy; top++;
            seen[sy][sx] = 1;
            while (top) {
                top--;
                int x = stk[top][0], y = stk[top][1];
                if (abs(x - 1) + abs(y - 1) == 1) touches_centre = 1;
                static const int d4[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
                for (int d = 0; d < 4; d++) {
                    int nx = x + d4[d][0], ny = y + d4[d][1];
                    if (nx < 0 || ny < 0 || nx > 2 || ny > 2) continue;
                    if (nx == 1 && ny == 1) continue;
                    if (!fg[ny][nx] || seen[ny][nx]) continue;
                    seen[ny][nx] = 1;
                    stk[top][0] = nx; stk[top][1] = ny; top++;
                }
            }
            t4 += touches_centre;
        }
    /* T8 of the background */
    memset(seen, 0, sizeof seen);
    int t8 = 0;
    for (int sy = 0; sy < 3; sy++)
        for (int sx = 0; sx < 3; sx++) {
            if ((sx == 1 && sy == 1) || fg[sy][sx] || seen[sy][sx]) continue;
            int stk[9][2], top = 0;
            stk[top][0] = sx; stk[top][1] = sy; top++;
            seen[sy][sx] = 1;
            while (top) {
                top--;
                int x = stk[top][0], y = stk[top][1];
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int nx = x + dx, ny = y + dy;
                        if (nx < 0 || ny < 0 || nx > 2 || ny > 2) continue;
                        if (nx == 1 && ny == 1) continue;
                        if (fg[ny][nx] || seen[ny][nx]) continue;
                        seen[ny][nx] = 1;
                        stk[top][0] = nx; stk[top][1] = ny; top++;
                    }
            }
            t8++;
        }
    return t4 == 1 && t8 == 1;
}

/* ------------------------------------------------------------- the state */

typedef struct {
    /* image */
    const uint8_t *rgb; int32_t W, H; int64_t stride;
    const orc_params *p;
    int32_t K;
    /* per superpixel statistics and means (Algorithm RAPID's vector S) */
    int64_t *n, *S, *T;        /* n[K], S[3K], T[2K] */
    int64_t *c, *mu;           /* c[3K], mu[2K] fixed point */
    int64_t *n0;               /* size at initialisation (size-bound invariant) */
    /* current stage */
    int32_t B, nbx, nby;
    int32_t *bl;               /* block labels (label matrix L at this stage) */
    int64_t *bs;               /* block colour sums, 3 per block */
    const uint8_t *gate;       /* NULL: every pair active */
    uint8_t *involved;         /* optional: superpixels in a proposal        */
    int64_t *moved;            /* optional: pixels moved in or out, per label */
    uint8_t *req;              /* merge on: asked to merge since the last pass */
} state;

static inline int64_t div_round(int64_t num, int64_t n, int F)
{
    /* floor((2^(F+1) num + n) / (2 n)): the mean num/n in fixed point,
     * rounded half up */
    i128 a = ((i128)num << (F + 1)) + n;
    i128 b = 2 * (i128)n;
    return (int64_t)(a / b); /* both positive */
}

static void refresh_means(state *s, int32_t k)
{
    int F = s->p->frac_bits;
    if (s->n[k] == 0) {   /* merged away: no pixels, means 0 */
        for (int ch = 0; ch < 3; ch++) s->c[3 * k + ch] = 0;
        for (int ax = 0; ax < 2; ax++) s->mu[2 * k + ax] = 0;
        return;
    }
    for (int ch = 0; ch < 3; ch++) s->c[3 * k + ch] = div_round(s->S[3 * k + ch], s->n[k], F);
    for (int ax = 0; ax < 2; ax++) s->mu[2 * k + ax] = div_round(s->T[2 * k + ax], s->n[k], F);
}

static inline const uint8_t *px(const state *s, int32_t x, int32_t y)
{
    return s->rgb + (int64_t)y * s->stride + 3 * (int64_t)x;
}

/* statistics from scratch: n, colour sums and coordinate sums of each label */
static int stats_from_labels(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                             const int32_t *lab, int32_t K,
                             int64_t *n, int64_t *S, int64_t *T)
{
    memset(n, 0, sizeof(int64_t) * K);
    memset(S, 0, sizeof(int64_t) * 3 * K);
    memset(T, 0, sizeof(int64_t) * 2 * K);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t k = lab[(int64_t)y * W + x];
            if (k < 0 || k >= K) return ORC_EINVAL;
            const uint8_t *q = rgb + (int64_t)y * stride + 3 * (int64_t)x;
            n[k]++;
            S[3 * k] += q[0]; S[3 * k + 1] += q[1]; S[3 * k + 2] += q[2];
            T[2 * k] += x; T[2 * k + 1] += y;
        }
    return ORC_OK;
}

/* block geometry at the current stage */
typedef struct { int32_t x0, y0, w, h; int64_t m, px_, py_; } blk;

static blk block_geom(const state *s, int32_t bx, int32_t by)
{
    blk b;
    b.x0 = bx * s->B; b.y0 = by * s->B;
    int32_t x1 = b.x0 + s->B < s->W ? b.x0 + s->B : s->W;
    int32_t y1 = b.y0 + s->B < s->H ? b.y0 + s->B : s->H;
    b.w = x1 - b.x0; b.h = y1 - b.y0;
    b.m = (int64_t)b.w * b.h;
    /* coordinate sums over the block: h * sum x and w * sum y */
    b.px_ = (int64_t)b.h * ((int64_t)(b.x0 + x1 - 1) * b.w / 2);
    b.py_ = (int64_t)b.w * ((int64_t)(b.y0 + y1 - 1) * b.h / 2);
    return b;
}

static inline int32_t blabel(const state *s, int32_t bx, int32_t by)
{
    if (bx < 0 || by < 0 || bx >= s->nbx || by >= s->nby) return -1;
    return s->bl[(int64_t)by * s->nbx + bx];
}

static inline int pair_active(const state *s, int32_t a, int32_t k)
{
    /* Eq. (7): which pairs of superpixels may exchange blocks under the
     * gate (no gate: every pair). */
    if (!s->gate) return 1;
    int ga = s->gate[a] != 0, gk = s->gate[k] != 0;
    switch (s->p->gate_rule) {
    case ORC_GATE_BOTH: return ga && gk;
    case ORC_GATE_DIFFER: return ga != gk;   /* classes differ across the pair */
    default: return ga || gk;
    }
}

/* A block is a boundary element (Eq. (2), or Eq. (7) under the gate) when a
 * 4-neighbour block inside the image carries another label of an active pair. */
static int eligible(const state *s, int32_t bx, int32_t by)
{
    int32_t a = blabel(s, bx, by);
    static const int d4[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    for (int d = 0; d < 4; d++) {
        int32_t k = blabel(s, bx + d4[d][0], by + d4[d][1]);
        if (k >= 0 && k != a && pair_active(s, a, k)) return 1;
    }
    return 0;
}

static int is_simple_block(const state *s, int32_t bx, int32_t by)
{
    int32_t a = blabel(s, bx, by);
    int mask = 0;
    for (int r = 0; r < 8; r++)
        if (blabel(s, bx + RING_DX[r], by + RING_DY[r]) == a) mask |= 1 << r;
    return orc_simple(mask);
}

/* E'(beta, k): the part of Eq. (1) that depends on the label k given to
 * block beta, with the means held fixed and the block-independent constant
 * terms dropped (Sec. 3.1: evaluate the energy difference only):
 *   w_col (m |c_k|^2 - 2^(F+1) <c_k, I_beta>)
 * + w_pos (m |mu_k|^2 - 2^(F+1) <mu_k, P_beta>)
 * + w_bnd 2^(2F) sum over in-image 4-neighbour blocks nu of e(beta,nu) [L(nu) != k]
 * where I_beta and P_beta are the colour and coordinate sums of the block and
 * e is the shared edge length in pixels (Eq. (2) counted over pixel pairs). */
static i128 block_energy(const state *s, int32_t bx, int32_t by, int32_t k)
{
    const orc_params *p = s->p;
    int F = p->frac_bits;
    blk b = block_geom(s, bx, by);
    const int64_t *I = s->bs + 3 * ((int64_t)by * s->nbx + bx);
    const int64_t *ck = s->c + 3 * (int64_t)k;
    const int64_t *mk = s->mu + 2 * (int64_t)k;
    i128 col = 0, dot = 0;
    for (int ch = 0; ch < 3; ch++) {
        col += (i128)ck[ch] * ck[ch];
        dot += (i128)ck[ch] * I[ch];
    }
    i128 e_col = (i128)b.m * col - ((i128)2 << F) * dot;
    i128 pos = (i128)mk[0] * mk[0] + (i128)mk[1] * mk[1];
    i128 pdot = (i128)mk[0] * b.px_ + (i128)mk[1] * b.py_;
    i128 e_pos = (i128)b.m * pos - ((i128)2 << F) * pdot;
    int64_t bnd = 0;
    int32_t nb;
    if ((nb = blabel(s, bx - 1, by)) >= 0 && nb != k) bnd += b.h;
    if ((nb = blabel(s, bx + 1, by)) >= 0 && nb != k) bnd += b.h;
    if ((nb = blabel(s, bx, by - 1)) >= 0 && nb != k) bnd += b.w;
    if ((nb = blabel(s, bx, by + 1)) >= 0 && nb != k) bnd += b.w;
    i128 e_bnd = (i128)bnd << (2 * F);
    return (i128)p->w_col * e_col + (i128)p->w_pos * e_pos + (i128)p->w_bnd * e_bnd;
}

/* Global energy of Eq. (1) at pixel level for the current labels and means,
 * with the fixed-point scaling of the means:
 *   sum_p w_col |2^F I(p) - c_{s_p}|^2 + w_pos |2^F p - mu_{s_p}|^2
 *   + w_bnd 2^(2F) #{unordered 4-adjacent pixel pairs with different labels}. */
static i128 global_energy(const state *s)
{
    const orc_params *p = s->p;
    int F = p->frac_bits;
    i128 ec = 0, ep = 0, eb = 0;
    for (int32_t y = 0; y < s->H; y++)
        for (int32_t x = 0; x < s->W; x++) {
            int32_t k = blabel(s, x / s->B, y / s->B);
            const uint8_t *q = px(s, x, y);
            for (int ch = 0; ch < 3; ch++) {
                i128 d = ((i128)q[ch] << F) - s->c[3 * (int64_t)k + ch];
                ec += d * d;
            }
            i128 dx = ((i128)x << F) - s->mu[2 * (int64_t)k];
            i128 dy = ((i128)y << F) - s->mu[2 * (int64_t)k + 1];
            ep += dx * dx + dy * dy;
            if (x + 1 < s->W && blabel(s, (x + 1) / s->B, y / s->B) != k) eb++;
            if (y + 1 < s->H && blabel(s, x / s->B, (y + 1) / s->B) != k) eb++;
        }
    return (i128)p->w_col * ec + (i128)p->w_pos * ep + (i128)p->w_bnd * (eb << (2 * F));
}

/* Debug invariants: every superpixel 4-connected and non-empty unless
 * merged away (then its sums are 0 as well), statistics equal to a
 * from-scratch recount, means equal to f(statistics). */
static int check_invariants(state *s)
{
    int32_t W = s->W, H = s->H, K = s->K;
    int64_t N = (int64_t)W * H;
    int32_t *lab = malloc(sizeof(int32_t) * N);
    int64_t *n = malloc(sizeof(int64_t) * K), *S = malloc(sizeof(int64_t) * 3 * K),
            *T = malloc(sizeof(int64_t) * 2 * K);
    uint8_t *seen = calloc(N, 1), *done = calloc(K, 1);
    int64_t *stk = malloc(sizeof(int64_t) * N);
    int ok = lab && n && S && T && seen && done && stk;
    if (ok) {
        for (int32_t y = 0; y < H; y++)
            for (int32_t x = 0; x < W; x++)
                lab[(int64_t)y * W + x] = blabel(s, x / s->B, y / s->B);
        ok = stats_from_labels(s->rgb, W, H, s->stride, lab, K, n, S, T) == ORC_OK;
    }
    for (int32_t k = 0; ok && k < K; k++) {
        if ((n[k] == 0 && !s->p->merge) || n[k] != s->n[k]) ok = 0;
        for (int ch = 0; ch < 3; ch++) if (S[3 * k + ch] != s->S[3 * k + ch]) ok = 0;
        for (int ax = 0; ax < 2; ax++) if (T[2 * k + ax] != s->T[2 * k + ax]) ok = 0;
        if (n[k] == 0) {
            for (int ch = 0; ch < 3; ch++) if (s->c[3 * k + ch] != 0) ok = 0;
            for (int ax = 0; ax < 2; ax++) if (s->mu[2 * k + ax] != 0) ok = 0;
            continue;
        }
        int F = s->p->frac_bits;
        for (int ch = 0; ch < 3; ch++) if (s->c[3 * k + ch] != div_round(S[3 * k + ch], n[k], F)) ok = 0;
        for (int ax = 0; ax < 2; ax++) if (s->mu[2 * k + ax] != div_round(T[2 * k + ax], n[k], F)) ok = 0;
    }
    /* one 4-connected component per label */
    for (int64_t i = 0; ok && i < N; i++) {
        if (seen[i]) continue;
        int32_t k = lab[i];
        if (done[k]) { ok = 0; break; }  /* second component of k */
        done[k] = 1;
        int64_t top = 0;
        stk[top++] = i; seen[i] = 1;
        while (top) {
            int64_t q = stk[--top];
            int32_t x = (int32_t)(q % W), y = (int32_t)(q / W);
            int64_t nb[4] = {x > 0 ? q - 1 : -1, x + 1 < W ? q + 1 : -1,
                             y > 0 ? q - W : -1, y + 1 < H ? q + W : -1};
            for (int d = 0; d < 4; d++)
                if (nb[d] >= 0 && !seen[nb[d]] && lab[nb[d]] == k) { seen[nb[d]] = 1; stk[top++] = nb[d]; }
        }
    }
    free(lab); free(n); free(S); free(T); free(seen); free(done); free(stk);
    return ok ? ORC_OK : ORC_EINVAR;
}

/* --------------------------------------------------------- one stage */

/* (Re)build the blocks of size B: their labels (which must agree over their
 * pixels) and their colour sums. */
static int build_blocks(state *s, int32_t B, const int32_t *lab)
{
    s->B = B;
    s->nbx = (s->W + B - 1) / B;
    s->nby = (s->H + B - 1) / B;
    int64_t nb = (int64_t)s->nbx * s->nby;
    free(s->bl); free(s->bs);
    s->bl = malloc(sizeof(int32_t) * nb);
    s->bs = calloc(3 * nb, sizeof(int64_t));
    if (!s->bl || !s->bs) return ORC_ENOMEM;
    for (int32_t by = 0; by < s->nby; by++)
        for (int32_t bx = 0; bx < s->nbx; bx++) {
            int64_t bi = (int64_t)by * s->nbx + bx;
            blk b = block_geom(s, bx, by);
            int32_t a = lab[(int64_t)b.y0 * s->W + b.x0];
            for (int32_t y = b.y0; y < b.y0 + b.h; y++)
                for (int32_t x = b.x0; x < b.x0 + b.w; x++) {
                    if (lab[(int64_t)y * s->W + x] != a) return ORC_EBLOCK;
                    const uint8_t *q = px(s, x, y);
                    s->bs[3 * bi] += q[0]; s->bs[3 * bi + 1] += q[1]; s->bs[3 * bi + 2] += q[2];
                }
            s->bl[bi] = a;
        }
    return ORC_OK;
}

static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { int32_t b, a, k; int64_t de; } proposal;

/* Proposals of one class from the state at class start (Eq. (3) with the
 * size bounds of Sec. 3.1 and the topology term).  Returns the count. */
static int64_t propose(state *s, int32_t cls, const uint8_t *active,
                       proposal *out, int64_t *skip_min, int64_t *skip_topo,
                       const int64_t *order, int64_t norder)
{
    const orc_params *p = s->p;
    int64_t np = 0;
    int32_t ci = cls % 3, cj = cls / 3;
    /* the blocks of the class: in the given order, or (order == NULL) row by
     * row stepping over the class's rows and columns */
    int64_t ncls = order ? norder
                         : (int64_t)((s->nby - cj + 2) / 3) * ((s->nbx - ci + 2) / 3);
    int32_t ncol = (s->nbx - ci + 2) / 3;
    for (int64_t oi = 0; oi < ncls; oi++) {
        int64_t bi;
        if (order) {
            bi = order[oi];
        } else {
            if (ncol <= 0) break;
            bi = (int64_t)(cj + 3 * (int32_t)(oi / ncol)) * s->nbx + ci + 3 * (int32_t)(oi % ncol);
        }
        int32_t bx = (int32_t)(bi % s->nbx), by = (int32_t)(bi / s->nbx);
        if (bx % 3 != ci || by % 3 != cj) continue;
        if (active && !active[bi]) continue;
        blk b = block_geom(s, bx, by);
        int32_t a = s->bl[bi];
        if (s->n[a] - b.m < p->min_size) {
            (*skip_min)++;
            if (s->req) s->req[a] = 1;   /* underflow: a merge candidate */
            continue;
        }
        if (!is_simple_block(s, bx, by)) { (*skip_topo)++; continue; }
        /* candidate labels: distinct in-image 4-neighbour labels != a, ascending */
        int32_t cand[4]; int nc = 0;
        int32_t nbl[4] = {blabel(s, bx - 1, by), blabel(s, bx + 1, by),
                          blabel(s, bx, by - 1), blabel(s, bx, by + 1)};
        for (int d = 0; d < 4; d++) {
            int32_t k = nbl[d];
            if (k < 0 || k == a) continue;
            int dup = 0;
            for (int e = 0; e < nc; e++) if (cand[e] == k) dup = 1;
            if (!dup) cand[nc++] = k;
        }
        for (int u = 1; u < nc; u++)       /* insertion sort, ascending */
            for (int v = u; v > 0 && cand[v - 1] > cand[v]; v--) {
                int32_t t = cand[v]; cand[v] = cand[v - 1]; cand[v - 1] = t;
            }
        int32_t best = a;
        i128 e0 = block_energy(s, bx, by, a), estar = e0;
        for (int e = 0; e < nc; e++) {
            int32_t k = cand[e];
            if (s->n[k] + b.m > p->max_size) continue;
            i128 ek = block_energy(s, bx, by, k);
            if (ek < estar) { estar = ek; best = k; }
        }
        if (best != a && pair_active(s, a, best)) {
            if (s->involved) { s->involved[a] = 1; s->involved[best] = 1; }
            out[np].b = (int32_t)bi; out[np].a = a; out[np].k = best;
            i128 de = estar - e0;   /* < 0; saturated for reporting only */
            out[np].de = de < -(i128)INT64_MAX ? -INT64_MAX : (int64_t)de;
            np++;
        }
    }
    return np;
}

/* ----------------------------------------------------- merge on underflow */

/* n |c|^2 - 2^(F+1) <c, S> over d components: the part of
 * sum_p |2^F v(p) - c|^2 over a superpixel's pixels that depends on c (the
 * sum of |2^F v(p)|^2 is the same before and after a merge and cancels). */
static i128 fit_term(const int64_t *c, const int64_t *S, int64_t n, int d, int F)
{
    i128 r = 0;
    for (int i = 0; i < d; i++)
        r += (i128)n * c[i] * c[i] - ((i128)2 << F) * c[i] * S[i];
    return r;
}

/* Energy change of Eq. (1) when superpixel m is merged into k (Eq. (4)):
 * the colour and position terms of both, re-fitted to the union's
 * fixed-point means, and the len shared boundary pixel pairs that stop
 * being boundary. */
static i128 merge_cost(const state *s, int32_t m, int32_t k, int64_t len)
{
    const orc_params *p = s->p;
    int F = p->frac_bits;
    int64_t nm = s->n[m], nk = s->n[k], nu = nm + nk;
    int64_t Su[3], cu[3], Tu[2], mu_u[2];
    for (int ch = 0; ch < 3; ch++) {
        Su[ch] = s->S[3 * (int64_t)m + ch] + s->S[3 * (int64_t)k + ch];
        cu[ch] = div_round(Su[ch], nu, F);
    }
    for (int ax = 0; ax < 2; ax++) {
        Tu[ax] = s->T[2 * (int64_t)m + ax] + s->T[2 * (int64_t)k + ax];
        mu_u[ax] = div_round(Tu[ax], nu, F);
    }
    i128 dc = fit_term(cu, Su, nu, 3, F) - fit_term(s->c + 3 * (int64_t)m, s->S + 3 * (int64_t)m, nm, 3, F) -
              fit_term(s->c + 3 * (int64_t)k, s->S + 3 * (int64_t)k, nk, 3, F);
    i128 dp = fit_term(mu_u, Tu, nu, 2, F) - fit_term(s->mu + 2 * (int64_t)m, s->T + 2 * (int64_t)m, nm, 2, F) -
              fit_term(s->mu + 2 * (int64_t)k, s->T + 2 * (int64_t)k, nk, 2, F);
    return (i128)p->w_col * dc + (i128)p->w_pos * dp - (i128)p->w_bnd * ((i128)len << (2 * F));
}

/* One merge pass (Sec. 3.1, Eqs. (4)-(5)), run when a sweep commits nothing.
 * Candidates: superpixels that asked since the last pass (a block of theirs
 * could not leave without going below min_size) and still hold fewer than
 * min_size + B^2 pixels.  Each candidate m picks, among the labels of
 * blocks 4-adjacent to its blocks (at most ORC_MERGE_MAX_NB distinct ones,
 * else no pick), those k with an active pair (m, k) and
 * n_m + n_k <= max_size, the one of least merge_cost, ties to the smaller
 * label.  A pick m -> t makes m leave when t picked nothing itself, or
 * when t picked m back and m > t (a mutual pair merges into its smaller
 * label); of the leaving superpixels that picked t, the smallest merges.
 * No target leaves and every target absorbs at most one superpixel, so the
 * applied merges are disjoint pairs whose energy changes add up.  Merged
 * blocks are marked in changed.  Returns the number of merges. */
static int64_t merge_pass(state *s, uint8_t *changed, int debug, int *rc)
{
    const orc_params *p = s->p;
    int32_t K = s->K;
    int64_t nb = (int64_t)s->nbx * s->nby, B2 = (int64_t)s->B * s->B, merged = 0;
    int32_t *key = malloc(sizeof(int32_t) * ORC_MERGE_MAX_NB * (int64_t)K);
    int64_t *len = malloc(sizeof(int64_t) * ORC_MERGE_MAX_NB * (int64_t)K);
    int32_t *cnt = malloc(sizeof(int32_t) * K), *tgt = malloc(sizeof(int32_t) * K);
    int32_t *win = malloc(sizeof(int32_t) * K);
    uint8_t *cand = calloc(K, 1), *com = calloc(K, 1);
    i128 *cost = malloc(sizeof(i128) * K);
    *rc = ORC_OK;
    if (!key || !len || !cnt || !tgt || !win || !cand || !com || !cost) { *rc = ORC_ENOMEM; goto done; }
    int any = 0;
    for (int32_t m = 0; m < K; m++) {
        cand[m] = s->req[m] && s->n[m] > 0 && s->n[m] < p->min_size + B2;
        any |= cand[m];
        cnt[m] = 0;
        tgt[m] = -1;
        win[m] = INT32_MAX;
    }
    if (!any) goto done;
    /* shared boundary length with every neighbour label, in pixel pairs */
    for (int32_t by = 0; by < s->nby; by++)
        for (int32_t bx = 0; bx < s->nbx; bx++) {
            int32_t a = blabel(s, bx, by);
            if (!cand[a]) continue;
            blk b = block_geom(s, bx, by);
            int32_t nl[4] = {blabel(s, bx - 1, by), blabel(s, bx + 1, by), blabel(s, bx, by - 1),
                             blabel(s, bx, by + 1)};
            int64_t el[4] = {b.h, b.h, b.w, b.w};
            for (int d = 0; d < 4; d++) {
                int32_t k = nl[d];
                if (k < 0 || k == a || cnt[a] > ORC_MERGE_MAX_NB) continue;
                int j = 0;
                while (j < cnt[a] && key[ORC_MERGE_MAX_NB * a + j] != k) j++;
                if (j == cnt[a]) {
                    if (cnt[a] == ORC_MERGE_MAX_NB) { cnt[a] = ORC_MERGE_MAX_NB + 1; continue; }
                    key[ORC_MERGE_MAX_NB * a + j] = k;
                    len[ORC_MERGE_MAX_NB * a + j] = 0;
                    cnt[a]++;
                }
                len[ORC_MERGE_MAX_NB * a + j] += el[d];
            }
        }
    /* picks (Eq. (4) under the size bound of Eq. (5)) */
    for (int32_t m = 0; m < K; m++) {
        if (!cand[m] || cnt[m] > ORC_MERGE_MAX_NB) continue;
        for (int j = 0; j < cnt[m]; j++) {
            int32_t k = key[ORC_MERGE_MAX_NB * m + j];
            if (s->n[m] + s->n[k] > p->max_size || !pair_active(s, m, k)) continue;
            i128 c = merge_cost(s, m, k, len[ORC_MERGE_MAX_NB * m + j]);
            if (tgt[m] < 0 || c < cost[m] || (c == cost[m] && k < tgt[m])) { tgt[m] = k; cost[m] = c; }
        }
    }
    for (int32_t m = 0; m < K; m++) {
        int32_t t = tgt[m];
        com[m] = t >= 0 && (tgt[t] < 0 || (tgt[t] == m && m > t));   /* leaves */
        if (com[m] && m < win[t]) win[t] = m;
    }
    for (int32_t m = 0; m < K; m++)
        if (com[m] && win[tgt[m]] != m) com[m] = 0;
    /* apply */
    i128 e_before = 0, de_sum = 0;
    if (debug) e_before = global_energy(s);
    for (int64_t i = 0; i < nb; i++) {
        int32_t a = s->bl[i];
        if (com[a]) { s->bl[i] = tgt[a]; changed[i] = 1; }
    }
    for (int32_t m = 0; m < K; m++) {
        if (!com[m]) continue;
        int32_t t = tgt[m];
        de_sum += cost[m];
        s->n[t] += s->n[m]; s->n[m] = 0;
        for (int ch = 0; ch < 3; ch++) {
            s->S[3 * (int64_t)t + ch] += s->S[3 * (int64_t)m + ch];
            s->S[3 * (int64_t)m + ch] = 0;
        }
        for (int ax = 0; ax < 2; ax++) {
            s->T[2 * (int64_t)t + ax] += s->T[2 * (int64_t)m + ax];
            s->T[2 * (int64_t)m + ax] = 0;
        }
        refresh_means(s, t);
        refresh_means(s, m);
        merged++;
    }
    if (debug) {
        /* the picks' energies add up to the change of Eq. (1) exactly */
        if (global_energy(s) - e_before != de_sum) { *rc = ORC_EINVAR; goto done; }
        if ((*rc = check_invariants(s)) != ORC_OK) goto done;
    }
done:
    memset(s->req, 0, K);
    free(key); free(len); free(cnt); free(tgt); free(win); free(cand); free(com); free(cost);
    return merged;
}

static int run_stage(state *s, int32_t level, int32_t B, int32_t *lab,
                     orc_stage_report *rep, int debug)
{
    const orc_params *p = s->p;
    int rc = build_blocks(s, B, lab);
    if (rc) return rc;
    int64_t nb = (int64_t)s->nbx * s->nby;
    int32_t K = s->K;
    uint8_t *active = calloc(nb, 1), *changed = calloc(nb, 1), *touched = calloc(K, 1);
    uint8_t *commit = NULL;
    int64_t cls_max = (int64_t)((s->nbx + 2) / 3) * ((s->nby + 2) / 3);
    proposal *props = malloc(sizeof(proposal) * cls_max);
    int64_t *out = calloc(K, sizeof(int64_t)), *in = calloc(K, sizeof(int64_t));
    int64_t *order = malloc(sizeof(int64_t) * nb);
    commit = malloc(cls_max);
    if (!active || !changed || !touched || !props || !out || !in || !order || !commit) {
        rc = ORC_ENOMEM; goto done;
    }
    for (int64_t i = 0; i < nb; i++) order[i] = i;
    if (p->shuffle_seed) {   /* any order within a class gives the same result */
        uint64_t st = (uint64_t)p->shuffle_seed * 0x2545F4914F6CDD1Dull + (uint64_t)B;
        for (int64_t i = nb - 1; i > 0; i--) {
            st = mix64(st);
            int64_t j = (int64_t)(st % (uint64_t)(i + 1));
            int64_t t = order[i]; order[i] = order[j]; order[j] = t;
        }
    }
    memset(rep, 0, sizeof *rep);
    rep->level = level; rep->block = B;
    for (int32_t by = 0; by < s->nby; by++)
        for (int32_t bx = 0; bx < s->nbx; bx++)
            active[(int64_t)by * s->nbx + bx] = (uint8_t)eligible(s, bx, by);

    for (int32_t t = 0; t < p->max_sweeps; t++) {
        for (int64_t i = 0; i < nb; i++) rep->active += active[i];
        memset(changed, 0, nb);
        int64_t sweep_commits = 0;
        for (int32_t cls = 0; cls < 9; cls++) {
            int64_t np = propose(s, cls, active, props, &rep->skip_min, &rep->skip_topo,
                                 p->shuffle_seed ? order : NULL, nb);
            rep->proposals += np;
            if (np == 0) continue;
            /* class-wide size filter: out/in flows of every proposal */
            for (int64_t q = 0; q < np; q++) {
                int64_t m = block_geom(s, props[q].b % s->nbx, props[q].b / s->nbx).m;
                out[props[q].a] += m;
                in[props[q].k] += m;
            }
            for (int64_t q = 0; q < np; q++)
                commit[q] = s->n[props[q].a] - out[props[q].a] >= p->min_size &&
                            s->n[props[q].k] + in[props[q].k] <= p->max_size;
            for (int64_t q = 0; q < np; q++) { out[props[q].a] = 0; in[props[q].k] = 0; }
            i128 e_before = 0, de_sum = 0;
            if (debug) e_before = global_energy(s);
            /* apply: relabel and move the block's sums from a to k */
            for (int64_t q = 0; q < np; q++) {
                if (!commit[q]) continue;
                int32_t bi = props[q].b, a = props[q].a, k = props[q].k;
                int32_t bx = bi % s->nbx, by = bi / s->nbx;
                blk b = block_geom(s, bx, by);
                s->bl[bi] = k;
                s->n[a] -= b.m; s->n[k] += b.m;
                for (int ch = 0; ch < 3; ch++) {
                    s->S[3 * (int64_t)a + ch] -= s->bs[3 * (int64_t)bi + ch];
                    s->S[3 * (int64_t)k + ch] += s->bs[3 * (int64_t)bi + ch];
                }
                s->T[2 * (int64_t)a] -= b.px_; s->T[2 * (int64_t)k] += b.px_;
                s->T[2 * (int64_t)a + 1] -= b.py_; s->T[2 * (int64_t)k + 1] += b.py_;
                changed[bi] = 1; touched[a] = 1; touched[k] = 1;
                if (s->moved) { s->moved[a] += b.m; s->moved[k] += b.m; }
                de_sum += block_energy(s, bx, by, k) - block_energy(s, bx, by, a);
                sweep_commits++;
                rep->commits++;
            }
            if (debug) {
                i128 e_after = global_energy(s);
                if (e_after - e_before != de_sum || (de_sum > 0)) { rc = ORC_EINVAR; goto done; }
            }
            /* means of every superpixel whose sums changed */
            for (int64_t q = 0; q < np; q++) {
                int32_t a = props[q].a, k = props[q].k;
                if (touched[a]) { refresh_means(s, a); touched[a] = 0; }
                if (touched[k]) { refresh_means(s, k); touched[k] = 0; }
            }
            if (debug) {
                i128 e_means = global_energy(s);
                if (e_means > e_before + de_sum) { rc = ORC_EINVAR; goto done; }
                /* an undersized superpixel cannot shrink, an oversized one
                 * cannot grow */
                for (int32_t k = 0; k < K && s->n0; k++) {
                    if (s->n[k] == 0 && p->merge) continue;   /* merged away */
                    int64_t lo = p->min_size < s->n0[k] ? p->min_size : s->n0[k];
                    int64_t hi = p->max_size > s->n0[k] ? p->max_size : s->n0[k];
                    if (s->n[k] < lo || s->n[k] > hi || s->n[k] < 1) { rc = ORC_EINVAR; goto done; }
                }
                if ((rc = check_invariants(s)) != ORC_OK) goto done;
            }
        }
        rep->sweeps = t + 1;
        if (sweep_commits == 0) {
            /* a quiet sweep: pending merges go now, and the merged blocks
             * seed the next sweep like committed moves */
            int64_t merged = 0;
            if (p->merge) {
                merged = merge_pass(s, changed, debug, &rc);
                if (rc) goto done;
            }
            if (merged == 0) { rep->converged = 1; break; }
            rep->merges += merged;
        }
        /* next active set: eligible blocks within one block of a changed one */
        memset(active, 0, nb);
        for (int32_t by = 0; by < s->nby; by++)
            for (int32_t bx = 0; bx < s->nbx; bx++) {
                if (!changed[(int64_t)by * s->nbx + bx]) continue;
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int32_t x = bx + dx, y = by + dy;
                        if (x >= 0 && y >= 0 && x < s->nbx && y < s->nby)
                            active[(int64_t)y * s->nbx + x] = 1;   /* near a change */
                    }
            }
        for (int32_t by = 0; by < s->nby; by++)
            for (int32_t bx = 0; bx < s->nbx; bx++) {
                int64_t bi = (int64_t)by * s->nbx + bx;
                if (active[bi]) active[bi] = (uint8_t)eligible(s, bx, by);
            }
    }
    if (s->req) memset(s->req, 0, K);   /* requests do not outlive the stage */
    /* write the block labels back to the pixels */
    for (int32_t y = 0; y < s->H; y++)
        for (int32_t x = 0; x < s->W; x++)
            lab[(int64_t)y * s->W + x] = s->bl[(int64_t)(y / B) * s->nbx + x / B];
done:
    free(active); free(changed); free(touched); free(props); free(out); free(in);
    free(order); free(commit);
    return rc;
}

/* ------------------------------------------------------------ driver */

static int check_params(const orc_params *p, int32_t W, int32_t H)
{
    if (W < 1 || H < 1 || W > 8192 || H > 8192) return ORC_EINVAL;
    if (p->n_levels < 1 || p->n_levels > ORC_MAX_LEVELS) return ORC_EINVAL;
    if (p->frac_bits < 0 || p->frac_bits > 8 || p->max_sweeps < 1) return ORC_EINVAL;
    if (p->gate_rule < ORC_GATE_EITHER || p->gate_rule > ORC_GATE_DIFFER) return ORC_EINVAL;
    if (p->merge != 0 && p->merge != 1) return ORC_EINVAL;
    if (p->w_col < 0 || p->w_pos < 0 || p->w_bnd < 0) return ORC_EINVAL;
    int32_t prev = 0;
    for (int l = 0; l < p->n_levels; l++) {
        if (p->factor[l] < 1 || p->n_stages[l] < 1 || p->n_stages[l] > ORC_MAX_STAGES)
            return ORC_EINVAL;
        for (int st = 0; st < p->n_stages[l]; st++) {
            int32_t B = p->stages[l][st] * p->factor[l];
            if (B < 1 || B > 64) return ORC_EINVAL;
            if (prev && (B > prev || prev % B)) return ORC_EINVAL;
            prev = B;
        }
    }
    return ORC_OK;
}

/* One full segmentation, Algorithm RAPID: grid labels and statistics once at
 * the first level, then every stage of every level in order; past the gate
 * level only gated pairs move.  labels: W*H int32 out.  stats_out: K'*6 int64
 * (n, S0, S1, S2, Tx, Ty), may be NULL.  rep: one entry per stage, may be
 * NULL.  Returns the number of stages run, or an error code. */
int orc_segment_ex(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                   const orc_params *p, const uint8_t *gate,
                   int32_t *labels, int64_t *stats_out,
                   orc_stage_report *rep, int32_t max_rep, int32_t debug,
                   uint8_t *involved, int64_t *moved);

int orc_segment(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                const orc_params *p, const uint8_t *gate,
                int32_t *labels, int64_t *stats_out,
                orc_stage_report *rep, int32_t max_rep, int32_t debug)
{
    return orc_segment_ex(rgb, W, H, stride, p, gate, labels, stats_out, rep, max_rep, debug,
                          NULL, NULL);
}

/* As orc_segment, plus two optional per-superpixel outputs:
 *   involved[k] = 1 when k is the source or target of any proposal at a
 *                 level >= gate_level (the gate's training target), else 0;
 *   moved[k]    = pixels moved into or out of k by committed moves. */
int orc_segment_ex(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                   const orc_params *p, const uint8_t *gate,
                   int32_t *labels, int64_t *stats_out,
                   orc_stage_report *rep, int32_t max_rep, int32_t debug,
                   uint8_t *involved, int64_t *moved)
{
    int rc = check_params(p, W, H);
    if (rc) return rc;
    if (!rgb || !labels || stride < 3 * (int64_t)W) return ORC_EINVAL;
    int32_t gx = p->gx, gy = p->gy;
    if (p->K > 0 && (rc = orc_grid(W, H, p->K, &gx, &gy))) return rc;
    if (gx < 1 || gy < 1) return ORC_EINVAL;
    int32_t B0 = p->stages[0][0] * p->factor[0];
    if ((rc = orc_init_labels(W, H, B0, gx, gy, labels))) return rc;
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = gx * gy;
    int32_t K = s.K;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.n0 = calloc(K, sizeof(int64_t));
    if (p->merge) s.req = calloc(K, 1);
    if (!s.n || !s.S || !s.T || !s.c || !s.mu || !s.n0 || (p->merge && !s.req)) { rc = ORC_ENOMEM; goto done; }
    /* statistics are computed once (first level) and reused afterwards */
    if ((rc = stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T))) goto done;
    for (int32_t k = 0; k < K; k++) {
        if (s.n[k] == 0) { rc = ORC_EINVAL; goto done; }
        s.n0[k] = s.n[k];
        refresh_means(&s, k);
    }
    int nrep = 0;
    if (involved) memset(involved, 0, K);
    if (moved) memset(moved, 0, sizeof(int64_t) * K);
    s.moved = moved;
    for (int l = 0; l < p->n_levels; l++) {
        s.gate = (gate && p->gate_level >= 0 && l >= p->gate_level) ? gate : NULL;
        s.involved = (involved && p->gate_level >= 0 && l >= p->gate_level) ? involved : NULL;
        for (int st = 0; st < p->n_stages[l]; st++) {
            orc_stage_report r;
            rc = run_stage(&s, l, p->stages[l][st] * p->factor[l], labels, &r, debug);
            if (rc) goto done;
            if (rep && nrep < max_rep) rep[nrep] = r;
            nrep++;
        }
    }
    if (stats_out)
        for (int32_t k = 0; k < K; k++) {
            stats_out[6 * (int64_t)k] = s.n[k];
            for (int ch = 0; ch < 3; ch++) stats_out[6 * (int64_t)k + 1 + ch] = s.S[3 * (int64_t)k + ch];
            stats_out[6 * (int64_t)k + 4] = s.T[2 * (int64_t)k];
            stats_out[6 * (int64_t)k + 5] = s.T[2 * (int64_t)k + 1];
        }
    rc = nrep;
done:
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu); free(s.n0); free(s.bl); free(s.bs);
    free(s.req);
    return rc;
}

/* --------------------------------------------- sequential FIFO baseline */

/* Best label for block (bx, by) under the current means, as in propose():
 * -1 when the block may not move (size, topology), else the label of least
 * E' among its own and its 4-neighbours' within max_size (strictly lower
 * energy, candidates in ascending order). */
static int32_t fifo_best(const state *s, int32_t bx, int32_t by)
{
    const orc_params *p = s->p;
    blk b = block_geom(s, bx, by);
    int32_t a = blabel(s, bx, by);
    if (s->n[a] - b.m < p->min_size || !is_simple_block(s, bx, by)) return -1;
    int32_t nbl[4] = {blabel(s, bx - 1, by), blabel(s, bx + 1, by), blabel(s, bx, by - 1), blabel(s, bx, by + 1)};
    int32_t cand[4];
    int nc = 0;
    for (int d = 0; d < 4; d++) {
        int32_t k = nbl[d];
        int dup = k < 0 || k == a;
        for (int e = 0; e < nc && !dup; e++) dup = cand[e] == k;
        if (!dup) cand[nc++] = k;
    }
    for (int u = 1; u < nc; u++)
        for (int v = u; v > 0 && cand[v - 1] > cand[v]; v--) {
            int32_t t = cand[v]; cand[v] = cand[v - 1]; cand[v - 1] = t;
        }
    int32_t best = a;
    i128 estar = block_energy(s, bx, by, a);
    for (int e = 0; e < nc; e++) {
        if (s->n[cand[e]] + b.m > p->max_size) continue;
        i128 ek = block_energy(s, bx, by, cand[e]);
        if (ek < estar) { estar = ek; best = cand[e]; }
    }
    return best;
}

/* Sequential CTFTPS with the boundary queue of Algorithm RAPID read
 * literally, as a baseline for the synchronous class schedule: at every
 * stage the boundary blocks (Eq. (2)) enter a FIFO in row-major order; a
 * popped block that is simple and may leave its superpixel takes the label
 * of least E' (Eq. (3)); a move updates the sums and both superpixels' means
 * at once and appends the moved block and its 4-neighbours that are
 * boundary blocks and not queued.  A stage ends when the queue is empty or
 * after max_sweeps x (blocks of the stage) pops.  Same grid, energy, size
 * bounds, levels and reuse as orc_segment; no gate and no merge.  labels:
 * W*H out; stats_out: K'*6 or NULL; moves_out: total moves or NULL.  Returns
 * the number of stages run, or an error code. */
int orc_segment_fifo(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride, const orc_params *p,
                     int32_t *labels, int64_t *stats_out, int64_t *moves_out, int32_t debug)
{
    int rc = check_params(p, W, H);
    if (rc) return rc;
    if (!rgb || !labels || stride < 3 * (int64_t)W || p->merge) return ORC_EINVAL;
    int32_t gx = p->gx, gy = p->gy;
    if (p->K > 0 && (rc = orc_grid(W, H, p->K, &gx, &gy))) return rc;
    if (gx < 1 || gy < 1) return ORC_EINVAL;
    int32_t B0 = p->stages[0][0] * p->factor[0];
    if ((rc = orc_init_labels(W, H, B0, gx, gy, labels))) return rc;
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = gx * gy;
    int32_t K = s.K;
    int64_t moves = 0;
    int nst = 0;
    int64_t *q = NULL;
    uint8_t *inq = NULL;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    if (!s.n || !s.S || !s.T || !s.c || !s.mu) { rc = ORC_ENOMEM; goto done; }
    if ((rc = stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T))) goto done;
    for (int32_t k = 0; k < K; k++) refresh_means(&s, k);
    for (int l = 0; l < p->n_levels; l++)
        for (int st = 0; st < p->n_stages[l]; st++) {
            int32_t B = p->stages[l][st] * p->factor[l];
            if ((rc = build_blocks(&s, B, labels))) goto done;
            int64_t nb = (int64_t)s.nbx * s.nby;
            free(q); free(inq);
            q = malloc(sizeof(int64_t) * nb);
            inq = calloc(nb, 1);
            if (!q || !inq) { rc = ORC_ENOMEM; goto done; }
            int64_t head = 0, len = 0;
            for (int64_t i = 0; i < nb; i++)
                if (eligible(&s, (int32_t)(i % s.nbx), (int32_t)(i / s.nbx))) { q[len++] = i; inq[i] = 1; }
            int64_t pops = 0, cap = (int64_t)p->max_sweeps * nb;
            while (len > 0 && pops < cap) {
                int64_t bi = q[head];
                head = (head + 1) % nb;
                len--;
                inq[bi] = 0;
                pops++;
                int32_t bx = (int32_t)(bi % s.nbx), by = (int32_t)(bi / s.nbx);
                int32_t a = s.bl[bi], k = fifo_best(&s, bx, by);
                if (k < 0 || k == a) continue;
                blk b = block_geom(&s, bx, by);
                s.bl[bi] = k;
                s.n[a] -= b.m; s.n[k] += b.m;
                for (int ch = 0; ch < 3; ch++) {
                    s.S[3 * (int64_t)a + ch] -= s.bs[3 * bi + ch];
                    s.S[3 * (int64_t)k + ch] += s.bs[3 * bi + ch];
                }
                s.T[2 * (int64_t)a] -= b.px_; s.T[2 * (int64_t)k] += b.px_;
                s.T[2 * (int64_t)a + 1] -= b.py_; s.T[2 * (int64_t)k + 1] += b.py_;
                refresh_means(&s, a);
                refresh_means(&s, k);
                moves++;
                static const int d5[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
                for (int d = 0; d < 5; d++) {
                    int32_t x = bx + d5[d][0], y = by + d5[d][1];
                    if (x < 0 || y < 0 || x >= s.nbx || y >= s.nby) continue;
                    int64_t ni = (int64_t)y * s.nbx + x;
                    if (!inq[ni] && eligible(&s, x, y)) {
                        q[(head + len) % nb] = ni;
                        len++;
                        inq[ni] = 1;
                    }
                }
            }
            for (int32_t y = 0; y < H; y++)
                for (int32_t x = 0; x < W; x++)
                    labels[(int64_t)y * W + x] = s.bl[(int64_t)(y / B) * s.nbx + x / B];
            if (debug && (rc = check_invariants(&s)) != ORC_OK) goto done;
            nst++;
        }
    if (stats_out)
        for (int32_t k = 0; k < K; k++) {
            stats_out[6 * (int64_t)k] = s.n[k];
            for (int ch = 0; ch < 3; ch++) stats_out[6 * (int64_t)k + 1 + ch] = s.S[3 * (int64_t)k + ch];
            stats_out[6 * (int64_t)k + 4] = s.T[2 * (int64_t)k];
            stats_out[6 * (int64_t)k + 5] = s.T[2 * (int64_t)k + 1];
        }
    if (moves_out) *moves_out = moves;
    rc = nst;
done:
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu); free(s.bl); free(s.bs); free(q); free(inq);
    return rc;
}

/* Eq. (1) at pixel level for pixel labels (statistics recounted, means
 * rounded as everywhere), saturated to the int64 range: the measure the
 * schedule comparison uses. */
int64_t orc_energy(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride, const orc_params *p,
                   const int32_t *labels, int32_t K)
{
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = K;
    int64_t r = INT64_MIN;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    if (s.n && s.S && s.T && s.c && s.mu &&
        stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T) == ORC_OK &&
        build_blocks(&s, 1, labels) == ORC_OK) {
        for (int32_t k = 0; k < K; k++) refresh_means(&s, k);
        i128 e = global_energy(&s);
        r = e > (i128)INT64_MAX ? INT64_MAX : (int64_t)e;
    }
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu); free(s.bl); free(s.bs);
    return r;
}

/* Proposals of class cls at block size B for an arbitrary valid state given
 * by pixel labels (all eligible blocks active, statistics recounted from the
 * labels).  props: 3 int32 per proposal (block index, from, to); eprime: the
 * energy change E'(beta,to) - E'(beta,from) of each.  Returns the count. */
int orc_propose_class(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                      const orc_params *p, const int32_t *labels, int32_t K,
                      int32_t B, int32_t cls, const uint8_t *gate,
                      int32_t *props, int64_t *eprime, int32_t max_props)
{
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = K; s.gate = gate;
    int rc = ORC_OK;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    proposal *pr = NULL; uint8_t *act = NULL; int64_t *order = NULL;
    if (!s.n || !s.S || !s.T || !s.c || !s.mu) { rc = ORC_ENOMEM; goto done; }
    if ((rc = stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T))) goto done;
    for (int32_t k = 0; k < K; k++) if (s.n[k]) refresh_means(&s, k);
    if ((rc = build_blocks(&s, B, labels))) goto done;
    int64_t nb = (int64_t)s.nbx * s.nby;
    pr = malloc(sizeof(proposal) * (int64_t)((s.nbx + 2) / 3) * ((s.nby + 2) / 3));
    act = malloc(nb); order = malloc(sizeof(int64_t) * nb);
    if (!pr || !act || !order) { rc = ORC_ENOMEM; goto done; }
    for (int64_t i = 0; i < nb; i++) { order[i] = i; act[i] = (uint8_t)eligible(&s, (int32_t)(i % s.nbx), (int32_t)(i / s.nbx)); }
    int64_t sm = 0, stp = 0;
    int64_t np = propose(&s, cls, act, pr, &sm, &stp, NULL, nb);
    if (np > max_props) { rc = ORC_EINVAL; goto done; }
    for (int64_t q = 0; q < np; q++) {
        props[3 * q] = pr[q].b; props[3 * q + 1] = pr[q].a; props[3 * q + 2] = pr[q].k;
        if (eprime) eprime[q] = pr[q].de;
    }
    rc = (int)np;
done:
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu); free(s.bl); free(s.bs);
    free(pr); free(act); free(order);
    return rc;
}

/* E'(beta, k) of block (bx, by) at block size B for a state given by pixel
 * labels (statistics recounted).  Saturates to INT64 range. */
int64_t orc_block_energy(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                         const orc_params *p, const int32_t *labels, int32_t K,
                         int32_t B, int32_t bx, int32_t by, int32_t k)
{
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = K;
    int64_t r = INT64_MIN;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    if (s.n && s.S && s.T && s.c && s.mu &&
        stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T) == ORC_OK) {
        for (int32_t k2 = 0; k2 < K; k2++) if (s.n[k2]) refresh_means(&s, k2);
        if (build_blocks(&s, B, labels) == ORC_OK) {
            i128 e = block_energy(&s, bx, by, k);
            r = e > (i128)INT64_MAX ? INT64_MAX : (e < -(i128)INT64_MAX ? -INT64_MAX : (int64_t)e);
        }
    }
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu); free(s.bl); free(s.bs);
    return r;
}


/* Energy change of merging superpixel m into k (merge_cost) for a state
 * given by pixel labels constant on blocks of size B (statistics recounted,
 * shared boundary counted over pixel pairs).  Saturates to INT64 range;
 * INT64_MIN on a bad argument. */
int64_t orc_merge_cost(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                       const orc_params *p, const int32_t *labels, int32_t K, int32_t m, int32_t k)
{
    state s;
    memset(&s, 0, sizeof s);
    s.rgb = rgb; s.W = W; s.H = H; s.stride = stride; s.p = p; s.K = K;
    int64_t r = INT64_MIN;
    if (m < 0 || k < 0 || m >= K || k >= K || m == k) return r;
    s.n = calloc(K, sizeof(int64_t)); s.S = calloc(3 * (int64_t)K, sizeof(int64_t));
    s.T = calloc(2 * (int64_t)K, sizeof(int64_t));
    s.c = calloc(3 * (int64_t)K, sizeof(int64_t)); s.mu = calloc(2 * (int64_t)K, sizeof(int64_t));
    if (s.n && s.S && s.T && s.c && s.mu &&
        stats_from_labels(rgb, W, H, stride, labels, K, s.n, s.S, s.T) == ORC_OK && s.n[m] && s.n[k]) {
        for (int32_t j = 0; j < K; j++) refresh_means(&s, j);
        int64_t len = 0;
        for (int32_t y = 0; y < H; y++)
            for (int32_t x = 0; x < W; x++) {
                int32_t a = labels[(int64_t)y * W + x];
                if (x + 1 < W) {
                    int32_t b = labels[(int64_t)y * W + x + 1];
                    len += (a == m && b == k) || (a == k && b == m);
                }
                if (y + 1 < H) {
                    int32_t b = labels[(int64_t)(y + 1) * W + x];
                    len += (a == m && b == k) || (a == k && b == m);
                }
            }
        i128 e = merge_cost(&s, m, k, len);
        r = e > (i128)INT64_MAX ? INT64_MAX : (e < -(i128)INT64_MAX ? -INT64_MAX : (int64_t)e);
    }
    free(s.n); free(s.S); free(s.T); free(s.c); free(s.mu);
    return r;
}

/* ------------------------------------------------------- gate features */

/* Sixteen features of every superpixel at the gate point (Eq. (6) needs a
 * feature vector x per superpixel; the paper's classifier uses absolute and
 * comparative colour and region dissimilarity -- these are this project's
 * own choice along those lines, all from exact integer accumulators):
 *   0-2  mean colour / 255
 *   3-5  colour standard deviation / 64 (pixel second moments)
 *   6    size / nominal area A
 *   7    boundary length / (4 sqrt A)
 *   8    compactness: boundary length^2 / (16 size)
 *   9    centroid drift from the initial grid cell centre / sqrt A
 *   10-12 max, edge-weighted rms and min colour contrast to neighbours
 *        (distance of fixed-point means) / (255 2^F)
 *   13   pixels moved in or out so far / size
 *   14   max of features 3-5
 *   15   1
 * (a superpixel merged away has all 16 features 0)
 * labels: pixel labels constant on blocks of size B (the last stage before
 * the gate); stats: K x 6 (n, S, T); moved: K (may be NULL: zeros). */
int orc_features(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                 const int32_t *labels, int32_t B, const int64_t *stats, const int64_t *moved,
                 int32_t gx, int32_t gy, int32_t F, float *out)
{
    int32_t K = gx * gy;
    int64_t *Q = calloc(3 * (int64_t)K, sizeof(int64_t));
    int64_t *bl = calloc(K, sizeof(int64_t)), *ced = calloc(K, sizeof(int64_t));
    int64_t *cmax = calloc(K, sizeof(int64_t)), *cmin = malloc(sizeof(int64_t) * K);
    int64_t *cm = malloc(sizeof(int64_t) * 3 * K);
    if (!Q || !bl || !ced || !cmax || !cmin || !cm) {
        free(Q); free(bl); free(ced); free(cmax); free(cmin); free(cm);
        return ORC_ENOMEM;
    }
    for (int32_t k = 0; k < K; k++) {
        cmin[k] = -1;
        for (int ch = 0; ch < 3; ch++)
            cm[3 * k + ch] = stats[6 * (int64_t)k] ? div_round(stats[6 * (int64_t)k + 1 + ch], stats[6 * (int64_t)k], F) : 0;
    }
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t k = labels[(int64_t)y * W + x];
            const uint8_t *q = rgb + (int64_t)y * stride + 3 * (int64_t)x;
            for (int ch = 0; ch < 3; ch++) Q[3 * k + ch] += (int64_t)q[ch] * q[ch];
            /* boundary pixel pairs to the right and below */
            for (int d = 0; d < 2; d++) {
                int32_t xx = x + (d == 0), yy = y + (d == 1);
                if (xx >= W || yy >= H) continue;
                int32_t j = labels[(int64_t)yy * W + xx];
                if (j == k) continue;
                int64_t d2 = 0;
                for (int ch = 0; ch < 3; ch++) {
                    int64_t df = cm[3 * k + ch] - cm[3 * j + ch];
                    d2 += df * df;
                }
                int32_t both[2] = {k, j};
                for (int u = 0; u < 2; u++) {
                    int32_t t = both[u];
                    bl[t] += 1;
                    ced[t] += d2;
                    if (d2 > cmax[t]) cmax[t] = d2;
                    if (cmin[t] < 0 || d2 < cmin[t]) cmin[t] = d2;
                }
            }
        }
    (void)B;
    double A = (double)(((int64_t)W * H) / K);
    double sA = sqrt(A);
    double cs = 255.0 * (double)(1 << F);
    for (int32_t k = 0; k < K; k++) {
        const int64_t *r = stats + 6 * (int64_t)k;
        double n = (double)r[0];
        float *f = out + 16 * (int64_t)k;
        if (r[0] == 0) {   /* merged away: all features 0 */
            for (int i = 0; i < 16; i++) f[i] = 0.0f;
            continue;
        }
        double sd[3];
        for (int ch = 0; ch < 3; ch++) {
            double mu = (double)r[1 + ch] / n;
            double v = (double)Q[3 * k + ch] / n - mu * mu;
            sd[ch] = sqrt(v > 0.0 ? v : 0.0);
            f[ch] = (float)(mu / 255.0);
            f[3 + ch] = (float)(sd[ch] / 64.0);
        }
        f[6] = (float)(n / A);
        f[7] = (float)((double)bl[k] / (4.0 * sA));
        f[8] = (float)((double)bl[k] * (double)bl[k] / (16.0 * n));
        int32_t col = k % gx, row = k / gx;
        double cx0 = (double)(2 * col + 1) * (double)W / (2.0 * gx) - 0.5;
        double cy0 = (double)(2 * row + 1) * (double)H / (2.0 * gy) - 0.5;
        double dx = (double)r[4] / n - cx0, dy = (double)r[5] / n - cy0;
        f[9] = (float)(sqrt(dx * dx + dy * dy) / sA);
        f[10] = (float)(sqrt((double)cmax[k]) / cs);
        f[11] = (float)(bl[k] ? sqrt((double)ced[k] / (double)bl[k]) / cs : 0.0);
        f[12] = (float)(cmin[k] >= 0 ? sqrt((double)cmin[k]) / cs : 0.0);
        f[13] = (float)((moved ? (double)moved[k] : 0.0) / n);
        double m3 = sd[0] > sd[1] ? sd[0] : sd[1];
        m3 = m3 > sd[2] ? m3 : sd[2];
        f[14] = (float)(m3 / 64.0);
        f[15] = 1.0f;
    }
    free(Q); free(bl); free(ced); free(cmax); free(cmin); free(cm);
    return ORC_OK;
}

/* The paper's four ROI features of every superpixel (Sec. 4: the feature
 * vector F in R^4 of absolute and comparative brightness, extra-region and
 * intra-region dissimilarity), in the 16-wide row layout of orc_features:
 *   0  absolute brightness: the mean of the three channel means, / 255;
 *   1  comparative brightness: that brightness minus the mean brightness of
 *      the superpixel's neighbours, one neighbour term per 4-adjacent pixel
 *      pair across its border, each the neighbour's three fixed-point means
 *      (round(2^F S / n), Eq. (1)'s means as the sweep keeps them) summed and
 *      divided by 3 2^F; / 255; 0 without neighbours;
 *   2  extra-region dissimilarity: the rms over those pixel pairs of the
 *      distance between the two fixed-point mean colours, / (255 2^F); 0
 *      without neighbours;
 *   3  intra-region dissimilarity: sqrt of the mean over the three channels
 *      of the pixel variance within the superpixel, / 64;
 *   4..14 zero, 15 one; a superpixel with no pixels has all 16 zero.
 * Plain pixel loops over the label map; stats is the K x 6 statistics. */
int orc_roi_features(const uint8_t *rgb, int32_t W, int32_t H, int64_t stride,
                     const int32_t *labels, const int64_t *stats, int32_t gx, int32_t gy, int32_t F,
                     float *out)
{
    int32_t K = gx * gy;
    int64_t *Q = calloc(3 * (int64_t)K, sizeof(int64_t));
    int64_t *pairs = calloc(K, sizeof(int64_t)), *dist2 = calloc(K, sizeof(int64_t));
    int64_t *nbright = calloc(K, sizeof(int64_t));
    int64_t *cm = malloc(sizeof(int64_t) * 3 * (K > 0 ? K : 1));
    if (!Q || !pairs || !dist2 || !nbright || !cm) {
        free(Q); free(pairs); free(dist2); free(nbright); free(cm);
        return ORC_ENOMEM;
    }
    for (int32_t k = 0; k < K; k++) {
        const int64_t n = stats[6 * (int64_t)k];
        for (int ch = 0; ch < 3; ch++) cm[3 * k + ch] = n ? div_round(stats[6 * (int64_t)k + 1 + ch], n, F) : 0;
    }
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            const int32_t k = labels[(int64_t)y * W + x];
            const uint8_t *px = rgb + (int64_t)y * stride + 3 * (int64_t)x;
            for (int ch = 0; ch < 3; ch++) Q[3 * k + ch] += (int64_t)px[ch] * px[ch];
            /* each 4-adjacent pixel pair once: the right and the lower one */
            for (int d = 0; d < 2; d++) {
                const int32_t xx = x + (d == 0), yy = y + (d == 1);
                if (xx >= W || yy >= H) continue;
                const int32_t j = labels[(int64_t)yy * W + xx];
                if (j == k) continue;
                int64_t d2 = 0;
                for (int ch = 0; ch < 3; ch++) {
                    const int64_t df = cm[3 * k + ch] - cm[3 * j + ch];
                    d2 += df * df;
                }
                pairs[k] += 1;
                pairs[j] += 1;
                dist2[k] += d2;
                dist2[j] += d2;
                nbright[k] += cm[3 * j] + cm[3 * j + 1] + cm[3 * j + 2];
                nbright[j] += cm[3 * k] + cm[3 * k + 1] + cm[3 * k + 2];
            }
        }
    for (int32_t k = 0; k < K; k++) {
        const int64_t *r = stats + 6 * (int64_t)k;
        float *f = out + 16 * (int64_t)k;
        for (int i = 0; i < 16; i++) f[i] = 0.0f;
        if (r[0] == 0) continue;
        const double n = (double)r[0];
        const double bright = ((double)r[1] + (double)r[2] + (double)r[3]) / (3.0 * n);
        double var = 0.0;
        for (int ch = 0; ch < 3; ch++) {
            const double mean = (double)r[1 + ch] / n;
            const double v = (double)Q[3 * k + ch] / n - mean * mean;
            var += v > 0.0 ? v : 0.0;
        }
        f[0] = (float)(bright / 255.0);
        if (pairs[k]) {
            const double nb = (double)nbright[k] / (3.0 * (double)pairs[k] * (double)(1 << F));
            f[1] = (float)((bright - nb) / 255.0);
            f[2] = (float)(sqrt((double)dist2[k] / (double)pairs[k]) / (255.0 * (double)(1 << F)));
        }
        f[3] = (float)(sqrt(var / 3.0) / 64.0);
        f[15] = 1.0f;
    }
    free(Q); free(pairs); free(dist2); free(nbright); free(cm);
    return ORC_OK;
}
