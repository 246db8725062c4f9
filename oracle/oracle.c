/*
 * CPU oracle for jump flooding (JFA) and dynamic jump flooding (dJFA).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library: the two sides
 * meet only through the seeded input generators and through the published
 * definition of splitmix64, which each side implements on its own.
 *
 * Plain scalar C, int64 arithmetic, no SIMD, no blocking, no fusion.  Rows of
 * one pass may be split over host threads; every pass reads one buffer and
 * writes another (Jacobi), so the result does not depend on the split.
 *
 * Paper: "GPU Voronoi Diagrams for Random Moving Seeds" (Stevenson-Regla and
 * Navarro).  Each function names the passage it follows.
 *
 * Label encodings (the paper leaves the label type open, Sec. II and Alg. 1):
 *   ID mode  (label_mode 0): label = seed index i in [0, S).
 *   XY mode  (label_mode 1): label = (y << 16) | x of the seed's position.
 *   Both: ORC_EMPTY (= -1, all bits set) marks a pixel no flood has reached.
 * Total order between two candidates of one pixel: smaller distance wins, a
 * tie goes to the smaller label read as an unsigned 32-bit value (lowest seed
 * index in ID mode, lowest packed position in XY mode).  Eq. (1) lets a
 * boundary pixel belong to several regions; the order picks one of them.
 *
 * Parity pins: every function here is checked against something other than
 * itself by the CPU tests (published splitmix64 vectors, Eq. (2)'s worked
 * example, closed forms of Eq. (5), exhaustive enumeration on tiny grids,
 * scipy distance matrices, single-seed exactness of JFA, fixed points).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_EMPTY (-1)

enum { ORC_EUCLID = 0, ORC_MANHATTAN = 1 };
enum { ORC_LABEL_ID = 0, ORC_LABEL_XY = 1 };
enum { ORC_MOORE = 0, ORC_VN = 1 };

/* ---------------------------------------------------------------------- */
/* splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number  */
/* generators", OOPSLA 2014; the mixing function is Stafford's variant 13). */
/* The generator state advances by the golden gamma; output n (n >= 0) of   */
/* the stream seeded with s is mix64(s + (n + 1) * gamma).                  */
/* ---------------------------------------------------------------------- */
static const uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_stream_out(uint64_t seed, uint64_t n)
{
    return orc_mix64(seed + (n + 1) * GOLDEN_GAMMA);
}

/* Map a 64-bit draw onto [0, m) with Lemire's multiply-shift on the top 32
 * bits (no rejection step, so no modulo and no data-dependent loop). */
uint32_t orc_bounded(uint64_t r, uint32_t m)
{
    return (uint32_t)(((r >> 32) * (uint64_t)m) >> 32);
}

/* ---------------------------------------------------------------------- */
/* SimulateParticles (Alg. 1; Sec. V-A: uniform random moves of up to      */
/* d_max discrete units).  Each seed moves independently on each axis by a */
/* uniform integer in [lo, hi], then is clamped to the grid.  The draw for */
/* (time step t >= 1, seed i, axis a) is output n = ((t-1)*S + i)*2 + a of */
/* the stream seeded with mix64(sim_seed ^ 0x6D6F7665), so any step can be */
/* recomputed without replaying earlier ones.                              */
/* ---------------------------------------------------------------------- */
static int32_t clamp_i32(int64_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : (int32_t)v);
}

void orc_move_seeds(int32_t W, int32_t H, int32_t S, uint64_t sim_seed,
                    int64_t t, int32_t lo, int32_t hi, int32_t *xy)
{
    uint64_t move_seed = orc_mix64(sim_seed ^ 0x6D6F7665ull);
    uint32_t span = (uint32_t)(hi - lo + 1);
    for (int32_t i = 0; i < S; ++i) {
        uint64_t base = ((uint64_t)(t - 1) * (uint64_t)S + (uint64_t)i) * 2u;
        int64_t dx = lo + (int64_t)orc_bounded(orc_stream_out(move_seed, base + 0), span);
        int64_t dy = lo + (int64_t)orc_bounded(orc_stream_out(move_seed, base + 1), span);
        xy[2 * i + 0] = clamp_i32(xy[2 * i + 0] + dx, 0, W - 1);
        xy[2 * i + 1] = clamp_i32(xy[2 * i + 1] + dy, 0, H - 1);
    }
}

/* ---------------------------------------------------------------------- */
/* Step schedules.                                                          */
/* ---------------------------------------------------------------------- */

/* Eq. (2): k_1 = 2^(ceil(log2 N) - 1) with N the grid side; N = max(W, H)
 * for a rectangular grid.  A 1-pixel grid has no passes (returns 0). */
int32_t orc_k1(int32_t W, int32_t H)
{
    int64_t N = W > H ? W : H;
    if (N <= 1) return 0;
    int64_t p = 1;                 /* smallest power of two >= N */
    while (p < N) p *= 2;
    return (int32_t)(p / 2);
}

/* Eq. (5) with Eq. (4): delta_1 = 2^ceil(log2 max(2 L_avg, d_max)), where
 * L_avg = sqrt(W*H / S).  The smallest power of two P with P >= d_max and
 * P >= 2 sqrt(W*H/S) is the smallest one with P >= d_max and
 * P*P*S >= 4*W*H, which needs no floating point.  delta_1 is capped at k_1
 * (the paper's worst case is "as fast as JFA", Sec. V-A). */
int32_t orc_delta1(int32_t W, int32_t H, int32_t S, int32_t dmax)
{
    int32_t k1 = orc_k1(W, H);
    if (k1 == 0) return 0;
    int64_t P = 1;
    while (P < dmax || P * P * (int64_t)S < 4 * (int64_t)W * (int64_t)H) P *= 2;
    return P < k1 ? (int32_t)P : k1;
}

/* ---------------------------------------------------------------------- */
/* Distances (Sec. V-C): squared Euclidean (the square root is monotone and */
/* is dropped, so the arithmetic is exact) and Manhattan.                   */
/* ---------------------------------------------------------------------- */
static int64_t dist(int32_t metric, int64_t dx, int64_t dy)
{
    if (metric == ORC_MANHATTAN) return (dx < 0 ? -dx : dx) + (dy < 0 ? -dy : dy);
    return dx * dx + dy * dy;
}

/* Position a label stands for. */
static void label_pos(int32_t label_mode, int32_t label, const int32_t *xy,
                      int64_t *sx, int64_t *sy)
{
    if (label_mode == ORC_LABEL_XY) {
        *sx = (uint32_t)label & 0xFFFFu;
        *sy = (uint32_t)label >> 16;
    } else {
        *sx = xy[2 * (int64_t)label + 0];
        *sy = xy[2 * (int64_t)label + 1];
    }
}

static int32_t pack_xy(int32_t x, int32_t y) { return (int32_t)(((uint32_t)y << 16) | (uint32_t)x); }

/* Does candidate (dc, lc) beat the incumbent (db, lb)? */
static int beats(int64_t dc, int32_t lc, int64_t db, int32_t lb)
{
    return dc < db || (dc == db && (uint32_t)lc < (uint32_t)lb);
}

/* ---------------------------------------------------------------------- */
/* Brute force from the definition of a Voronoi region, Eq. (1): each pixel */
/* takes the seed at the smallest distance; ties go to the lowest index.    */
/* ---------------------------------------------------------------------- */
void orc_brute_force(int32_t W, int32_t H, int32_t S, const int32_t *xy,
                     int32_t metric, int32_t *map)
{
    for (int32_t y = 0; y < H; ++y)
        for (int32_t x = 0; x < W; ++x) {
            int64_t bd = INT64_MAX;
            int32_t bi = ORC_EMPTY;
            for (int32_t i = 0; i < S; ++i) {
                int64_t d = dist(metric, (int64_t)x - xy[2 * i], (int64_t)y - xy[2 * i + 1]);
                if (d < bd) { bd = d; bi = i; }   /* strict: the lowest index keeps a tie */
            }
            map[(int64_t)y * W + x] = bi;
        }
}

/* Exact nearest seed (Euclidean) of sampled pixels, by an O(S) scan each. */
void orc_nearest_scan(int32_t S, const int32_t *xy, int64_t npix,
                      const int32_t *px, const int32_t *py,
                      int32_t *out_id, int64_t *out_d)
{
    for (int64_t p = 0; p < npix; ++p) {
        int64_t bd = INT64_MAX;
        int32_t bi = ORC_EMPTY;
        for (int32_t i = 0; i < S; ++i) {
            int64_t d = dist(ORC_EUCLID, (int64_t)px[p] - xy[2 * i], (int64_t)py[p] - xy[2 * i + 1]);
            if (d < bd) { bd = d; bi = i; }
        }
        out_id[p] = bi;
        out_d[p] = bd;
    }
}

/* Exact nearest seed (Euclidean) of sampled pixels with a uniform bucket
 * grid: seeds are binned into B x B cells; rings of cells around the pixel's
 * cell are searched outward.  Every seed in a ring r+1 or farther differs
 * from the pixel by at least r*B + 1 on some axis, so once the best squared
 * distance found is below (r*B + 1)^2 no unseen seed can reach or tie it.
 * Same answer as orc_nearest_scan (the tests check this); used where the
 * scan is too slow (millions of pixels against millions of seeds). */
void orc_nearest_bucketed(int32_t W, int32_t H, int32_t S, const int32_t *xy,
                          int64_t npix, const int32_t *px, const int32_t *py,
                          int32_t *out_id, int64_t *out_d)
{
    /* cell side so that a cell holds about two seeds */
    int64_t B = 1;
    while (B * B * (int64_t)S < 2 * (int64_t)W * (int64_t)H) B *= 2;
    int64_t CW = (W + B - 1) / B, CH = (H + B - 1) / B;
    int64_t ncell = CW * CH;
    int64_t *start = (int64_t *)calloc((size_t)(ncell + 1), sizeof(int64_t));
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(S > 0 ? S : 1));
    int64_t *fill = (int64_t *)calloc((size_t)(ncell + 1), sizeof(int64_t));
    for (int32_t i = 0; i < S; ++i) start[(xy[2 * i + 1] / B) * CW + xy[2 * i] / B + 1]++;
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    for (int32_t i = 0; i < S; ++i) {
        int64_t c = (xy[2 * i + 1] / B) * CW + xy[2 * i] / B;
        ids[start[c] + fill[c]++] = i;
    }
    int64_t maxr = CW > CH ? CW : CH;
    for (int64_t p = 0; p < npix; ++p) {
        int64_t cx = px[p] / B, cy = py[p] / B;
        int64_t bd = INT64_MAX;
        int32_t bi = ORC_EMPTY;
        for (int64_t r = 0; r <= maxr; ++r) {
            for (int64_t gy = cy - r; gy <= cy + r; ++gy) {
                if (gy < 0 || gy >= CH) continue;
                for (int64_t gx = cx - r; gx <= cx + r; ++gx) {
                    if (gx < 0 || gx >= CW) continue;
                    if (gy != cy - r && gy != cy + r && gx != cx - r && gx != cx + r) continue;
                    int64_t c = gy * CW + gx;
                    for (int64_t j = start[c]; j < start[c + 1]; ++j) {
                        int32_t i = ids[j];
                        int64_t d = dist(ORC_EUCLID, (int64_t)px[p] - xy[2 * i], (int64_t)py[p] - xy[2 * i + 1]);
                        if (d < bd || (d == bd && i < bi)) { bd = d; bi = i; }
                    }
                }
            }
            if (bi != ORC_EMPTY && bd < (r * B + 1) * (r * B + 1)) break;
        }
        out_id[p] = bi;
        out_d[p] = bd;
    }
    free(start);
    free(ids);
    free(fill);
}

/* ---------------------------------------------------------------------- */
/* Map initialisation.                                                      */
/* ---------------------------------------------------------------------- */

/* Every pixel unclaimed: JFA starts from an empty grid (Sec. III). */
void orc_fill_empty(int64_t npix, int32_t *map)
{
    for (int64_t p = 0; p < npix; ++p) map[p] = ORC_EMPTY;
}

/* Seeds are the starting points of the floods (Sec. III).  Each seed's own
 * pixel gets that seed's label; where several seeds share a pixel the lowest
 * index wins (ID mode).  In XY mode the label is the pixel's own position. */
void orc_splat_active(int32_t W, int32_t S, const int32_t *xy, const uint8_t *active,
                      int32_t label_mode, int32_t *map)
{
    for (int32_t i = S - 1; i >= 0; --i) {     /* descending: the lowest index is written last */
        if (active && !active[i]) continue;    /* a removed seed is no flood start */
        int64_t p = (int64_t)xy[2 * i + 1] * W + xy[2 * i];
        map[p] = label_mode == ORC_LABEL_XY ? pack_xy(xy[2 * i], xy[2 * i + 1]) : i;
    }
}

void orc_splat(int32_t W, int32_t S, const int32_t *xy, int32_t label_mode, int32_t *map)
{
    orc_splat_active(W, S, xy, NULL, label_mode, map);
}

/* XY mode only: after a move, a label of the previous map is an old seed
 * position.  It becomes the new position of the lowest-index seed that sat
 * there.  (ID labels survive a move unchanged, so ID mode needs nothing.)
 * A label that is no old seed position becomes EMPTY. */
void orc_relabel_xy_active(int32_t W, int32_t H, int32_t S, const int32_t *old_xy,
                           const uint8_t *keep, const int32_t *new_xy, int32_t *map)
{
    /* label l (an old position) -> the moved position of the lowest-index
     * seed that sat at l when the diagram was made and has stayed in the
     * seed set since (keep[i] != 0; NULL: every seed); unclaimed if there
     * is none */
    int64_t npix = (int64_t)W * H;
    int32_t *at = (int32_t *)malloc(sizeof(int32_t) * (size_t)npix);
    for (int64_t p = 0; p < npix; ++p) at[p] = ORC_EMPTY;
    for (int32_t i = S - 1; i >= 0; --i)
        if (!keep || keep[i]) at[(int64_t)old_xy[2 * i + 1] * W + old_xy[2 * i]] = i;
    for (int64_t p = 0; p < npix; ++p) {
        int32_t l = map[p];
        if (l == ORC_EMPTY) continue;
        int64_t lx = (uint32_t)l & 0xFFFFu, ly = (uint32_t)l >> 16;
        int32_t i = (lx < W && ly < H) ? at[ly * W + lx] : ORC_EMPTY;
        map[p] = i == ORC_EMPTY ? ORC_EMPTY : pack_xy(new_xy[2 * i], new_xy[2 * i + 1]);
    }
    free(at);
}

void orc_relabel_xy(int32_t W, int32_t H, int32_t S, const int32_t *old_xy,
                    const int32_t *new_xy, int32_t *map)
{
    orc_relabel_xy_active(W, H, S, old_xy, NULL, new_xy, map);
}

/* ID labels of seeds that have left the seed set since the diagram was
 * made (keep[i] == 0: removed, or removed and inserted again) become
 * unclaimed. */
void orc_purge_id(int64_t npix, const uint8_t *keep, int32_t *map)
{
    for (int64_t p = 0; p < npix; ++p)
        if (map[p] != ORC_EMPTY && !keep[map[p]]) map[p] = ORC_EMPTY;
}

/* ---------------------------------------------------------------------- */
/* One flood pass at step k (Sec. III, Table I; Sec. V-B).                  */
/*                                                                          */
/* The paper states the pass as each pixel pushing its seed to the pixels   */
/* of its neighbourhood in place (Alg. 1).  Both neighbourhoods are         */
/* symmetric, so pushing from p to p+o offers exactly the pairs that pixel  */
/* q gathers from q-o.  The oracle gathers, reading `in` and writing `out`: */
/* out[q] = best of in[q] and in[q + o] over the offsets o, by (distance    */
/* from q to the label's seed, label).  Offsets that leave the grid and     */
/* EMPTY labels offer nothing; out[q] is EMPTY only if nothing is offered.  */
/* ---------------------------------------------------------------------- */

/* Table I: the Moore offsets at distance k (neighbours 1..8); the Von
 * Neumann neighbourhood keeps the four axis-aligned ones (Fig. 4). */
static const int32_t MOORE_OFF[8][2] = {
    {+1, 0}, {+1, +1}, {0, +1}, {-1, +1}, {-1, 0}, {-1, -1}, {0, -1}, {+1, -1},
};

typedef struct {
    int32_t W, H, k, nbhd, metric, label_mode;
    const int32_t *xy, *in;
    int32_t *out;
    int32_t y0, y1;
} pass_job;

static void pass_rows(const pass_job *j)
{
    for (int32_t y = j->y0; y < j->y1; ++y)
        for (int32_t x = 0; x < j->W; ++x) {
            int64_t bd = INT64_MAX;
            int32_t bl = ORC_EMPTY;
            for (int32_t o = -1; o < 8; ++o) {           /* o = -1: the pixel itself */
                int64_t cx = x, cy = y;
                if (o >= 0) {
                    if (j->nbhd == ORC_VN && MOORE_OFF[o][0] != 0 && MOORE_OFF[o][1] != 0) continue;
                    cx += (int64_t)MOORE_OFF[o][0] * j->k;
                    cy += (int64_t)MOORE_OFF[o][1] * j->k;
                }
                if (cx < 0 || cx >= j->W || cy < 0 || cy >= j->H) continue;
                int32_t l = j->in[cy * j->W + cx];
                if (l == ORC_EMPTY) continue;
                int64_t sx, sy;
                label_pos(j->label_mode, l, j->xy, &sx, &sy);
                int64_t d = dist(j->metric, (int64_t)x - sx, (int64_t)y - sy);
                if (bl == ORC_EMPTY || beats(d, l, bd, bl)) { bd = d; bl = l; }
            }
            j->out[(int64_t)y * j->W + x] = bl;
        }
}

static void *pass_thread(void *arg)
{
    pass_rows((const pass_job *)arg);
    return NULL;
}

void orc_pass(int32_t W, int32_t H, const int32_t *xy, const int32_t *in, int32_t *out,
              int32_t k, int32_t nbhd, int32_t metric, int32_t label_mode, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > H) nthreads = H;
    if (nthreads > 256) nthreads = 256;
    pass_job jobs[256];
    pthread_t tid[256];
    for (int32_t t = 0; t < nthreads; ++t) {
        pass_job j = {W, H, k, nbhd, metric, label_mode, xy, in, out,
                      (int32_t)((int64_t)H * t / nthreads), (int32_t)((int64_t)H * (t + 1) / nthreads)};
        jobs[t] = j;
    }
    if (nthreads == 1) {
        pass_rows(&jobs[0]);
        return;
    }
    for (int32_t t = 0; t < nthreads; ++t) pthread_create(&tid[t], NULL, pass_thread, &jobs[t]);
    for (int32_t t = 0; t < nthreads; ++t) pthread_join(tid[t], NULL);
}

/* ---------------------------------------------------------------------- */
/* Pass schedules.                                                          */
/* ---------------------------------------------------------------------- */

/* Writes the step sizes and neighbourhoods of one time step; returns the
 * number of passes.  JFA (Sec. III, Eq. (2)): k_1, k_1/2, ..., 1, all Moore.
 * dJFA (Sec. V-A, Eq. (5); Sec. V-B): delta_1, delta_1/2, ..., 1; the first
 * min(vn_passes, passes - 1) use the Von Neumann neighbourhood, the rest
 * Moore, so the last k = 1 pass always sees all eight neighbours.  Extra
 * passes (JFA+1 / JFA+2, Sec. III; the optional extra step of Sec. V-A):
 * one appends k = 1, two append k = 2 then k = 1, both Moore. */
int32_t orc_schedule(int32_t W, int32_t H, int32_t S, int32_t dynamic, int32_t dmax,
                     int32_t vn_passes, int32_t extra_passes, int32_t *ks, int32_t *nbhds,
                     int32_t cap)
{
    int32_t first = dynamic ? orc_delta1(W, H, S, dmax) : orc_k1(W, H);
    int32_t n = 0;
    int32_t main_passes = 0;
    for (int32_t k = first; k >= 1; k /= 2) ++main_passes;
    int32_t vn = dynamic ? (vn_passes < main_passes - 1 ? vn_passes : main_passes - 1) : 0;
    if (vn < 0) vn = 0;
    for (int32_t k = first; k >= 1; k /= 2) {
        if (n < cap) { ks[n] = k; nbhds[n] = n < vn ? ORC_VN : ORC_MOORE; }
        ++n;
    }
    for (int32_t e = extra_passes; e >= 1; --e) {
        if (n < cap) { ks[n] = e; nbhds[n] = ORC_MOORE; }
        ++n;
    }
    return n;
}

/* Runs passes in order, ping-ponging between map and tmp; the result ends
 * in map. */
static void run_passes(int32_t W, int32_t H, const int32_t *xy, int32_t *map, int32_t *tmp,
                       const int32_t *ks, const int32_t *nbhds, int32_t n, int32_t metric,
                       int32_t label_mode, int32_t nthreads)
{
    int64_t npix = (int64_t)W * H;
    int32_t *a = map, *b = tmp;
    for (int32_t i = 0; i < n; ++i) {
        orc_pass(W, H, xy, a, b, ks[i], nbhds[i], metric, label_mode, nthreads);
        int32_t *t = a; a = b; b = t;
    }
    if (a != map) memcpy(map, a, sizeof(int32_t) * (size_t)npix);
}

/* A custom pass list on the given map (used for the Von Neumann-only and
 * reduction checks). */
void orc_run_passes(int32_t W, int32_t H, const int32_t *xy, int32_t *map,
                    const int32_t *ks, const int32_t *nbhds, int32_t n, int32_t metric,
                    int32_t label_mode, int32_t nthreads)
{
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * (size_t)H);
    run_passes(W, H, xy, map, tmp, ks, nbhds, n, metric, label_mode, nthreads);
    free(tmp);
}

/* Full JFA on the current seed positions (Sec. III): an empty grid, the
 * seeds as flood starting points, then the passes of Eq. (2). */
void orc_jfa_step_active(int32_t W, int32_t H, int32_t S, const int32_t *xy,
                         const uint8_t *active, int32_t metric, int32_t label_mode,
                         int32_t extra_passes, int32_t *map, int32_t nthreads)
{
    int32_t ks[80], nb[80];
    int32_t n = orc_schedule(W, H, S, 0, 0, 0, extra_passes, ks, nb, 80);
    orc_fill_empty((int64_t)W * H, map);
    orc_splat_active(W, S, xy, active, label_mode, map);
    orc_run_passes(W, H, xy, map, ks, nb, n, metric, label_mode, nthreads);
}

void orc_jfa_step(int32_t W, int32_t H, int32_t S, const int32_t *xy, int32_t metric,
                  int32_t label_mode, int32_t extra_passes, int32_t *map, int32_t nthreads)
{
    orc_jfa_step_active(W, H, S, xy, NULL, metric, label_mode, extra_passes, map, nthreads);
}

/* dJFA after the seed set has changed (insertion and removal of seeds, a
 * case the paper leaves to future work, Sec. VII).  keep[i] != 0 marks the
 * seeds present when the diagram was made and ever since; active[i] != 0
 * the seeds present now (both NULL: the plain step).  Labels of the other
 * seeds leave the diagram first (ID: purged to unclaimed; XY: by the
 * relabel), only present seeds are splatted, and Eq. (5) takes the number
 * of present seeds.  A removed seed's cell must be refilled by its
 * neighbours within the passes; if a pixel is still unclaimed afterwards,
 * the step becomes a full JFA step instead.  Returns 1 in that case. */
int32_t orc_djfa_step_active(int32_t W, int32_t H, int32_t S, const int32_t *old_xy,
                             const int32_t *xy, const uint8_t *keep, const uint8_t *active,
                             int32_t dmax, int32_t metric, int32_t label_mode,
                             int32_t vn_passes, int32_t extra_passes, int32_t *map,
                             int32_t nthreads)
{
    int32_t ks[80], nb[80];
    int32_t S_on = S;
    if (active) {
        S_on = 0;
        for (int32_t i = 0; i < S; ++i) S_on += active[i] ? 1 : 0;
    }
    int32_t n = orc_schedule(W, H, S_on, 1, dmax, vn_passes, extra_passes, ks, nb, 80);
    int64_t npix = (int64_t)W * H;
    if (label_mode == ORC_LABEL_XY)
        orc_relabel_xy_active(W, H, S, old_xy, keep, xy, map);
    else if (keep)
        orc_purge_id(npix, keep, map);
    orc_splat_active(W, S, xy, active, label_mode, map);
    orc_run_passes(W, H, xy, map, ks, nb, n, metric, label_mode, nthreads);
    if (!keep) return 0;
    for (int64_t p = 0; p < npix; ++p) {
        if (map[p] == ORC_EMPTY) {
            orc_jfa_step_active(W, H, S, xy, active, metric, label_mode, extra_passes, map,
                                nthreads);
            return 1;
        }
    }
    return 0;
}

/* One dJFA time step (Alg. 1, after SimulateParticles): start from the
 * previous diagram, (XY mode) move its labels to the seeds' new positions,
 * re-seed every seed's own pixel, then the delta schedule of Eq. (5). */
void orc_djfa_step(int32_t W, int32_t H, int32_t S, const int32_t *old_xy, const int32_t *xy,
                   int32_t dmax, int32_t metric, int32_t label_mode, int32_t vn_passes,
                   int32_t extra_passes, int32_t *map, int32_t nthreads)
{
    orc_djfa_step_active(W, H, S, old_xy, xy, NULL, NULL, dmax, metric, label_mode, vn_passes,
                         extra_passes, map, nthreads);
}

/* ---------------------------------------------------------------------- */
/* Similarity (Sec. VI-A): 100 * matching pixels / total pixels.            */
/* ---------------------------------------------------------------------- */

/* Pixels whose labels are equal in two maps (the paper's dJFA-vs-JFA). */
int64_t orc_count_equal(int64_t npix, const int32_t *a, const int32_t *b)
{
    int64_t c = 0;
    for (int64_t p = 0; p < npix; ++p) c += a[p] == b[p];
    return c;
}

/* Pixels (of a sample) whose label's seed is at the exact nearest Euclidean
 * distance; nearest_d holds that distance for each sampled pixel.  Equal
 * distance counts as a match, so any of several tied seeds is accepted. */
int64_t orc_count_exact(int32_t W, const int32_t *xy, int32_t label_mode, const int32_t *map,
                        int64_t npix, const int32_t *px, const int32_t *py,
                        const int64_t *nearest_d)
{
    int64_t c = 0;
    for (int64_t p = 0; p < npix; ++p) {
        int32_t l = map[(int64_t)py[p] * W + px[p]];
        if (l == ORC_EMPTY) continue;
        int64_t sx, sy;
        label_pos(label_mode, l, xy, &sx, &sy);
        c += dist(ORC_EUCLID, (int64_t)px[p] - sx, (int64_t)py[p] - sy) == nearest_d[p];
    }
    return c;
}
