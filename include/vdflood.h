/*
 * vdflood -- C ABI of the MI355X (gfx950) jump-flooding library.
 *
 * Computes Voronoi diagrams of seeds that move over time on a 2D pixel grid,
 * following "GPU Voronoi Diagrams for Random Moving Seeds" (Stevenson-Regla
 * and Navarro): the Jump Flooding Algorithm (JFA, Sec. III) recomputed from
 * scratch at each time step, and the paper's dynamic JFA (dJFA, Sec. V,
 * Alg. 1), which starts from the previous step's diagram and runs fewer
 * passes.  Every step of the path runs in HIP kernels on the device.
 *
 * Conventions shared by every call:
 *  - Pointers named dev_* are device memory, host_* are host memory.
 *  - Device work is enqueued on the HIP stream given to vd_init_sim and is
 *    asynchronous, except the vd_read_* calls, which wait for it.
 *  - A call returns VD_OK (0) or a negative vd_status; it never throws and
 *    never aborts.  On failure vd_last_error() describes the cause, and the
 *    simulation is left as it was before the call, except after
 *    VD_EDEVICE, after which only vd_destroy is safe.
 *  - Arguments are validated before any device work is enqueued.
 *  - One vd_sim must not be driven from two threads at once; different
 *    vd_sim handles may be.
 *
 * Labels: a diagram is a row-major width x height array of 32-bit labels.
 *  VD_LABEL_ID32: the label is the index of the pixel's seed, in [0, S).
 *  VD_LABEL_XY16: the label is the seed's position packed as (y << 16) | x.
 *  Both use VD_EMPTY (all bits set) for a pixel no flood has reached.
 * When two seeds are at the same distance from a pixel, the smaller label
 * (read as unsigned) wins: the lowest seed index, or the lowest packed
 * position.  Eq. (1) admits either seed; this rule makes the result unique.
 */
#ifndef VDFLOOD_H
#define VDFLOOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VD_ABI_VERSION 1

typedef enum vd_status {
    VD_OK = 0,
    VD_EINVAL = -1,   /* an argument is out of range or NULL */
    VD_ENOMEM = -2,   /* workspace too small, or a host allocation failed */
    VD_EDEVICE = -3,  /* a HIP call failed (the message names it) */
    VD_ESTATE = -4,   /* the call does not fit the object's state */
    VD_EBUSY = -5     /* a wait timed out; the work is still in progress */
} vd_status;

enum { VD_LABEL_ID32 = 0, VD_LABEL_XY16 = 1 };
enum { VD_EUCLID = 0, VD_MANHATTAN = 1 };

#define VD_EMPTY (-1)
/* Largest grid side (2^14 - 16).  Positions pack into two 16-bit halves
 * with an offset of 16384, and every squared distance, to a seed or to the
 * library's far sentinel position (-16384, -16384), stays below
 * 2^31 - 2^20. */
#define VD_MAX_SIDE 16368
#define VD_MAX_EXTRA_PASSES 2

/* dmax_override value: d_max measured per dJFA step instead of configured
 * (see vd_config). */
#define VD_DMAX_MEASURED (-1)

/* Parameters of one simulation (Sec. II: grid X, seed set S; Sec. V-A: the
 * move bound d_max; Sec. V-B/V-C: neighbourhood and distance choices). */
typedef struct vd_config {
    int32_t width, height;   /* grid, 1 .. VD_MAX_SIDE each */
    int32_t num_seeds;       /* S, 1 .. width * height */
    int32_t disp_lo;         /* each move draws a uniform integer in [disp_lo, disp_hi] */
    int32_t disp_hi;         /*   per axis, then clamps to the grid; |value| <= VD_MAX_SIDE */
    int32_t label;           /* VD_LABEL_ID32 or VD_LABEL_XY16 */
    int32_t metric;          /* VD_EUCLID (dJFAe) or VD_MANHATTAN (dJFAm), Sec. V-C */
    int32_t vn_passes;       /* dJFA: leading Von Neumann passes, Sec. V-B; default 2 */
    int32_t extra_passes;    /* 0, 1 (k = 1) or 2 (k = 2, 1) appended to each step (JFA+1/+2) */
    int32_t dmax_override;   /* d_max of Eq. (5): > 0 that value; 0 max(|disp_lo|, |disp_hi|);
                                VD_DMAX_MEASURED: per dJFA step, the sum over the moves
                                since the previous step of each move's largest per-axis
                                displacement after clamping, measured on the device (the
                                dJFA step then waits for its stream; not for capture) */
    uint64_t sim_seed;       /* seeds the move stream (splitmix64) */
} vd_config;

typedef struct vd_sim vd_sim;  /* opaque; owned by the library */

typedef struct vd_sim_info {
    int32_t width, height, num_seeds, label, metric;
    int32_t k1;              /* first JFA step, Eq. (2); 0 on a 1-pixel grid */
    int32_t delta1;          /* first dJFA step, Eq. (5) (capped at k1) */
    int32_t passes_jfa;      /* flood passes per JFA step, extras included */
    int32_t passes_djfa;     /* flood passes per dJFA step, extras included */
    int64_t t;               /* time step: 0 after init, +1 per vd_move_seeds */
} vd_sim_info;

/* Timing gathered with HIP events on the simulation's stream while enabled
 * (vd_set_timing).  The flood passes of a step are timed as one run between
 * two events (so flood_ms includes the short gaps between consecutive
 * passes); durations are summed over runs and steps. */
typedef struct vd_timing {
    int64_t flood_launches;  /* flood passes timed */
    double flood_ms;         /* their summed duration (gaps between passes included) */
    int64_t flood_pixels;    /* pixel-updates they performed (width*height each) */
    int64_t step_count;      /* whole JFA / dJFA steps timed */
    double step_ms;          /* their summed duration (fill/splat/relabel + passes) */
} vd_timing;

/* Fills *cfg with the defaults: ID labels, Euclidean distance, vn_passes 2,
 * extra_passes 0, dmax_override 0, sim_seed 1, moves in [-1, 1]; the caller
 * sets width, height and num_seeds. */
void vd_config_default(vd_config *cfg);

/* Device bytes vd_init_sim needs for cfg: two ping-pong label maps
 * (4 B per pixel each; in XY mode a third, the old-position index of dJFA
 * steps), the seed table (4 B per seed plus one sentinel entry; in XY mode
 * also the positions the diagram refers to), 256 B of
 * step counters, the seed-set state (1 B per seed; in ID mode also 4 B per
 * seed for the positions of removed seeds) and 256 B of alignment slack,
 * each part 256-B aligned.
 * Returns 0 if cfg is invalid. */
size_t vd_footprint_bytes(const vd_config *cfg);

/* Bytes of the fixed device array vd_jfa_noalloc takes its scratch from
 * (one array per GPU, held from the library's first use of that GPU until
 * the process ends): 72 MiB. */
#define VD_NOALLOC_SCRATCH_BYTES (72u << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, serving loops (hipMalloc and hipFree can stall every stream of
 * the device), harnesses that forbid allocation: the diagram vd_init_sim
 * computes as VD_0 (a full JFA step on the given positions: Sec. III,
 * Table I, Eq. (2)), written straight into caller memory, with no
 * simulation, no workspace and no allocation.  The library's scratch (the
 * seed table, 4 B per seed plus the sentinel entry, 1 B per seed of state,
 * and the second ping-pong map, 4 B per pixel, each part 256-B aligned)
 * comes from a fixed device array of VD_NOALLOC_SCRATCH_BYTES, so
 * width*height is limited to about 18.8 M pixels (4096 x 4096 with up to
 * 2^20 seeds); a larger request returns VD_EINVAL and launches nothing.
 *  cfg:     width, height, num_seeds, label, metric and extra_passes are
 *           used (validated as by vd_init_sim); the rest is ignored.
 *  dev_xy:  device memory, 2*num_seeds int32: (x, y) of seed i at [2i],
 *           [2i+1].  A seed off the grid takes no part (its label never
 *           appears); positions need not be distinct.
 *  dev_map: device memory, width*height int32, row-major; receives the
 *           labels in vd_read_map's encoding.  Must not overlap dev_xy.
 *  hip_stream: hipStream_t the work is queued on (NULL: default stream).
 * Asynchronous: returns once the work is queued.  Every call on one GPU
 * shares that GPU's scratch array, so calls whose work overlaps on one GPU
 * (on different streams or threads, without ordering between them) race;
 * calls on one stream are ordered.  The first call on a device resolves
 * the array's address there (hipGetSymbolAddress). */
int vd_jfa_noalloc(const vd_config *cfg, const int32_t *dev_xy, int32_t *dev_map,
                   void *hip_stream);

/* Initial seed positions as the paper's experiments draw them (Sec. VI-A:
 * seeds uniformly at random on the grid), host only (no device work):
 * num_seeds distinct pixels taken in order from the splitmix64 stream of
 * `seed` (Steele, Lea and Flood, 2014: output n is mix64(seed + (n + 1) *
 * 0x9E3779B97F4A7C15) with Stafford's variant-13 mixer); pair j is
 * (x, y) = (bounded(output 2j, width), bounded(output 2j + 1, height)),
 * bounded(r, m) = ((r >> 32) * m) >> 32, and a pair whose pixel is already
 * taken is skipped.
 *  host_xy: receives 2*num_seeds int32 values, (x, y) of seed i at [2i],
 *           [2i+1].
 * Returns VD_EINVAL for sizes outside those vd_init_sim accepts
 * (1 <= num_seeds <= width*height) or a NULL host_xy, VD_ENOMEM if the
 * width*height-byte mask of taken pixels cannot be allocated.  With
 * num_seeds close to width*height the number of draws grows like
 * width*height*ln(width*height). */
int vd_place_seeds(int32_t width, int32_t height, int32_t num_seeds, uint64_t seed,
                   int32_t *host_xy);

/* Creates a simulation (Sec. IV: the diagram VD and the seed set S are the
 * state carried across time steps) and computes VD_0 by a full JFA on the
 * initial positions; t = 0.
 *  host_xy:  2*S int32 values, (x, y) of seed i at [2i], [2i+1]; positions in
 *            the grid; need not be distinct.  Copied; the caller keeps it.
 *            NULL: the positions vd_place_seeds draws from cfg->sim_seed.
 *  dev_workspace, ws_bytes: device buffer of at least vd_footprint_bytes(cfg)
 *            bytes, any alignment.  Owned by the caller, who keeps it alive
 *            and untouched until vd_destroy.
 *  hip_stream: hipStream_t every later call of this simulation runs on
 *            (NULL: the default stream).
 *  out:      receives the handle.
 * Returns before VD_0 is complete (stream order applies). */
int vd_init_sim(const vd_config *cfg, const int32_t *host_xy, void *dev_workspace,
                size_t ws_bytes, void *hip_stream, vd_sim **out);

/* SimulateParticles of Alg. 1 (Sec. V-A: uniform random moves of up to
 * d_max units): t += 1, then every present seed i (see vd_remove_seeds)
 * moves by (dx, dy), each drawn
 * uniformly from [disp_lo, disp_hi] as output ((t-1)*S + i)*2 + axis of the
 * splitmix64 stream seeded with mix64(sim_seed ^ 0x6D6F7665), mapped onto
 * the range by ((r >> 32) * span) >> 32; positions clamp to the grid.
 * Does not touch the diagram. */
int vd_move_seeds(vd_sim *sim);

/* Seed movement of any kind (the generalisation Sec. VII leaves open): t
 * += 1, then seed i moves to (host_xy[2i], host_xy[2i+1]); count must be
 * 2*S and every position on the grid (VD_EINVAL otherwise, nothing
 * changed).  With dmax_override = VD_DMAX_MEASURED the next dJFA step sizes
 * its first jump from the displacement.  Does not touch the diagram; waits
 * for the stream (the positions are copied before it returns). */
int vd_set_seeds(vd_sim *sim, const int32_t *host_xy, size_t count);

/* A changing seed set: insertion and removal of seeds between time steps
 * (named as future work in Sec. VII).  The seed table of a simulation has
 * num_seeds slots, all present after vd_init_sim; a seed keeps its index
 * (its ID label) while present.  Removed seeds neither move nor take part in
 * a step; vd_read_seeds still reports their last positions.  Neither call is
 * a time step (t is unchanged) nor touches the diagram; the next step takes
 * the change into account:
 *  - vd_jfa_step floods from the present seeds only;
 *  - vd_djfa_step first drops the labels of every seed that has not been
 *    present without a break since the diagram was made (ID: those pixels
 *    become unclaimed; XY: a label resolves to the lowest-index such seed
 *    that sat at the labelled position, else unclaimed), splats the present
 *    seeds, and runs the Eq. (5) schedule for the number of present seeds.
 *    If a pixel is still unclaimed after its passes (a removed cell too wide
 *    for them to refill), the step is redone as a full JFA step.  Such a
 *    step counts the unclaimed pixels on the device and waits for its
 *    stream.
 * Batches (vd_batch_create) refuse a simulation once a seed has been
 * inserted or removed, and both calls return VD_ESTATE for a batch member.
 * Both wait for the stream (the host buffers are copied before return).
 *
 * vd_remove_seeds: host_ids holds n distinct indices of present seeds; at
 * least one seed must stay present (VD_EINVAL otherwise, nothing changed). */
int vd_remove_seeds(vd_sim *sim, const int32_t *host_ids, size_t n);

/* vd_insert_seeds: n new seeds at (host_xy[2j], host_xy[2j+1]) take free
 * slots in ascending index order, first the slots free since before the
 * last step, then slots removed since (only the latter make the next dJFA
 * step purge their old labels, one extra pass over the map in ID mode);
 * host_ids[j] receives the index of seed j.  VD_ESTATE if fewer than n
 * slots are free, VD_EINVAL for a position off the grid (nothing changed in
 * either case). */
int vd_insert_seeds(vd_sim *sim, const int32_t *host_xy, size_t n, int32_t *host_ids);

/* The seed set: host_present (NULL: skipped; else count == num_seeds bytes)
 * receives 1 for a present seed and 0 for a free slot; *num_present the
 * number of present seeds; *fallbacks the number of dJFA steps redone as
 * JFA steps (either pointer may be NULL). */
int vd_get_seed_set(const vd_sim *sim, uint8_t *host_present, size_t count,
                    int32_t *num_present, int64_t *fallbacks);

/* JFA on the current positions (Sec. III): every pixel EMPTY, each seed's
 * own pixel labelled (lowest index where seeds coincide), then flood passes
 * at k = k1, k1/2, ..., 1 over the Moore neighbourhood of Table I, each
 * pixel keeping the best of itself and its in-grid neighbours at offset k,
 * plus the extra passes.  Replaces the current diagram. */
int vd_jfa_step(vd_sim *sim);

/* dJFA (Sec. V, Alg. 1) on the current positions, starting from the current
 * diagram (the previous step's): in XY mode each label is first moved to
 * its seed's new position; each seed's own pixel is relabelled; then passes
 * at delta = delta1, ..., 1 (Eq. (5)), the first min(vn_passes, passes - 1)
 * over the Von Neumann neighbourhood, the rest Moore, plus the extra
 * passes.  Replaces the current diagram. */
int vd_djfa_step(vd_sim *sim);

/* Copies the current diagram (width*height labels, row-major) to host_dst;
 * count must equal width*height.  Waits for the stream. */
int vd_read_map(vd_sim *sim, int32_t *host_dst, size_t count);

/* Copies the current positions, (x, y) per seed, to host_xy; count must be
 * 2*S.  Waits for the stream. */
int vd_read_seeds(vd_sim *sim, int32_t *host_xy, size_t count);

/* Device address of the current diagram (width*height uint32 labels).  It
 * stays valid until the next step call; the data are ready once the
 * simulation's stream has reached this point.  ID labels are as read by
 * vd_read_map.  XY labels are stored as ((y + 16384) << 16) | (x + 16384)
 * with 0 for EMPTY; vd_read_map converts them. */
int vd_map_device(vd_sim *sim, const void **dev_map);

/* Sizes, schedule and time step of a simulation. */
int vd_get_info(const vd_sim *sim, vd_sim_info *out);

/* Enables (1) or disables (0) per-launch HIP-event timing of flood passes
 * and steps on the simulation's stream, and clears the totals. */
int vd_set_timing(vd_sim *sim, int enable);

/* Waits for the stream and returns the totals gathered since timing was
 * enabled or last read; then clears them. */
int vd_get_timing(vd_sim *sim, vd_timing *out);

/* Selects the flood-pass kernel variant for every pass of this simulation:
 * 0, 1 or 2 request each row's labels 1, 2 or 3 rows ahead of the row being
 * written; 3 shares each row across a workgroup through LDS for steps up to
 * 128 (and is 1 above); 4 and 5 give each lane four adjacent columns
 * (16-byte loads and stores) and request rows 2 or 3 rows ahead where the
 * width is a multiple of 4, and are 3 (ID) or 1 (XY) for other widths;
 * 6-11 are 0-5 with non-temporal stores of the output map (faster when the
 * two maps exceed the 256 MB Infinity Cache); -1 restores the defaults:
 * per pass, 4 in JFA and 3 in dJFA steps for ID labels, 4 for JFA steps of
 * k >= 512 and 1 otherwise for XY labels, plus 6 where the two maps exceed
 * 192 MiB.  An XY JFA step that starts from the previous diagram instead of
 * a filled map (where its first pass has k of at least a quarter of both
 * sides, and width and k are multiples of 4) runs that pass with one lane
 * per block of four-column groups whatever the variant, which then picks
 * only the store policy.  Variants differ in speed only: every variant
 * writes the same labels. */
int vd_set_flood_variant(vd_sim *sim, int variant);

/* Tail fusion: a step's last passes (the longest run of steps 1, 2 or 4
 * summing to at most 8, at most four passes, e.g. k = 4, 2, 1) run as one
 * launch that keeps tiles of the map in LDS between them; the map is the
 * same either way.  mode 16, 24 or 32: on, with tiles of 48 x mode
 * outputs; 1: on with 16-row tiles; 0: off; -1: the default (on for maps
 * of up to 2048^2 pixels with ID labels and 1536^2 with XY labels, 16-row
 * tiles up to 2^19 pixels, else 24) or the choice vd_autotune made for the
 * step kind.  VD_EINVAL for another mode; VD_ESTATE for a batch member (a
 * batch runs its solo members' steps with the fusion they had when it was
 * built). */
int vd_set_tail_fusion(vd_sim *sim, int mode);

/* Passes each step kind currently runs fused (0: none). */
int vd_get_tail_fusion(const vd_sim *sim, int32_t *jfa, int32_t *djfa);

/* Chooses, by timing, the kernel variant and the segment length of every
 * flood pass of this simulation's JFA and dJFA steps.  One JFA step (from
 * scratch on the current seeds) and one dJFA step (from the current
 * diagram) are replayed; before each pass every candidate with ordinary
 * stores (variants 0-5) runs reps times (after one warm-up launch) on that
 * pass's actual input.  Then each step kind's passes are replayed whole
 * with the chosen kernels, with ordinary and with non-temporal stores, and
 * the faster store policy is kept for all of them.  The diagram is
 * saved first and put back after (device scratch of width*height*4 bytes,
 * plus the seed table in XY mode, is allocated and freed), so the
 * simulation's state does not change.  The choices also enter a
 * process-wide table keyed by (GPU architecture, width, height, seed count,
 * label, metric, k, neighbourhood, step kind) that later vd_init_sim calls
 * consult.  Results never depend on the choices.  Waits for the stream.
 * VD_ENOMEM if the scratch cannot be allocated. */
int vd_autotune(vd_sim *sim, int32_t reps);

/* Best measured duration (microseconds per launch) of each pass's chosen
 * candidate in this process's autotuning, JFA passes first then dJFA
 * passes; 0 for a pass never tuned.  cap must be at least passes_jfa +
 * passes_djfa. */
int vd_get_tuning_us(const vd_sim *sim, float *us, int32_t cap);

/* Variant and segment length (0: automatic) of each pass, JFA passes first
 * then dJFA passes; cap must be at least passes_jfa + passes_djfa.  Either
 * output array may be NULL. */
int vd_get_tuning(const vd_sim *sim, int32_t *variants, int32_t *seg_rows, int32_t cap);

/* The process-wide tuning table as text, one "key|variant|seg_rows" line
 * per entry.  *needed receives the size including the terminating NUL; buf
 * may be NULL to query it. */
int vd_tuning_export(char *buf, size_t cap, size_t *needed);

/* Adds the entries of a text produced by vd_tuning_export (overwriting
 * equal keys); simulations created afterwards use them. */
int vd_tuning_import(const char *text);

/* Empties the process-wide tuning table (simulations that exist keep the
 * choices they made; later ones start from the defaults). */
int vd_tuning_clear(void);

/* Releases the handle (never the caller's workspace).  Waits for the
 * simulation's pending work.  NULL is ignored.  A simulation that still
 * belongs to a batch is only marked: vd_batch_destroy releases it, and its
 * workspace must stay untouched until then. */
void vd_destroy(vd_sim *sim);

/* ---------------------------------------------------------------------- */
/* Batches: many simulations advanced together with fused launches.        */
/* ---------------------------------------------------------------------- */

typedef struct vd_batch vd_batch;   /* opaque; owned by the library */

enum { VD_STEP_JFA = 0, VD_STEP_DJFA = 1 };

/* Device bytes of a batch of n simulations (its tables and counters); 0 if
 * n is outside [1, 32768]. */
size_t vd_batch_footprint_bytes(int32_t n);

/* Groups n existing simulations so that vd_batch_step advances them all.
 * Members (ID or XY labels, mixed as needed) must use one metric and the
 * batch's hip_stream (the stream they were created on); their own
 * workspaces stay in use.  While a simulation belongs to the batch,
 * vd_move_seeds / vd_jfa_step / vd_djfa_step on it return VD_ESTATE, and
 * vd_destroy only marks it: vd_batch_destroy then releases the handle (its
 * workspace must stay untouched until then); reads and vd_get_info keep
 * working.  dev_workspace (any alignment, at least
 * vd_batch_footprint_bytes(n) bytes) is owned by the caller and must stay
 * untouched until vd_batch_destroy.  The pointer array is copied. */
int vd_batch_create(vd_sim *const *sims, int32_t n, void *dev_workspace, size_t ws_bytes,
                    void *hip_stream, vd_batch **out);

/* One time step of every member: if move != 0 the seeds move first
 * (exactly as vd_move_seeds), then a JFA (mode VD_STEP_JFA) or a dJFA
 * (VD_STEP_DJFA) step, each member's result identical to running that
 * member alone.  Pass level i of every member runs in one persistent
 * launch that balances the members' tiles over the GPU.  Asynchronous. */
int vd_batch_step(vd_batch *b, int32_t mode, int32_t move);

/* enable != 0: each kind of step (mode, move) is captured into a hipGraph
 * the first time it runs and replayed afterwards (one graph launch per
 * step).  enable == 0 drops the graphs and launches kernels directly. */
int vd_batch_set_graph(vd_batch *b, int enable);

/* Persistent flood grid: wg_per_cu workgroups per compute unit (0: as
 * many as fit, the default).  Speed only; results do not change. */
int vd_batch_set_shape(vd_batch *b, int32_t wg_per_cu);

/* Chooses by timing, separately for JFA and dJFA steps, the persistent
 * grid (1, 2, 4 or 8 workgroups per compute unit, or as many as fit) and
 * which members run solo (none, or all members of at least one of the
 * members' sizes; see vd_batch_set_solo): each candidate runs the step's
 * flood work reps times reading the current diagrams and writing the idle
 * buffers, so no simulation changes.  Drops captured graphs.  Waits for the
 * stream. */
int vd_batch_autotune(vd_batch *b, int32_t reps);

/* Members of at least min_pixels pixels (<= 0: none) run the passes of
 * `mode` steps solo: with their own launches, kernel variants and tail
 * fusion (as chosen by vd_autotune / vd_set_flood_variant /
 * vd_set_tail_fusion before the batch was built), on four streams forked
 * from the batch's stream and joined before the step ends: members of
 * 4096 x 4096 pixels and up one after another on the first, those of
 * 2048 x 2048 and up on the second, so each keeps its maps in the Infinity
 * Cache across its passes, the smaller ones alternating on the other two
 * (one stream while per-launch timing is on); the others share one
 * persistent launch per pass level.  Move, fill, splat and the step's
 * bookkeeping stay batched.  Results do not change.  Drops captured graphs;
 * waits for the stream. */
int vd_batch_set_solo(vd_batch *b, int32_t mode, int64_t min_pixels);

/* Per-level flood and per-step timing with HIP events, as for a single
 * simulation (not recorded inside captured graphs: with graphs on, only
 * whole steps are timed). */
int vd_batch_set_timing(vd_batch *b, int enable);
int vd_batch_get_timing(vd_batch *b, vd_timing *out);

/* Pass levels of a JFA and a dJFA step, and the persistent grid size. */
int vd_batch_info(const vd_batch *b, int32_t *levels_jfa, int32_t *levels_djfa, int32_t *grid);

/* Waits for the batch's work and releases it; members become free
 * simulations again, with their state as the last step left it. */
void vd_batch_destroy(vd_batch *b);

/* Message of the last failed call on this thread ("" if none). */
const char *vd_last_error(void);

/* ---------------------------------------------------------------------- */
/* Serving: time-step requests of many resident simulations, run by a      */
/* scheduler thread either as whole steps or batched at pass granularity.  */
/* ---------------------------------------------------------------------- */

typedef struct vd_server vd_server;   /* opaque; owned by the library */

typedef struct vd_server_stats {
    int64_t submitted;        /* requests submitted since the last reset */
    int64_t completed;        /* requests finished since the last reset */
    int64_t pixel_updates;    /* flood pixel-updates of finished ticks */
    int64_t ticks;            /* ticks issued (whole-step groups or batched pass launches) */
    double elapsed_s;         /* wall time since the last reset */
    double mean_ms, p50_ms, p99_ms, max_ms;   /* request latency: submit -> done */
    int32_t resident;         /* simulations with device state */
    int32_t waiting_admission;/* simulations waiting for memory */
} vd_server_stats_t;

/* Device bytes the server's own tables take from the pool for up to
 * max_sims simulations; simulations need vd_footprint_bytes each on top. */
size_t vd_server_footprint_bytes(int32_t max_sims);

/* Starts a server (and its scheduler thread) for up to max_sims
 * simulations (ID or XY labels) of one metric.  dev_pool (pool_bytes, any alignment) is
 * caller-owned device memory holding the server tables and every
 * simulation's workspace; it must outlive vd_server_destroy.  All device
 * work runs on hip_stream. */
int vd_server_create(int32_t max_sims, int32_t metric, void *dev_pool, size_t pool_bytes,
                     void *hip_stream, vd_server **out);

/* Registers a simulation (cfg as for vd_init_sim; the metric must be the
 * server's) and returns its id.  It becomes resident (workspace
 * placed in the pool, VD_0 computed) as soon as its footprint fits;
 * simulations wait for memory in registration order.  host_xy is copied;
 * NULL: the positions vd_place_seeds draws from cfg->sim_seed. */
int vd_server_add_sim(vd_server *sv, const vd_config *cfg, const int32_t *host_xy,
                      int32_t *sim_id);

/* How requests started from now on run.  The scheduler forms ticks on the
 * server's stream (at most two in flight); a tick starts the next request
 * of every resident simulation that has one, and every request completes
 * with its tick.  VD_SERVE_STEPS: each request as its simulation's move
 * and step with that simulation's own launches (tuned kernel variants,
 * fused tail), one simulation after another.  VD_SERVE_PASSES (the
 * default; continuous batching of the tick's requests): their moves and
 * step starts run in shared launches over all of them; then each runs its
 * passes with its own launches on one of four streams -- simulations of
 * 4096 x 4096 pixels and up one after another on the first, so each keeps
 * its maps in the Infinity Cache, the others round the other three beside
 * them -- or, below vd_server_set_solo's size when two or more start in the
 * tick, in one persistent launch per pass level over all of them.  A tick
 * in which a single request starts runs it as a whole step.  Results are
 * identical either way.  VD_EINVAL for another value. */
enum { VD_SERVE_STEPS = 0, VD_SERVE_PASSES = 1 };
int vd_server_set_policy(vd_server *sv, int32_t policy);

/* VD_SERVE_PASSES ticks: simulations of at least min_pixels pixels run
 * their passes with their own launches, smaller ones share the pass-level
 * launches (min_pixels <= 0, the default: every simulation alone).
 * Takes effect from the next tick; results never change. */
int vd_server_set_solo(vd_server *sv, int64_t min_pixels);

/* Queues one time step of a simulation: a move, then a JFA (VD_STEP_JFA) or
 * dJFA (VD_STEP_DJFA) step.  Requests of one simulation run in submission
 * order; its result equals the same sequence of vd_move_seeds + step calls
 * on a lone simulation.  Returns at once with a ticket. */
int vd_server_submit(vd_server *sv, int32_t sim_id, int32_t mode, int64_t *ticket);

/* Waits (timeout_ms < 0: without limit) until a ticket's step has
 * finished on the GPU; *latency_ms receives submit-to-finish time.  A
 * ticket can be waited for once.  VD_EBUSY on timeout. */
int vd_server_wait(vd_server *sv, int64_t ticket, double timeout_ms, double *latency_ms);

/* Waits until every submitted request has finished (VD_EBUSY on timeout). */
int vd_server_drain(vd_server *sv, double timeout_ms);

/* Unregisters a simulation: waits for its running request, drops queued
 * ones, frees its memory (admitting waiting simulations). */
int vd_server_remove_sim(vd_server *sv, int32_t sim_id);

/* The current diagram of an idle resident simulation (VD_ESTATE while it
 * has requests in progress or is not resident; the server's error once a
 * launch or tick has failed); as vd_read_map. */
int vd_server_read_map(vd_server *sv, int32_t sim_id, int32_t *host_dst, size_t count);

/* Whether a simulation is resident, its time step and its pending requests. */
int vd_server_sim_state(vd_server *sv, int32_t sim_id, int32_t *resident, int64_t *t,
                        int32_t *pending);

/* Counters and latency quantiles since the last reset (reset != 0 starts a
 * new measuring window). */
int vd_server_stats(vd_server *sv, vd_server_stats_t *out, int reset);

/* Stops the scheduler, waits for the GPU and releases every simulation. */
void vd_server_destroy(vd_server *sv);

#ifdef __cplusplus
}
#endif

#endif /* VDFLOOD_H */
