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
    VD_ESTATE = -4    /* the call does not fit the object's state */
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
    int32_t dmax_override;   /* d_max of Eq. (5); <= 0 means max(|disp_lo|, |disp_hi|) */
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

/* Per-kernel timing gathered with HIP events on the simulation's stream
 * while enabled (vd_set_timing).  Durations are summed over launches. */
typedef struct vd_timing {
    int64_t flood_launches;  /* flood passes timed */
    double flood_ms;         /* their summed duration */
    int64_t flood_pixels;    /* pixel-updates they performed (width*height each) */
    int64_t step_count;      /* whole JFA / dJFA steps timed */
    double step_ms;          /* their summed duration (fill/splat/relabel + passes) */
} vd_timing;

/* Fills *cfg with the defaults: ID labels, Euclidean distance, vn_passes 2,
 * extra_passes 0, dmax_override 0, sim_seed 1, moves in [-1, 1]; the caller
 * sets width, height and num_seeds. */
void vd_config_default(vd_config *cfg);

/* Device bytes vd_init_sim needs for cfg: two ping-pong label maps
 * (4 B per pixel each), the seed table (4 B per seed plus one sentinel
 * entry; in XY mode also the positions the diagram refers to) and 256 B of
 * alignment slack.  Returns 0 if cfg is invalid. */
size_t vd_footprint_bytes(const vd_config *cfg);

/* Creates a simulation (Sec. IV: the diagram VD and the seed set S are the
 * state carried across time steps) and computes VD_0 by a full JFA on the
 * initial positions; t = 0.
 *  host_xy:  2*S int32 values, (x, y) of seed i at [2i], [2i+1]; positions in
 *            the grid; need not be distinct.  Copied; the caller keeps it.
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
 * d_max units): t += 1, then every seed i moves by (dx, dy), each drawn
 * uniformly from [disp_lo, disp_hi] as output ((t-1)*S + i)*2 + axis of the
 * splitmix64 stream seeded with mix64(sim_seed ^ 0x6D6F7665), mapped onto
 * the range by ((r >> 32) * span) >> 32; positions clamp to the grid.
 * Does not touch the diagram. */
int vd_move_seeds(vd_sim *sim);

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
 * 128 (and is 1 above); -1 restores the default (3 for ID labels, 1 for
 * XY labels).  Variants differ in speed only: every variant writes the same
 * labels. */
int vd_set_flood_variant(vd_sim *sim, int variant);

/* Releases the handle (never the caller's workspace).  Waits for the
 * simulation's pending work.  NULL is ignored. */
void vd_destroy(vd_sim *sim);

/* Message of the last failed call on this thread ("" if none). */
const char *vd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VDFLOOD_H */
