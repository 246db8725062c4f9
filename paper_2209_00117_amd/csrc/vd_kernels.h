// Launch helpers of the vdflood kernels (internal to the library).
//
// Device data layout (internal encodings; vd_read_map converts):
//   seed table  uint32[S + 1]; entry 0 is the sentinel position 0, entry
//               i + 1 is seed i's position packed as
//               ((y + kOff) << 16) | (x + kOff).  The sentinel stands for
//               (-kOff, -kOff), farther from every pixel than any seed.
//   label map   row-major uint32[width * height]; 0 marks an unclaimed
//               pixel in both modes.
//               ID labels: seed index + 1 (an index into the seed table).
//               XY labels: the seed's packed position.
// The smaller internal label still wins a tie: index + 1 orders like the
// index, and the packed position orders like (y << 16) | x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vd {

constexpr uint32_t kOff = 16384;          // added to x and y before packing
constexpr uint32_t kEmpty = 0u;           // unclaimed pixel, both modes

enum Label { kLabelId = 0, kLabelXy = 1 };
enum Metric { kEuclid = 0, kManhattan = 1 };

inline uint32_t pack_pos(int32_t x, int32_t y)
{
    return ((uint32_t)(y + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff);
}

// Seed-set state, one byte per seed (a changing seed set: insertion and
// removal).  kPresent: the seed is in the set now; kKept: it has been in
// the set since the current diagram was made; kGone: it was removed since
// then (host bookkeeping; kernels ignore it).  Launchers take a null state
// when every seed is present and kept.
constexpr uint32_t kPresent = 1u;
constexpr uint32_t kKept = 2u;
constexpr uint32_t kGone = 4u;

// map[0 .. n) = value.
hipError_t launch_fill(uint32_t *map, int64_t n, uint32_t value, hipStream_t s);

// Seed pixels (Sec. III, flood starting points) of the present seeds;
// `table` is the seed table (sentinel first).  ID labels take the lowest
// index among coincident seeds, in one launch of compare-and-swap loops
// that replace the labels left from the previous step (see k_splat_swap).
// XY labels write the pixel's own packed position.
hipError_t launch_splat_id(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                           const uint8_t *state, hipStream_t s);
hipError_t launch_splat_xy(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                           const uint8_t *state, hipStream_t s);
// The same with the top bit set (a seed pixel of this step, over the
// previous diagram: see launch_flood_seeds).
hipError_t launch_splat_xy_marked(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                                  const uint8_t *state, hipStream_t s);
// The ID splat on a map filled with all ones (a JFA step's start): the
// atomic minimum alone.  All ones is no label: it indexes past the seed
// table, whose answer is the sentinel position, so the flood passes treat
// such pixels exactly as unclaimed ones (and a JFA step claims every pixel).
hipError_t launch_splat_id_over_ones(uint32_t *map, const uint32_t *table, int32_t S,
                                     int32_t W, const uint8_t *state, hipStream_t s);

// Uniform random integer moves of every present seed, clamped to the grid.
// With disp (two device words) non-null, disp[0] then grows by the move's
// largest per-axis displacement.
hipError_t launch_move(uint32_t *table, int32_t S, int32_t W, int32_t H, uint64_t move_seed,
                       int64_t t, int32_t lo, int32_t hi, const uint8_t *state, uint32_t *disp,
                       hipStream_t s);

// Seeds moved to the S packed positions in `staged` (device memory); disp
// as for launch_move (present seeds only).  `parked` (ID labels, else null)
// receives the positions of absent seeds.
hipError_t launch_set_seeds(uint32_t *table, const uint32_t *staged, int32_t S,
                            const uint8_t *state, uint32_t *parked, uint32_t *disp, hipStream_t s);

// Seed table (S + 1 entries, sentinel first) and state bytes (S) from S
// (x, y) int32 pairs in device memory; seeds off the grid take no part.
hipError_t launch_pack_positions(uint32_t *table, uint8_t *state, const int32_t *xy, int32_t S,
                                 int32_t W, int32_t H, hipStream_t s);

// Inserted seeds: n (index, packed position) pairs staged in device memory.
hipError_t launch_place(uint32_t *table, const uint32_t *staged, int32_t n, hipStream_t s);

// Removed seeds with ID labels (n indices staged in device memory): the
// position is kept in parked[i], the table entry becomes the sentinel.
hipError_t launch_park(uint32_t *table, uint32_t *parked, const uint32_t *ids, int32_t n,
                       hipStream_t s);

// ID labels of seeds without kKept become unclaimed (state: S bytes; the
// map's n pixels, 16-byte aligned).
hipError_t launch_purge(uint32_t *map, const uint8_t *state, int32_t S, int64_t n,
                        hipStream_t s);

// *count = number of unclaimed pixels of map[0 .. n) (16-byte aligned):
// label 0, or with state (S bytes) non-null, ID labels of seeds without
// kPresent.
hipError_t launch_count_unclaimed(const uint32_t *map, int64_t n, const uint8_t *state,
                                  int32_t S, uint32_t *count, hipStream_t s);

// After a step: present seeds become kept, absent ones lose kKept.
hipError_t launch_settle(uint8_t *state, int32_t S, hipStream_t s);

// XY labels after a move.  idx[old position] = new position of the lowest
// kept seed that sat there, all ones if none did (old_table: the positions
// the map refers to, table: the current ones, both sentinel first); then
// every label, an old position, becomes idx of it (unclaimed for all
// ones).  idx is a width*height scratch map; only entries at old positions
// are written or read.
hipError_t launch_index_old(uint32_t *idx, const uint32_t *old_table, const uint32_t *table,
                            int32_t S, int32_t W, const uint8_t *state, hipStream_t s);
hipError_t launch_relabel(uint32_t *map, const uint32_t *idx, int32_t W, int32_t H,
                          hipStream_t s);
// The single-launch old-position index (index_mark_seed): 32-bit entries of
// a 3-bit epoch, a 21-bit label and an 8-bit move code.
constexpr uint32_t kIndexNoLabel = 0x1FFFFFu;   // label field: no kept seed
constexpr int kIndexEpochs = 8;                 // epoch values before a refill
constexpr int kIndexMaxReach = 7;               // largest move per axis it encodes

// The single-launch form of launch_index_old for a dJFA step whose first
// pass reads through the index (launch_flood_relabel): idx (a width*height
// map of its own) is filled with all ones when it is carved out and again
// every kIndexEpochs builds; `epoch` is kIndexEpochs - 1 minus the builds
// since that fill.  Each seed marks its old position with one atomic
// minimum, and present seeds mark their pixels of this step in `map` with
// the top bit set (a seed pixel of this step, which the first pass takes as
// it is).  Needs S + 1 < kIndexNoLabel, and no kept seed more than
// kIndexMaxReach pixels per axis from the position the diagram refers to.
hipError_t launch_index_marked(uint32_t *idx, uint32_t *map, const uint32_t *old_table,
                               const uint32_t *table, int32_t S, int32_t W, const uint8_t *state,
                               uint32_t epoch, hipStream_t s);

// Internal labels to the external encoding of include/vdflood.h.
hipError_t launch_export(const uint32_t *map, uint32_t *out, int64_t n, int32_t label,
                         hipStream_t s);

// Tile decomposition of one flood pass: ncol column tiles of 256 x
// min(k, H) chains (rows congruent mod k) x nseg segments of at most L rows,
// numbered chain-major, column-minor; nblocks tiles in all.
struct FloodGrid {
    uint32_t ncol, nseg;
    int32_t L;
    uint32_t nblocks;
};

// Grid of a pass at step k >= 1 on a W x H map with segments of seg_rows
// rows (<= 0: chosen from the map size); nblocks == 0 if too large.
constexpr int kMaxTunedSegRows = 128;
FloodGrid flood_grid(int32_t W, int32_t H, int32_t k, int32_t seg_rows);

// Work items of a persistent (batched or served) pass: tiles of 32-row
// segments (the batch gives parallelism, so segments need not be short) --
// four-column tiles of 1024 columns where quad_ok(W, k), else one-column
// tiles of 256 -- grouped so that one item covers about 8192 output pixels
// even where chains are short (large k).  Item i covers tiles
// [i*per, (i+1)*per).
struct ItemGrid {
    FloodGrid g;
    uint32_t per;      // tiles per item
    uint32_t items;
    int32_t quad;      // tiles of the four-column kernels (flood_grid_quad)
};
ItemGrid item_grid(int32_t W, int32_t H, int32_t k);

// Largest step the shared-row (LDS) kernels handle: one column per lane,
// and four columns per lane (ID labels; two row sizes, the wider one for
// steps above kMaxLdsStep).
constexpr int kMaxLdsStep = 128;
constexpr int kMaxQuadLdsStep = 512;

// Grid of the four-columns-per-lane kernels (1024 columns per workgroup),
// and whether they handle a pass: width a multiple of 4 and k = 1, 2 or a
// multiple of 4.
FloodGrid flood_grid_quad(int32_t W, int32_t H, int32_t k, int32_t seg_rows);
bool quad_ok(int32_t W, int32_t k);

// One flood pass at step k: dst[p] = best of src[p] and src[p + o] over the
// Moore (vn == 0) or Von Neumann (vn != 0) offsets o at distance k.
// `variant` (0 .. kFloodVariants - 1) selects the kernel; every variant
// gives the same map.  0, 1, 2: the chain walk requesting loads 1, 2 or 3
// rows ahead; 3: rows shared through LDS for k <= 128 (2 rows ahead),
// otherwise variant 1; 4, 5: four columns per lane where quad_ok holds (ID
// labels: rows shared through LDS for k <= 512, direct loads above),
// requesting rows 2 (4) or 3 (5) rows ahead, otherwise variant 3 (ID) or 1
// (XY); at a step of at least a quarter of both sides (block_ok: a step's
// first two passes when it starts at k1) both run one lane per 2 x 2 or
// 4 x 4 block of groups, which reads and writes every pixel once; at other
// steps of 128 and up whose column classes (columns congruent mod k) fit 16
// lanes of 2 or 4 groups (class_groups), variant 4 gives lanes whole classes
// and swaps their end groups over DPP, so no row is shared through LDS and
// no label is looked up twice.  Variants 6-11 are 0-5 with
// non-temporal stores of the output map.
constexpr int kFloodVariants = 12;
hipError_t launch_flood(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                        int32_t W, int32_t H, int32_t k, int32_t vn, int32_t label,
                        int32_t metric, int32_t variant, int32_t seg_rows, hipStream_t s);

// The first pass of an XY-label JFA step on the previous diagram instead of
// a filled map: src holds the previous diagram with this step's seed pixels
// splatted with the top bit set (launch_splat_xy_marked); only those count
// as claimed, so dst equals the pass on the filled and splatted map.  The
// block tile runs it (flood_seeds_ok(W, H, k): widths and k multiples of 4,
// k at least a quarter of both sides, as at a step's first pass); `variant`
// picks only the store policy.
bool flood_seeds_ok(int32_t W, int32_t H, int32_t k);
hipError_t launch_flood_seeds(const uint32_t *src, uint32_t *dst, int32_t W, int32_t H, int32_t k,
                              int32_t vn, int32_t metric, int32_t variant, hipStream_t s);

// The first two passes of a step (k, then k / 2, both Moore) in one
// launch: where both sides are at most 2 k, the width is a
// multiple of 4 and k of 8 (flood_pair_ok), every candidate of both passes
// for a pixel lies in one 4 x 4 block of four-column groups at spacing
// k / 2, which a lane loads once.  With seeds (XY labels), the first pass
// reads as launch_flood_seeds does.  dst equals the two passes run one after
// the other (through a map in between).
bool flood_pair_ok(int32_t W, int32_t H, int32_t k);
hipError_t launch_flood_pair(const uint32_t *src, uint32_t *dst, const uint32_t *table,
                             int32_t S, int32_t W, int32_t H, int32_t k, int32_t label,
                             bool seeds, int32_t metric, bool nt, hipStream_t s);

// The first pass of an XY-label dJFA step, reading the previous diagram
// through the old-position index instead of after a relabel pass: src holds
// old positions (and this step's seed pixels, marked with the top bit by
// launch_index_marked), idx is the index that launch built.  dst equals the
// pass run on the relabelled
// and splatted map.  Available where relabel_fold_ok(W, k) holds (width a
// multiple of 4, k a multiple of 4 up to kMaxQuadLdsStep); `variant` picks
// the rows in flight and the store policy as for launch_flood.
bool relabel_fold_ok(int32_t W, int32_t k);
hipError_t launch_flood_relabel(const uint32_t *src, uint32_t *dst, const uint32_t *idx,
                                int32_t W, int32_t H, int32_t k, int32_t vn, int32_t metric,
                                int32_t variant, int32_t seg_rows, hipStream_t s);

// The last n passes of a step in one launch (tiles in LDS, see vd_tail.h):
// steps ks[0..n) (each 1, 2 or 4, in pass order, summing to at most
// kTailHalo) with Von Neumann flags vns; 2 <= n <= kTailMaxPasses; tiles of
// 48 x th outputs, th = 16, 24 or 32.  Gives the same dst as the n passes
// run one after another.
constexpr int kTailHalo = 8;
constexpr int kTailMaxPasses = 4;
struct TailPlan {
    int32_t n, halo;
    int32_t k[kTailMaxPasses], vn[kTailMaxPasses];
    uint32_t ntx;   // tiles across the map
};
hipError_t launch_flood_tail(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                             int32_t W, int32_t H, const int32_t *ks, const int32_t *vns,
                             int32_t n, int32_t label, int32_t metric, bool nt, int32_t th,
                             hipStream_t s);

}  // namespace vd
