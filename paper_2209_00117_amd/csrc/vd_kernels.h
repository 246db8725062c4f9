// Launch helpers of the vdflood kernels (internal to the library).
//
// Device data layout:
//   label map   row-major uint32[width * height]; ID labels or packed
//               (y << 16) | x positions; kEmpty marks an unclaimed pixel.
//   seed table  uint32[S], position of seed i packed as (y << 16) | x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vd {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;

enum Label { kLabelId = 0, kLabelXy = 1 };
enum Metric { kEuclid = 0, kManhattan = 1 };

// map[0 .. n) = value.
hipError_t launch_fill(uint32_t *map, int64_t n, uint32_t value, hipStream_t s);

// Seed pixels (Sec. III, flood starting points).  ID labels take the lowest
// index among coincident seeds in two launches: reset the seed pixels to
// kEmpty, then an unsigned atomic minimum of the indices.  XY labels write
// the pixel's own position.
hipError_t launch_splat_reset(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                              hipStream_t s);
hipError_t launch_splat_min(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                            hipStream_t s);
hipError_t launch_splat_xy(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                           hipStream_t s);

// Uniform random integer moves of every seed, clamped to the grid.
hipError_t launch_move(uint32_t *pos, int32_t S, int32_t W, int32_t H, uint64_t move_seed,
                       int64_t t, int32_t lo, int32_t hi, hipStream_t s);

// XY labels after a move: idx[old position of seed i] = lowest such i, then
// every label (an old position) becomes the new position of that seed.
// idx is a width*height scratch map; only entries at old positions are read.
hipError_t launch_index_old(uint32_t *idx, const uint32_t *pos_old, int32_t S, int32_t W,
                            hipStream_t s);
hipError_t launch_relabel(uint32_t *map, const uint32_t *idx, const uint32_t *pos_new,
                          int32_t S, int32_t W, int32_t H, hipStream_t s);

// One flood pass at step k: dst[p] = best of src[p] and src[p + o] over the
// Moore (vn == 0) or Von Neumann (vn != 0) offsets o at distance k.
hipError_t launch_flood(const uint32_t *src, uint32_t *dst, const uint32_t *pos, int32_t W,
                        int32_t H, int32_t k, int32_t vn, int32_t label, int32_t metric,
                        hipStream_t s);

}  // namespace vd
