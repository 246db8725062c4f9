// Device pieces shared by the launches that serve many simulations at once
// (batched time steps and the serving loop's pass-level ticks): the flood
// tiles of one simulation's pass, chosen as a lone simulation's kernels
// would be, and the claiming of work items from a tick-or-level work list.
#pragma once

#include "vd_quad.h"

namespace vd {

namespace {

// One simulation's pass inside a persistent launch.  `quad`: tiles of the
// four-column kernels (width a multiple of 4, k = 1, 2 or a multiple of 4;
// g from flood_grid_quad), else of the one-column kernels (g from
// flood_grid).  Every field is wave-uniform.
struct MemberPass {
    const uint32_t *src;
    uint32_t *dst;
    const uint32_t *table;
    int32_t W, H, S, k, vn, label, quad;
    FloodGrid g;
};

// Shared memory of a persistent flood launch: the largest of the tiles'
// row buffers (two wide four-column rows).
constexpr size_t kMultiLds = 2 * sizeof(QuadRowWide);

// Tiles [t0, t1) of one simulation's pass, with the tile functions of the
// single-simulation kernels (rows requested two ahead, ordinary stores):
// four-column tiles where the pass allows them (ID labels: rows shared
// through LDS up to k = 512, direct loads above; XY labels: direct loads),
// one-column tiles otherwise (ID labels: rows shared through LDS up to
// k = 128, the chain walk above; XY labels: the chain walk).  A barrier
// separates consecutive tiles (their LDS rows).
template <int METRIC, int VN>
__device__ __forceinline__ void member_tiles_vn(const MemberPass &mp, uint32_t t0, uint32_t t1,
                                                uint8_t *lds)
{
    const i32x4 tab = table_rsrc(mp.table, (uint32_t)mp.S);
    const int32_t W = mp.W, H = mp.H, k = mp.k;
    for (uint32_t tile = t0; tile < t1; ++tile) {
        if (tile != t0) __syncthreads();
        if (mp.quad) {
            if (mp.label == kLabelId) {
                const TableLookup lk{tab};
                if (k > kMaxQuadLdsStep)
                    flood_quad_id_direct_tile<METRIC, VN, 3, 0>(mp.src, mp.dst, tab, W, H, k, mp.g,
                                                                tile);
                else if (k > kMaxLdsStep)
                    flood_quad_id_tile<METRIC, VN, 0, 3, 0>(mp.src, mp.dst, lk, W, H, k, mp.g,
                                                            tile, (QuadRowWide *)lds);
                else if (k == 1)
                    flood_quad_id_tile<METRIC, VN, 1, 3, 0>(mp.src, mp.dst, lk, W, H, k, mp.g,
                                                            tile, (QuadRow *)lds);
                else if (k == 2)
                    flood_quad_id_tile<METRIC, VN, 2, 3, 0>(mp.src, mp.dst, lk, W, H, k, mp.g,
                                                            tile, (QuadRow *)lds);
                else
                    flood_quad_id_tile<METRIC, VN, 0, 3, 0>(mp.src, mp.dst, lk, W, H, k, mp.g,
                                                            tile, (QuadRow *)lds);
            } else {
                if (k == 1)
                    flood_quad_xy_tile<METRIC, VN, 1, 3, 0>(mp.src, mp.dst, W, H, k, mp.g, tile);
                else if (k == 2)
                    flood_quad_xy_tile<METRIC, VN, 2, 3, 0>(mp.src, mp.dst, W, H, k, mp.g, tile);
                else
                    flood_quad_xy_tile<METRIC, VN, 0, 3, 0>(mp.src, mp.dst, W, H, k, mp.g, tile);
            }
        } else if (mp.label == kLabelId) {
            if (k <= kMaxLdsStep)
                flood_lds_tile<kLabelId, METRIC, VN, 2>(mp.src, mp.dst, tab, W, H, k, mp.g, tile,
                                                        (uint2(*)[kLdsRow])lds);
            else
                flood_chain_tile<kLabelId, METRIC, VN, 2>(mp.src, mp.dst, tab, W, H, k, mp.g,
                                                          tile);
        } else {
            flood_chain_tile<kLabelXy, METRIC, VN, 2>(mp.src, mp.dst, tab, W, H, k, mp.g, tile);
        }
    }
}

template <int METRIC>
__device__ __forceinline__ void member_tiles(const MemberPass &mp, uint32_t t0, uint32_t t1,
                                             uint8_t *lds)
{
    if (mp.vn)
        member_tiles_vn<METRIC, 1>(mp, t0, t1, lds);
    else
        member_tiles_vn<METRIC, 0>(mp, t0, t1, lds);
}

// The next work item of a persistent launch for this workgroup, or all ones
// once every chunk is drained.  Items [chunk[c], chunk[c + 1]) form XCD c's
// chunk; a workgroup drains its own XCD's chunk first (block b runs on XCD
// b % 8), then helps the others (`probe` counts chunks found empty).  One
// atomic per attempt on the chunk's counter; every attempt either claims an
// item or moves on to the next chunk, so the loop ends after at most eight
// empty chunks.  Called by all threads; the result is wave-uniform.
__device__ __forceinline__ uint32_t claim_item(const uint32_t *chunk, uint32_t *ctr,
                                               uint32_t &probe, uint32_t *s_item)
{
    __syncthreads();   // the previous item's LDS reads and s_item reads are finished
    if (threadIdx.x == 0) {
        const uint32_t home = blockIdx.x & 7u;
        uint32_t item = 0xFFFFFFFFu;
        while (probe < 8u) {
            const uint32_t c = (home + probe) & 7u;
            const uint32_t lo = chunk[c], hi = chunk[c + 1];
            const uint32_t i = lo < hi ? atomicAdd(&ctr[c], 1u) : 0xFFFFFFFFu;
            if (i < hi - lo) {
                item = lo + i;
                break;
            }
            ++probe;
        }
        *s_item = item;
    }
    __syncthreads();
    return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)*s_item);
}

}  // namespace

}  // namespace vd
