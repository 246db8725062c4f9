// vdflood single-simulation kernels for gfx950 (CDNA4, wave64) and their
// launchers.  The flood-pass device code (and the reasoning behind it) is in
// vd_device.h.
#include <type_traits>

#include "vd_device.h"
#include "vd_quad.h"
#include "vd_tail.h"

namespace vd {

namespace {

__global__ void __launch_bounds__(kBlock) k_fill(uint32_t *__restrict__ map, int64_t n,
                                                 uint32_t value)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        map[i] = value;
}

// Seed pixels over whatever they held before, in one launch (see
// splat_swap_seed).  Seed i takes part if part_state has a bit of
// part_need (all seeds for a null part_state).
__global__ void __launch_bounds__(kBlock) k_splat_swap(uint32_t *__restrict__ map,
                                                       const uint32_t *__restrict__ table,
                                                       int32_t S, int32_t W,
                                                       const uint8_t *__restrict__ part_state,
                                                       uint32_t part_need,
                                                       const uint8_t *__restrict__ label_state,
                                                       uint32_t label_need)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S && takes_part(part_state, i, part_need))
        splat_swap_seed(map, table, S, W, i, label_state, label_need);
}

__global__ void __launch_bounds__(kBlock) k_splat_min(uint32_t *__restrict__ map,
                                                      const uint32_t *__restrict__ table,
                                                      int32_t S, int32_t W,
                                                      const uint8_t *__restrict__ state,
                                                      uint32_t need)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S && takes_part(state, i, need)) splat_min_seed(map, table, i, W);
}

// `mark` is or-ed into the written position (0, or the top bit).
__global__ void __launch_bounds__(kBlock) k_splat_xy(uint32_t *__restrict__ map,
                                                     const uint32_t *__restrict__ table,
                                                     int32_t S, int32_t W,
                                                     const uint8_t *__restrict__ state,
                                                     uint32_t mark)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S && takes_part(state, i, kPresent)) splat_xy_seed(map, table, i, W, mark);
}

// Largest per-axis displacement between two packed positions.
__device__ __forceinline__ uint32_t cheb(uint32_t a, uint32_t b)
{
    const int32_t dx = abs((int32_t)(a & 0xFFFFu) - (int32_t)(b & 0xFFFFu));
    const int32_t dy = abs((int32_t)(a >> 16) - (int32_t)(b >> 16));
    return (uint32_t)max(dx, dy);
}

// The wave's largest value into *word (one atomic per wave); every lane of
// the wave must call it.
__device__ __forceinline__ void wave_max_into(uint32_t *word, uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    if ((threadIdx.x & 63u) == 0u && v) atomicMax(word, v);
}

// Seeds absent from the seed set (state) stay where they are.  `disp`
// (optional): disp[1] receives the largest per-axis displacement of this
// move (after clamping).
__global__ void __launch_bounds__(kBlock) k_move(uint32_t *__restrict__ table, int32_t S,
                                                 int32_t W, int32_t H, uint64_t move_seed,
                                                 uint64_t t, int32_t lo, uint32_t span,
                                                 const uint8_t *__restrict__ state,
                                                 uint32_t *__restrict__ disp)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t moved = 0;
    if (i < S && takes_part(state, i, kPresent)) {
        const uint32_t p = move_one(table, i, S, W, H, move_seed, t, lo, span);
        moved = cheb(p, table[i + 1]);
    }
    if (disp) wave_max_into(&disp[1], moved);
}

// Seeds moved to caller-given positions (packed, staged in device memory);
// only present seeds count towards the displacement.  With `parked`
// non-null (ID labels), an absent seed's position goes there: its table
// entry holds the sentinel.
__global__ void __launch_bounds__(kBlock) k_set_seeds(uint32_t *__restrict__ table,
                                                      const uint32_t *__restrict__ staged,
                                                      int32_t S, const uint8_t *__restrict__ state,
                                                      uint32_t *__restrict__ parked,
                                                      uint32_t *__restrict__ disp)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t moved = 0;
    if (i < S) {
        const uint32_t q = staged[i];
        if (takes_part(state, i, kPresent)) {
            moved = cheb(table[i + 1], q);
            table[i + 1] = q;
        } else if (parked) {
            parked[i] = q;
        } else {
            table[i + 1] = q;
        }
    }
    if (disp) wave_max_into(&disp[1], moved);
}

// Inserted seeds: staged[2j] is a seed index, staged[2j + 1] its packed
// position, j < n.
__global__ void __launch_bounds__(kBlock) k_place(uint32_t *__restrict__ table,
                                                  const uint32_t *__restrict__ staged, int32_t n)
{
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) table[staged[2 * j] + 1] = staged[2 * j + 1];
}

// Seed table and seed-set bytes from caller positions (x, y int32 pairs in
// device memory): entry 0 is the sentinel and entry i + 1 seed i's packed
// position; a seed off the grid gets the sentinel and state 0, so it takes
// no part (it is never splatted, and no pixel ever carries its label).
__global__ void __launch_bounds__(kBlock) k_pack_positions(uint32_t *__restrict__ table,
                                                           uint8_t *__restrict__ state,
                                                           const int32_t *__restrict__ xy,
                                                           int32_t S, int32_t W, int32_t H)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) table[0] = 0u;
    if (i < S) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        const bool in = x >= 0 && x < W && y >= 0 && y < H;
        table[i + 1] = in ? ((uint32_t)(y + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff)
                          : 0u;
        state[i] = in ? (uint8_t)(kPresent | kKept) : (uint8_t)0;
    }
}

// Removed seeds (ID labels): the position moves to `parked` and the table
// entry becomes the sentinel position, so every flood pass finds the seed's
// labels farther than any present seed's -- exactly as if they were
// unclaimed pixels (label 0 also reads the sentinel; a tie between the two
// only decides which unclaimed label a pixel holds).
__global__ void __launch_bounds__(kBlock) k_park(uint32_t *__restrict__ table,
                                                 uint32_t *__restrict__ parked,
                                                 const uint32_t *__restrict__ ids, int32_t n)
{
    int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) {
        const uint32_t i = ids[j];
        parked[i] = table[i + 1];
        table[i + 1] = 0u;
    }
}

// Whole-map scans of the seed-set code (purge, unclaimed count): each lane
// takes kScanVec 16-byte vectors, kScanVec * (lanes in the grid) apart,
// and requests them all before using any; a label's state byte is fetched
// only where it differs from the label to its left (the fetch of a reusing
// lane goes to offset -1, which the hardware answers without a memory
// access).  Each 16-byte vector covers four pixels; n & 3 tail pixels are
// handled one per lane.
constexpr int kScanVec = 4;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t bytes_rsrc(const uint8_t *p, int32_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, p ? n : 0, kRsrcWord3);
}

// State bytes of the four labels of v (0 for label 0 and for a label equal
// to its left neighbour; `left` is the label left of v[0]).
__device__ __forceinline__ u32x4 state4(__amdgpu_buffer_rsrc_t sr, const u32x4 &v, uint32_t left)
{
    u32x4 b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t l = v[e], lft = e == 0 ? left : v[e - 1];
        const int32_t at = (l != kEmpty && l != lft) ? (int32_t)l - 1 : -1;
        b[e] = __builtin_amdgcn_raw_buffer_load_b8(sr, at, 0, 0);
    }
    return b;
}

// ID labels of seeds not kept since the diagram was made become unclaimed
// (vectors where nothing changes are not written).
__global__ void __launch_bounds__(kBlock) k_purge(uint32_t *__restrict__ map, int64_t n,
                                                  const uint8_t *__restrict__ state, int32_t S)
{
    const int64_t n4 = n >> 2;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const __amdgpu_buffer_rsrc_t sr = bytes_rsrc(state, S);
    u32x4 *m4 = reinterpret_cast<u32x4 *>(map);
    for (int64_t q0 = g; q0 < n4; q0 += kScanVec * T) {
        u32x4 v[kScanVec];
#pragma unroll
        for (int u = 0; u < kScanVec; ++u) {
            const int64_t q = q0 + u * T;
            v[u] = q < n4 ? m4[q] : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < kScanVec; ++u) {
            const u32x4 b = state4(sr, v[u], kEmpty);
            u32x4 o = v[u];
            bool dirty = false;
            bool gone = false;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // a label equal to its left neighbour shares its verdict
                gone = (e > 0 && v[u][e] == v[u][e - 1]) ? gone
                                                         : (v[u][e] != kEmpty && (b[e] & kKept) == 0u);
                o[e] = gone ? kEmpty : v[u][e];
                dirty = dirty || gone;
            }
            const int64_t q = q0 + u * T;
            if (dirty && q < n4) m4[q] = o;
        }
    }
    const int64_t tail = 4 * n4 + g;
    if (tail < n) {
        const uint32_t l = map[tail];
        if (l != kEmpty && (l > (uint32_t)S || (state[l - 1] & kKept) == 0u)) map[tail] = kEmpty;
    }
}

// *count += the number of unclaimed pixels of map[0 .. n): label 0, or with
// state non-null (ID labels) the label of an absent seed; one atomic per
// wave that found any.
__global__ void __launch_bounds__(kBlock) k_count_unclaimed(const uint32_t *__restrict__ map,
                                                            int64_t n,
                                                            const uint8_t *__restrict__ state,
                                                            int32_t S,
                                                            uint32_t *__restrict__ count)
{
    const int64_t n4 = n >> 2;
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const __amdgpu_buffer_rsrc_t sr = bytes_rsrc(state, S);
    const u32x4 *m4 = reinterpret_cast<const u32x4 *>(map);
    uint32_t c = 0;
    for (int64_t q0 = g; q0 < n4; q0 += kScanVec * T) {
        u32x4 v[kScanVec];
#pragma unroll
        for (int u = 0; u < kScanVec; ++u) {
            const int64_t q = q0 + u * T;
            // past the end: a claimed label (state byte 1 is never fetched for it)
            v[u] = q < n4 ? m4[q] : u32x4{1u, 1u, 1u, 1u};
        }
#pragma unroll
        for (int u = 0; u < kScanVec; ++u) {
            const int64_t q = q0 + u * T;
            if (q >= n4) continue;
            const u32x4 b = state4(sr, v[u], kEmpty);
            uint32_t un = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                un = (e > 0 && v[u][e] == v[u][e - 1])
                         ? un
                         : ((v[u][e] == kEmpty || (state && (b[e] & kPresent) == 0u)) ? 1u : 0u);
                c += un;
            }
        }
    }
    const int64_t tail = 4 * n4 + g;
    if (tail < n) {
        const uint32_t l = map[tail];
        c += (l == kEmpty || (state && (l > (uint32_t)S || (state[l - 1] & kPresent) == 0u)))
                 ? 1u
                 : 0u;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
    if ((threadIdx.x & 63u) == 0u && c) atomicAdd(count, c);
}

// After a step: every present seed is kept from now on, absent ones not.
__global__ void __launch_bounds__(kBlock) k_settle(uint8_t *__restrict__ state, int32_t S)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) state[i] = (state[i] & kPresent) ? (uint8_t)(kPresent | kKept) : (uint8_t)0;
}

// disp[0] += disp[1] (this move's largest displacement), disp[1] = 0.
__global__ void k_disp_acc(uint32_t *__restrict__ disp)
{
    if (threadIdx.x == 0) {
        disp[0] += disp[1];
        disp[1] = 0u;
    }
}

// The old-position index after k_splat_swap (see index_resolve_seed).
__global__ void __launch_bounds__(kBlock) k_index_resolve(uint32_t *__restrict__ idx,
                                                          const uint32_t *__restrict__ old_table,
                                                          const uint32_t *__restrict__ table,
                                                          int32_t S, int32_t W,
                                                          const uint8_t *__restrict__ state)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S && takes_part(state, i, kKept)) index_resolve_seed(idx, old_table, table, i, W);
}

// The single-launch old-position index (see index_mark_seed) and, in the same
// launch, the present seeds' pixels of this step marked in `map`
// (splat_xy_seed with the top bit).
__global__ void __launch_bounds__(kBlock) k_index_mark_splat(
    uint32_t *__restrict__ idx, uint32_t *__restrict__ map,
    const uint32_t *__restrict__ old_table, const uint32_t *__restrict__ table, int32_t S,
    int32_t W, const uint8_t *__restrict__ state, uint32_t epoch)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const uint32_t now = table[i + 1];
    const uint8_t st = state ? state[i] : (uint8_t)(kPresent | kKept);
    index_mark_seed(idx, old_table[i + 1], now, i, W, (st & kKept) != 0u, epoch);
    if (st & kPresent) map[pixel_of(now, W)] = now | kMarked;   // as splat_xy_seed
}

__global__ void __launch_bounds__(kBlock) k_relabel(uint32_t *__restrict__ map,
                                                    const uint32_t *__restrict__ idx,
                                                    int32_t W, int32_t H)
{
    int64_t n = (int64_t)W * H;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
        map[p] = relabel_one(map[p], idx, W, H);
}

// k_relabel for widths divisible by 4 (see relabel_block): workgroup b
// relabels block b of the map.
__global__ void __launch_bounds__(kBlock) k_relabel_deep(uint32_t *__restrict__ map,
                                                         const uint32_t *__restrict__ idx,
                                                         int32_t W, int32_t H, int32_t rows)
{
    relabel_block(map, idx, W, H, rows, blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_export(const uint32_t *__restrict__ map,
                                                   uint32_t *__restrict__ out, int64_t n,
                                                   int32_t label)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t l = map[p];
        // ID: index + 1 -> index, and 0 -> all ones.  XY: strip the offsets.
        out[p] = label == kLabelId ? l - 1u
                                   : (l == kEmpty ? 0xFFFFFFFFu : l - ((kOff << 16) | kOff));
    }
}

template <int LABEL, int METRIC, int VN, int P, int ST>
__global__ void __launch_bounds__(kTW) k_flood(const uint32_t *__restrict__ src,
                                               uint32_t *__restrict__ dst,
                                               const uint32_t *__restrict__ table, uint32_t S,
                                               int32_t W, int32_t H, int32_t k, FloodGrid g)
{
    flood_chain_tile<LABEL, METRIC, VN, P, ST>(src, dst, table_rsrc(table, S), W, H, k, g,
                                           xcd_logical(blockIdx.x, g.nblocks));
}

template <int LABEL, int METRIC, int VN, int P, int ST>
__global__ void __launch_bounds__(kTW) k_flood_lds(const uint32_t *__restrict__ src,
                                                   uint32_t *__restrict__ dst,
                                                   const uint32_t *__restrict__ table,
                                                   uint32_t S, int32_t W, int32_t H, int32_t k,
                                                   FloodGrid g)
{
    __shared__ uint2 lds[2][kLdsRow];
    flood_lds_tile<LABEL, METRIC, VN, P, ST>(src, dst, table_rsrc(table, S), W, H, k, g,
                                         xcd_logical(blockIdx.x, g.nblocks), lds);
}

template <int METRIC, int VN, int KC, int NS, int ST>
__global__ void __launch_bounds__(kBlock) k_flood_quad_xy(const uint32_t *__restrict__ src,
                                                          uint32_t *__restrict__ dst, int32_t W,
                                                          int32_t H, int32_t k, FloodGrid g)
{
    flood_quad_xy_tile<METRIC, VN, KC, NS, ST>(src, dst, W, H, k, g,
                                           xcd_logical(blockIdx.x, g.nblocks));
}

// WIDE: shared rows sized for steps up to kMaxQuadLdsStep.
template <int METRIC, int VN, int KC, int NS, int ST, bool WIDE>
__global__ void __launch_bounds__(kBlock) k_flood_quad_id(const uint32_t *__restrict__ src,
                                                          uint32_t *__restrict__ dst,
                                                          const uint32_t *__restrict__ table,
                                                          uint32_t S, int32_t W, int32_t H,
                                                          int32_t k, FloodGrid g)
{
    using Q = typename std::conditional<WIDE, QuadRowWide, QuadRow>::type;
    __shared__ Q lds[2];
    const TableLookup lk{table_rsrc(table, S)};
    flood_quad_id_tile<METRIC, VN, KC, NS, ST>(src, dst, lk, W, H, k, g,
                                               seg_major(xcd_logical(blockIdx.x, g.nblocks), g),
                                               lds);
}

template <int METRIC, int VN, int NS, int ST>
__global__ void __launch_bounds__(kBlock) k_flood_quad_idd(const uint32_t *__restrict__ src,
                                                           uint32_t *__restrict__ dst,
                                                           const uint32_t *__restrict__ table,
                                                           uint32_t S, int32_t W, int32_t H,
                                                           int32_t k, FloodGrid g)
{
    flood_quad_id_direct_tile<METRIC, VN, NS, ST>(src, dst, table_rsrc(table, S), W, H, k, g,
                                              xcd_logical(blockIdx.x, g.nblocks));
}

// LABEL of k_flood_block for the first pass of an XY JFA step that reads the
// previous diagram with this step's seed pixels marked (SeedMarks).
constexpr int kLabelXySeeds = 2;

// One lane per NB x NB block of four-column groups {x0 + n k} x {y0 + m k}
// (x0 = 4 * the lane's group, y0 = blockIdx.y), for steps with
// block_span(W, H, k) == NB.
template <int NB, int LABEL, int METRIC, int VN, int ST>
__global__ void __launch_bounds__(kBlock) k_flood_block(const uint32_t *__restrict__ src,
                                                        uint32_t *__restrict__ dst,
                                                        const uint32_t *__restrict__ table,
                                                        uint32_t S, int32_t W, int32_t H,
                                                        int32_t k)
{
    const int32_t gx = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (kQuad * gx >= min(k, W)) return;
    if (LABEL == kLabelId)
        flood_block_tile<NB, METRIC, VN, ST>(src, dst, TableLookup{table_rsrc(table, S)}, W, H,
                                             k, gx, (int32_t)blockIdx.y);
    else if (LABEL == kLabelXy)
        flood_block_tile<NB, METRIC, VN, ST>(src, dst, PosLabels{}, W, H, k, gx,
                                             (int32_t)blockIdx.y);
    else   // kLabelXySeeds
        flood_block_tile<NB, METRIC, VN, ST>(src, dst, SeedMarks{}, W, H, k, gx,
                                             (int32_t)blockIdx.y);
}

// The first two passes of a step, k and kh = k / 2, both Moore, in one
// launch (flood_block_pair_tile; pair_ok(W, H, k)): one lane per 4 x 4
// block of groups at spacing kh.
template <int LABEL, int METRIC, int ST>
__global__ void __launch_bounds__(kBlock) k_flood_pair(const uint32_t *__restrict__ src,
                                                       uint32_t *__restrict__ dst,
                                                       const uint32_t *__restrict__ table,
                                                       uint32_t S, int32_t W, int32_t H,
                                                       int32_t kh)
{
    const int32_t gx = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (kQuad * gx >= min(kh, W)) return;
    const int32_t y0 = (int32_t)blockIdx.y;
    if (LABEL == kLabelId)
        flood_block_pair_tile<METRIC, ST>(src, dst, TableLookup{table_rsrc(table, S)}, W, H, kh,
                                          gx, y0);
    else if (LABEL == kLabelXy)
        flood_block_pair_tile<METRIC, ST>(src, dst, PosLabels{}, W, H, kh, gx, y0);
    else   // kLabelXySeeds
        flood_block_pair_tile<METRIC, ST>(src, dst, SeedMarks{}, W, H, kh, gx, y0);
}

// Column-class tiles (see flood_class_tile): G groups per lane, C lanes per
// class.
template <int G, int LABEL, int METRIC, int VN, int ST>
__global__ void __launch_bounds__(kBlock) k_flood_class(const uint32_t *__restrict__ src,
                                                        uint32_t *__restrict__ dst,
                                                        const uint32_t *__restrict__ table,
                                                        uint32_t S, int32_t W, int32_t H,
                                                        int32_t k, int32_t C, FloodGrid g)
{
    const uint32_t logical = xcd_logical(blockIdx.x, g.nblocks);
    if (LABEL == kLabelId)
        flood_class_tile<G, METRIC, VN, 3, ST>(src, dst, TableLookup{table_rsrc(table, S)}, W, H,
                                               k, C, g, seg_major(logical, g));
    else
        flood_class_tile<G, METRIC, VN, 3, ST>(src, dst, PosLabels{}, W, H, k, C, g, logical);
}

template <int LABEL, int METRIC, int ST, int TH>
__global__ void __launch_bounds__(kBlock) k_flood_tail(const uint32_t *__restrict__ src,
                                                       uint32_t *__restrict__ dst,
                                                       const uint32_t *__restrict__ table,
                                                       uint32_t S, int32_t W, int32_t H,
                                                       TailPlan plan)
{
    __shared__ TailBuf<TH> buf[2];
    flood_tail_tile<LABEL, METRIC, ST, TH>(src, dst, table, S, W, H, plan,
                                           xcd_logical(blockIdx.x, gridDim.x), buf);
}

inline dim3 grid1d(int64_t n, int64_t cap = 1 << 20)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return dim3((unsigned)b);
}

}  // namespace

hipError_t launch_fill(uint32_t *map, int64_t n, uint32_t value, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, grid1d(n, 8192), dim3(kBlock), 0, s, map, n, value);
    return hipGetLastError();
}


hipError_t launch_splat_id(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                           const uint8_t *state, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_swap, grid1d(S), dim3(kBlock), 0, s, map, table, S, W, state,
                       (uint32_t)kPresent, state, (uint32_t)kPresent);
    return hipGetLastError();
}

hipError_t launch_splat_id_over_ones(uint32_t *map, const uint32_t *table, int32_t S,
                                     int32_t W, const uint8_t *state, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_min, grid1d(S), dim3(kBlock), 0, s, map, table, S, W, state,
                       kPresent);
    return hipGetLastError();
}

hipError_t launch_splat_xy(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                           const uint8_t *state, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_xy, grid1d(S), dim3(kBlock), 0, s, map, table, S, W, state, 0u);
    return hipGetLastError();
}

hipError_t launch_splat_xy_marked(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                                  const uint8_t *state, hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_xy, grid1d(S), dim3(kBlock), 0, s, map, table, S, W, state,
                       kMarked);
    return hipGetLastError();
}

hipError_t launch_move(uint32_t *table, int32_t S, int32_t W, int32_t H, uint64_t move_seed,
                       int64_t t, int32_t lo, int32_t hi, const uint8_t *state, uint32_t *disp,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_move, grid1d(S), dim3(kBlock), 0, s, table, S, W, H, move_seed,
                       (uint64_t)t, lo, (uint32_t)(hi - lo + 1), state, disp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !disp) return e;
    hipLaunchKernelGGL(k_disp_acc, dim3(1), dim3(64), 0, s, disp);
    return hipGetLastError();
}

hipError_t launch_set_seeds(uint32_t *table, const uint32_t *staged, int32_t S,
                            const uint8_t *state, uint32_t *parked, uint32_t *disp, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_seeds, grid1d(S), dim3(kBlock), 0, s, table, staged, S, state,
                       parked, disp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !disp) return e;
    hipLaunchKernelGGL(k_disp_acc, dim3(1), dim3(64), 0, s, disp);
    return hipGetLastError();
}

hipError_t launch_pack_positions(uint32_t *table, uint8_t *state, const int32_t *xy, int32_t S,
                                 int32_t W, int32_t H, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_positions, grid1d(S), dim3(kBlock), 0, s, table, state, xy, S, W, H);
    return hipGetLastError();
}

hipError_t launch_place(uint32_t *table, const uint32_t *staged, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, grid1d(n), dim3(kBlock), 0, s, table, staged, n);
    return hipGetLastError();
}

hipError_t launch_park(uint32_t *table, uint32_t *parked, const uint32_t *ids, int32_t n,
                       hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_park, grid1d(n), dim3(kBlock), 0, s, table, parked, ids, n);
    return hipGetLastError();
}

namespace {

// Grid of a whole-map scan: one round of kScanVec vectors per lane where
// the map allows, at most 8192 workgroups, and every tail pixel covered.
dim3 scan_grid(int64_t n)
{
    const int64_t per_block = (int64_t)kBlock * kScanVec;
    int64_t blocks = ((n >> 2) + per_block - 1) / per_block;
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(blocks, 1), 8192));
}

}  // namespace

hipError_t launch_purge(uint32_t *map, const uint8_t *state, int32_t S, int64_t n,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_purge, scan_grid(n), dim3(kBlock), 0, s, map, n, state, S);
    return hipGetLastError();
}

hipError_t launch_count_unclaimed(const uint32_t *map, int64_t n, const uint8_t *state,
                                  int32_t S, uint32_t *count, hipStream_t s)
{
    hipError_t e = launch_fill(count, 1, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_unclaimed, scan_grid(n), dim3(kBlock), 0, s, map, n, state, S,
                       count);
    return hipGetLastError();
}

hipError_t launch_settle(uint8_t *state, int32_t S, hipStream_t s)
{
    hipLaunchKernelGGL(k_settle, grid1d(S), dim3(kBlock), 0, s, state, S);
    return hipGetLastError();
}

hipError_t launch_index_old(uint32_t *idx, const uint32_t *old_table, const uint32_t *table,
                            int32_t S, int32_t W, const uint8_t *state, hipStream_t s)
{
    // every seed marks its old position (a label may name a seed not kept):
    // with the lowest kept label there, else with all ones
    hipLaunchKernelGGL(k_splat_swap, grid1d(S), dim3(kBlock), 0, s, idx, old_table, S, W,
                       (const uint8_t *)nullptr, 0u, state, (uint32_t)kKept);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_index_resolve, grid1d(S), dim3(kBlock), 0, s, idx, old_table, table, S,
                       W, state);
    return hipGetLastError();
}

hipError_t launch_index_marked(uint32_t *idx, uint32_t *map, const uint32_t *old_table,
                               const uint32_t *table, int32_t S, int32_t W, const uint8_t *state,
                               uint32_t epoch, hipStream_t s)
{
    if (S + 1 >= (int32_t)kIndexNoLabel || epoch >= (uint32_t)kIndexEpochs)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_index_mark_splat, grid1d(S), dim3(kBlock), 0, s, idx, map, old_table,
                       table, S, W, state, epoch);
    return hipGetLastError();
}

hipError_t launch_relabel(uint32_t *map, const uint32_t *idx, int32_t W, int32_t H,
                          hipStream_t s)
{
    if (W % kQuad == 0) {
        hipLaunchKernelGGL(k_relabel_deep, dim3((unsigned)relabel_blocks(W, H)), dim3(kBlock), 0,
                           s, map, idx, W, H, kRelabelBlockRows);
    } else {
        hipLaunchKernelGGL(k_relabel, grid1d((int64_t)W * H, 8192), dim3(kBlock), 0, s, map,
                           idx, W, H);
    }
    return hipGetLastError();
}

hipError_t launch_export(const uint32_t *map, uint32_t *out, int64_t n, int32_t label,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_export, grid1d(n, 8192), dim3(kBlock), 0, s, map, out, n, label);
    return hipGetLastError();
}

namespace {

// Segment length (seg_rows <= 0): long enough to amortise the two overlap
// rows, short enough to give the 256 CUs about `blocks` workgroups.
FloodGrid grid_of(int32_t W, int32_t H, int32_t k, int32_t seg_rows, int32_t tw, int64_t blocks)
{
    FloodGrid g{};
    int64_t npix = (int64_t)W * H;
    int32_t L = (int32_t)(npix / ((int64_t)tw * blocks));
    L = L < 1 ? 1 : (L > kMaxSegRows ? kMaxSegRows : L);
    if (seg_rows > 0) L = seg_rows < kMaxTunedSegRows ? seg_rows : kMaxTunedSegRows;
    uint32_t nres = (uint32_t)(k < H ? k : H);
    int32_t chain = (H + k - 1) / k;                      // rows on the longest chain
    g.ncol = (uint32_t)((W + tw - 1) / tw);
    g.nseg = (uint32_t)((chain + L - 1) / L);
    g.L = L;
    uint64_t nb = (uint64_t)g.ncol * nres * g.nseg;
    g.nblocks = (k < 1 || nb > 0x7FFFFFFFull) ? 0u : (uint32_t)nb;
    return g;
}

}  // namespace

FloodGrid flood_grid(int32_t W, int32_t H, int32_t k, int32_t seg_rows)
{
    return grid_of(W, H, k, seg_rows, kTW, 2048);
}

FloodGrid flood_grid_quad(int32_t W, int32_t H, int32_t k, int32_t seg_rows)
{
    return grid_of(W, H, k, seg_rows, kTWQ, 1024);
}

bool quad_ok(int32_t W, int32_t k)
{
    return W % kQuad == 0 && (k == 1 || k == 2 || k % kQuad == 0);
}

ItemGrid item_grid(int32_t W, int32_t H, int32_t k)
{
    ItemGrid it{};
    it.quad = quad_ok(W, k) ? 1 : 0;
    it.g = it.quad ? flood_grid_quad(W, H, k, kMaxSegRows) : flood_grid(W, H, k, kMaxSegRows);
    if (it.g.nblocks == 0) return it;
    const int64_t chain = (H + k - 1) / k;
    const int64_t rows = chain < it.g.L ? chain : it.g.L;
    const int64_t tile_px = (int64_t)(it.quad ? kTWQ : kTW) * rows;
    it.per = (uint32_t)((8192 + tile_px - 1) / tile_px);
    it.items = (it.g.nblocks + it.per - 1) / it.per;
    return it;
}

namespace {

// Variants 0-5 with store cache policy ST.
template <int ST>
hipError_t launch_flood_st(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                           int32_t W, int32_t H, int32_t k, int32_t vn, int32_t label,
                           int32_t metric, int32_t variant, int32_t seg_rows, hipStream_t s)
{
    uint32_t uS = (uint32_t)S;
    if (label == kLabelXySeeds && !block_ok(W, H, k)) return hipErrorInvalidValue;
    if ((variant >= 4 || label == kLabelXySeeds) && block_ok(W, H, k)) {
        // every pixel's candidates in one block of 2 x 2 or 4 x 4 groups per lane
        const int32_t gx = std::min(k, W) / kQuad;
        const dim3 grid((unsigned)((gx + kBlock - 1) / kBlock), (unsigned)std::min(k, H));
        const bool two = block_span(W, H, k) == 2;
#define VD_BLOCK(LB, MT, V)                                                                    \
    do {                                                                                       \
        if (two)                                                                               \
            hipLaunchKernelGGL((k_flood_block<2, LB, MT, V, ST>), grid, dim3(kBlock), 0, s, src,  \
                               dst, table, uS, W, H, k);                                       \
        else                                                                                   \
            hipLaunchKernelGGL((k_flood_block<4, LB, MT, V, ST>), grid, dim3(kBlock), 0, s, src,  \
                               dst, table, uS, W, H, k);                                       \
    } while (0)
#define VD_BLOCK_M(LB)                                                                         \
    do {                                                                                       \
        if (metric == kEuclid) {                                                               \
            if (vn) VD_BLOCK(LB, kEuclid, 1); else VD_BLOCK(LB, kEuclid, 0);                   \
        } else {                                                                               \
            if (vn) VD_BLOCK(LB, kManhattan, 1); else VD_BLOCK(LB, kManhattan, 0);             \
        }                                                                                      \
    } while (0)
        if (label == kLabelId)
            VD_BLOCK_M(kLabelId);
        else if (label == kLabelXy)
            VD_BLOCK_M(kLabelXy);
        else
            VD_BLOCK_M(kLabelXySeeds);
#undef VD_BLOCK_M
#undef VD_BLOCK
        return hipGetLastError();
    }
    if (variant == 4 && k >= kClassMinStep && class_groups(W, k) > 0) {
        // whole column classes per group of lanes, neighbours over DPP
        const int32_t G = class_groups(W, k), C = class_lanes(W, k, G);
        FloodGrid g = flood_grid_quad(W, H, k, seg_rows);
        const uint64_t nb = (uint64_t)class_blocks(k, C) * (uint64_t)std::min(k, H) * g.nseg;
        if (nb == 0 || nb > 0x7FFFFFFFull) return hipErrorInvalidValue;
        g.ncol = (uint32_t)class_blocks(k, C);
        g.nblocks = (uint32_t)nb;
        const dim3 grid(g.nblocks), block(kBlock);
#define VD_CLASS(LB, MT, V)                                                                    \
    do {                                                                                       \
        if (G == 2)                                                                            \
            hipLaunchKernelGGL((k_flood_class<2, LB, MT, V, ST>), grid, block, 0, s, src, dst,    \
                               table, uS, W, H, k, C, g);                                      \
        else                                                                                   \
            hipLaunchKernelGGL((k_flood_class<4, LB, MT, V, ST>), grid, block, 0, s, src, dst,    \
                               table, uS, W, H, k, C, g);                                      \
    } while (0)
#define VD_CLASS_M(LB)                                                                         \
    do {                                                                                       \
        if (metric == kEuclid) {                                                               \
            if (vn) VD_CLASS(LB, kEuclid, 1); else VD_CLASS(LB, kEuclid, 0);                   \
        } else {                                                                               \
            if (vn) VD_CLASS(LB, kManhattan, 1); else VD_CLASS(LB, kManhattan, 0);             \
        }                                                                                      \
    } while (0)
        if (label == kLabelId) VD_CLASS_M(kLabelId); else VD_CLASS_M(kLabelXy);
#undef VD_CLASS_M
#undef VD_CLASS
        return hipGetLastError();
    }
    if (variant >= 4) {
        if (!quad_ok(W, k)) {
            variant = label == kLabelId ? 3 : 1;   // same labels, single-column kernels
        } else {
            FloodGrid g = flood_grid_quad(W, H, k, seg_rows);
            if (g.nblocks == 0) return hipErrorInvalidValue;
            dim3 grid(g.nblocks), block(kBlock);
#define VD_QUAD(MT, V, KC, NS)                                                                 \
    do {                                                                                       \
        if (label == kLabelId && k > kMaxQuadLdsStep)                                          \
            hipLaunchKernelGGL((k_flood_quad_idd<MT, V, NS, ST>), grid, block, 0, s, src, dst,       \
                               table, uS, W, H, k, g);                                         \
        else if (label == kLabelId && k > kMaxLdsStep)                                         \
            hipLaunchKernelGGL((k_flood_quad_id<MT, V, 0, NS, ST, true>), grid, block, 0, s, src,    \
                               dst, table, uS, W, H, k, g);                                    \
        else if (label == kLabelId)                                                            \
            hipLaunchKernelGGL((k_flood_quad_id<MT, V, KC, NS, ST, false>), grid, block, 0, s, src,  \
                               dst, table, uS, W, H, k, g);                                    \
        else                                                                                   \
            hipLaunchKernelGGL((k_flood_quad_xy<MT, V, KC, NS, ST>), grid, block, 0, s, src, dst, W, \
                               H, k, g);                                                       \
    } while (0)
#define VD_QUAD_NS(MT, V, KC)                                                                  \
    do {                                                                                       \
        if (variant == 4) VD_QUAD(MT, V, KC, 3); else VD_QUAD(MT, V, KC, 4);                   \
    } while (0)
#define VD_QUAD_K(MT, V)                                                                       \
    do {                                                                                       \
        if (k == 1) VD_QUAD_NS(MT, V, 1);                                                      \
        else if (k == 2) VD_QUAD_NS(MT, V, 2);                                                 \
        else VD_QUAD_NS(MT, V, 0);                                                             \
    } while (0)
            if (metric == kEuclid) {
                if (vn) VD_QUAD_K(kEuclid, 1); else VD_QUAD_K(kEuclid, 0);
            } else {
                if (vn) VD_QUAD_K(kManhattan, 1); else VD_QUAD_K(kManhattan, 0);
            }
#undef VD_QUAD_K
#undef VD_QUAD_NS
#undef VD_QUAD
            return hipGetLastError();
        }
    }
    FloodGrid g = flood_grid(W, H, k, seg_rows);
    if (g.nblocks == 0) return hipErrorInvalidValue;
    dim3 grid(g.nblocks), block(kTW);
#define VD_LAUNCH(LB, MT, V, P)                                                              \
    hipLaunchKernelGGL((k_flood<LB, MT, V, P, ST>), grid, block, 0, s, src, dst, table, uS, W, H,  \
                       k, g)
#define VD_LAUNCH_LDS(LB, MT, V, P)                                                           \
    hipLaunchKernelGGL((k_flood_lds<LB, MT, V, P, ST>), grid, block, 0, s, src, dst, table, uS, W,  \
                       H, k, g)
#define VD_LAUNCH_P(LB, MT, V)                                                                \
    do {                                                                                      \
        if (variant == 0) VD_LAUNCH(LB, MT, V, 1);                                            \
        else if (variant == 1 || (variant == 3 && k > kMaxLdsStep)) VD_LAUNCH(LB, MT, V, 2);     \
        else if (variant == 2) VD_LAUNCH(LB, MT, V, 3);                                       \
        else VD_LAUNCH_LDS(LB, MT, V, 2);                                                     \
    } while (0)
    if (label == kLabelId) {
        if (metric == kEuclid) {
            if (vn) VD_LAUNCH_P(kLabelId, kEuclid, 1); else VD_LAUNCH_P(kLabelId, kEuclid, 0);
        } else {
            if (vn) VD_LAUNCH_P(kLabelId, kManhattan, 1); else VD_LAUNCH_P(kLabelId, kManhattan, 0);
        }
    } else {
        if (metric == kEuclid) {
            if (vn) VD_LAUNCH_P(kLabelXy, kEuclid, 1); else VD_LAUNCH_P(kLabelXy, kEuclid, 0);
        } else {
            if (vn) VD_LAUNCH_P(kLabelXy, kManhattan, 1); else VD_LAUNCH_P(kLabelXy, kManhattan, 0);
        }
    }
#undef VD_LAUNCH_P
#undef VD_LAUNCH_LDS
#undef VD_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_flood_tail(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                             int32_t W, int32_t H, const int32_t *ks, const int32_t *vns,
                             int32_t n, int32_t label, int32_t metric, bool nt, int32_t th,
                             hipStream_t s)
{
    if (n < 2 || n > kTailMaxPasses) return hipErrorInvalidValue;
    if (th != 16 && th != 24 && th != 32) return hipErrorInvalidValue;
    TailPlan plan{};
    plan.n = n;
    for (int32_t i = 0; i < n; ++i) {
        if (ks[i] != 1 && ks[i] != 2 && ks[i] != 4) return hipErrorInvalidValue;
        plan.k[i] = ks[i];
        plan.vn[i] = vns[i] ? 1 : 0;
        plan.halo += ks[i];
    }
    if (plan.halo > kTailHalo) return hipErrorInvalidValue;
    plan.ntx = (uint32_t)((W + kTailTW - 1) / kTailTW);
    const int64_t blocks = (int64_t)plan.ntx * ((H + th - 1) / th);
    dim3 grid((unsigned)blocks), block(kBlock);
    const uint32_t uS = (uint32_t)S;
#define VD_TAIL_TH(LB, MT, ST)                                                                 \
    do {                                                                                       \
        if (th == 16)                                                                          \
            hipLaunchKernelGGL((k_flood_tail<LB, MT, ST, 16>), grid, block, 0, s, src, dst,    \
                               table, uS, W, H, plan);                                         \
        else if (th == 24)                                                                     \
            hipLaunchKernelGGL((k_flood_tail<LB, MT, ST, 24>), grid, block, 0, s, src, dst,    \
                               table, uS, W, H, plan);                                         \
        else                                                                                   \
            hipLaunchKernelGGL((k_flood_tail<LB, MT, ST, 32>), grid, block, 0, s, src, dst,    \
                               table, uS, W, H, plan);                                         \
    } while (0)
#define VD_TAIL(LB, MT)                                                                        \
    do {                                                                                       \
        if (nt) VD_TAIL_TH(LB, MT, kStoreNT); else VD_TAIL_TH(LB, MT, 0);                       \
    } while (0)
    if (label == kLabelId) {
        if (metric == kEuclid) VD_TAIL(kLabelId, kEuclid); else VD_TAIL(kLabelId, kManhattan);
    } else {
        if (metric == kEuclid) VD_TAIL(kLabelXy, kEuclid); else VD_TAIL(kLabelXy, kManhattan);
    }
#undef VD_TAIL
#undef VD_TAIL_TH
    return hipGetLastError();
}

hipError_t launch_flood(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                        int32_t W, int32_t H, int32_t k, int32_t vn, int32_t label,
                        int32_t metric, int32_t variant, int32_t seg_rows, hipStream_t s)
{
    if (variant < 0 || variant >= kFloodVariants) return hipErrorInvalidValue;
    if (variant >= kFloodVariants / 2)
        return launch_flood_st<kStoreNT>(src, dst, table, S, W, H, k, vn, label, metric,
                                         variant - kFloodVariants / 2, seg_rows, s);
    return launch_flood_st<0>(src, dst, table, S, W, H, k, vn, label, metric, variant, seg_rows,
                              s);
}

bool flood_seeds_ok(int32_t W, int32_t H, int32_t k) { return block_ok(W, H, k); }

bool flood_pair_ok(int32_t W, int32_t H, int32_t k) { return pair_ok(W, H, k); }

hipError_t launch_flood_pair(const uint32_t *src, uint32_t *dst, const uint32_t *table,
                             int32_t S, int32_t W, int32_t H, int32_t k, int32_t label,
                             bool seeds, int32_t metric, bool nt, hipStream_t s)
{
    if (!pair_ok(W, H, k) || (seeds && label != kLabelXy)) return hipErrorInvalidValue;
    const int32_t kh = k / 2;
    const int32_t gx = std::min(kh, W) / kQuad;
    const dim3 grid((unsigned)((gx + kBlock - 1) / kBlock), (unsigned)std::min(kh, H));
    const uint32_t uS = (uint32_t)S;
    const int lb = seeds ? kLabelXySeeds : label;
#define VD_PAIR(LB, MT)                                                                        \
    do {                                                                                       \
        if (nt)                                                                                \
            hipLaunchKernelGGL((k_flood_pair<LB, MT, kStoreNT>), grid, dim3(kBlock), 0, s, src, \
                               dst, table, uS, W, H, kh);                                      \
        else                                                                                   \
            hipLaunchKernelGGL((k_flood_pair<LB, MT, 0>), grid, dim3(kBlock), 0, s, src, dst,   \
                               table, uS, W, H, kh);                                           \
    } while (0)
#define VD_PAIR_M(LB)                                                                          \
    do {                                                                                       \
        if (metric == kEuclid) VD_PAIR(LB, kEuclid); else VD_PAIR(LB, kManhattan);             \
    } while (0)
    if (lb == kLabelId)
        VD_PAIR_M(kLabelId);
    else if (lb == kLabelXy)
        VD_PAIR_M(kLabelXy);
    else
        VD_PAIR_M(kLabelXySeeds);
#undef VD_PAIR_M
#undef VD_PAIR
    return hipGetLastError();
}

hipError_t launch_flood_seeds(const uint32_t *src, uint32_t *dst, int32_t W, int32_t H, int32_t k,
                              int32_t vn, int32_t metric, int32_t variant, hipStream_t s)
{
    return launch_flood(src, dst, nullptr, 0, W, H, k, vn, kLabelXySeeds, metric, variant, 0, s);
}

}  // namespace vd
