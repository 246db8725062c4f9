// Device building blocks of the vdflood kernels (included by the kernel
// translation units; everything has internal linkage).
//
// Flood pass (Sec. III, Table I; Sec. V-B, Alg. 1).  The paper's kernel has
// each pixel push its seed into its neighbours in place, which races when
// two pixels push into one.  Here each pixel gathers from the symmetric
// neighbourhood instead and the pass reads one buffer and writes the other,
// so the result is a function of the input map alone.
//
// Candidate order.  A candidate is the pair (d, label) with d the distance
// from the pixel to the label's seed; the smaller d wins and a tie goes to
// the smaller label.  Both are packed into one 64-bit key, d in the high
// word, and the key is minimised as an IEEE double: for a non-negative high
// word below 0x7FF00000 (no NaN or infinity patterns) doubles order exactly
// like their bit patterns read as unsigned integers, denormals included,
// so one v_min_f64 replaces a 64-bit compare and two selects.  Squared
// distances stay below 2^31 - 2^20 because grid sides are at most 16368 and
// the sentinel position is (-16384, -16384).  An unclaimed pixel carries
// label 0 in both modes, whose position is the sentinel: it is farther from
// every pixel than any seed, so an unclaimed candidate never beats a
// claimed one, and if every candidate is unclaimed the result is label 0,
// unclaimed.  The kernels are built without IEEE mode and with denormals
// kept (the code object's default), so v_min_f64 is exact on these keys.
//
// Distances are computed on packed 16-bit coordinates: one v_pk_sub_i16
// gives (dx, dy) and one v_dot2 gives dx*dx + dy*dy exactly in int32.
#pragma once

#include <utility>

#include "vd_kernels.h"

typedef int32_t vd_i32x4 __attribute__((ext_vector_type(4)));

// Indexed (structured) buffer load: address = base + index * stride.
__device__ uint32_t vd_struct_buffer_load(vd_i32x4 rsrc, int32_t vindex, int32_t voffset,
                                          int32_t soffset, int32_t aux)
    __asm("llvm.amdgcn.struct.buffer.load.i32");

namespace vd {

namespace {

constexpr int kBlock = 256;
constexpr int kTW = 256;           // flood pass: columns per workgroup (one per thread)
constexpr int kMaxSegRows = 32;    // flood pass: rows of one chain segment, at most
constexpr int kLdsRow = kTW + 2 * kMaxLdsStep;   // entries of one shared row
constexpr int32_t kRsrcWord3 = 0x00020000;   // buffer descriptor word 3 on gfx9 parts
// Cache-policy operand of a buffer store: 0, or non-temporal (streamed past
// the caches).  An output map is not read again within its pass; when the
// maps do not fit in the Infinity Cache, non-temporal stores keep the
// caches for the input rows and let HBM see long write streams.
constexpr int kStoreNT = 2;

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef vd_i32x4 i32x4;


__device__ __forceinline__ int64_t pixel_of(uint32_t p, int32_t W)
{
    return (int64_t)((int32_t)(p >> 16) - (int32_t)kOff) * W +
           ((int32_t)(p & 0xFFFFu) - (int32_t)kOff);
}

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014): output n of the stream
// seeded with s is mix64(s + (n + 1) * gamma); Stafford's variant-13 mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int32_t draw(uint64_t seed, uint64_t n, int32_t lo, uint32_t span)
{
    uint64_t r = mix64(seed + (n + 1) * 0x9E3779B97F4A7C15ull);
    return lo + (int32_t)(((r >> 32) * (uint64_t)span) >> 32);
}

// ---------------------------------------------------------------------------
// Per-seed steps shared by the single-simulation kernels and the batched and
// served ones (which run them over many simulations in one launch).  Seed i
// lives in table[i + 1]; table[0] is the sentinel.
// ---------------------------------------------------------------------------

// `state` (optional, one byte per seed): a seed takes part only if its
// byte has a bit of `need` (kPresent: in the seed set now; kKept: in it
// since the diagram was made).  Null: every seed takes part.
__device__ __forceinline__ bool takes_part(const uint8_t *state, int32_t i, uint32_t need)
{
    return !state || (state[i] & need) != 0u;
}

// Moves seed i at time step t >= 1 (Alg. 1, SimulateParticles; Sec. V-A):
// per axis a uniform integer in [lo, lo + span) from draw n = ((t - 1) S +
// i) 2 + axis of the move stream, then clamped to the grid.  Returns the
// position before the move; the table holds the new one.
__device__ __forceinline__ uint32_t move_one(uint32_t *table, int32_t i, int32_t S, int32_t W,
                                             int32_t H, uint64_t move_seed, uint64_t t,
                                             int32_t lo, uint32_t span)
{
    const uint64_t n = ((t - 1) * (uint64_t)S + (uint64_t)i) * 2u;
    const uint32_t p = table[i + 1];
    int32_t x = (int32_t)(p & 0xFFFFu) - (int32_t)kOff + draw(move_seed, n + 0, lo, span);
    int32_t y = (int32_t)(p >> 16) - (int32_t)kOff + draw(move_seed, n + 1, lo, span);
    x = min(max(x, 0), W - 1);
    y = min(max(y, 0), H - 1);
    table[i + 1] = ((uint32_t)(y + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff);
    return p;
}

// Seed pixel of seed i on a map whose other pixels hold all ones (a JFA
// step's start): the atomic minimum leaves the lowest coincident label.
__device__ __forceinline__ void splat_min_seed(uint32_t *map, const uint32_t *table, int32_t i,
                                               int32_t W)
{
    atomicMin(&map[pixel_of(table[i + 1], W)], (uint32_t)(i + 1));
}

// XY labels: the seed pixel takes its own packed position, or-ed with
// `mark` (0, or the top bit for a pass that reads through an index).
__device__ __forceinline__ void splat_xy_seed(uint32_t *map, const uint32_t *table, int32_t i,
                                              int32_t W, uint32_t mark)
{
    const uint32_t p = table[i + 1];
    map[pixel_of(p, W)] = p | mark;
}

// Seed pixel of seed i over whatever the pixel held before (a dJFA step's
// splat into the previous diagram, or the old-position index).  The seed
// claims its pixel with label i + 1 if label_state has a bit of label_need,
// else with all ones (no label).  A pixel's value is settled if it is all
// ones or the label of a label-claiming seed that sits on that pixel (per
// `table`); any other value is stale.  A seed leaves a settled value no
// larger than its own claim and otherwise puts its claim in by
// compare-and-swap.  At one pixel the value only goes from stale to all
// ones or a label, from all ones to a label, and from a label to a smaller
// one, so every loop ends, and the final value is the smallest label of the
// label-claiming seeds on the pixel, or all ones if every seed there claims
// without one -- whatever the pixel held before.
__device__ __forceinline__ void splat_swap_seed(uint32_t *map, const uint32_t *table, int32_t S,
                                                int32_t W, int32_t i,
                                                const uint8_t *label_state, uint32_t label_need)
{
    const uint32_t p = table[i + 1];
    const uint32_t me = takes_part(label_state, i, label_need) ? (uint32_t)(i + 1) : 0xFFFFFFFFu;
    uint32_t *const at = &map[pixel_of(p, W)];
    uint32_t cur = __hip_atomic_load(at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const bool settled =
            cur == 0xFFFFFFFFu ||
            (cur - 1u < (uint32_t)S && takes_part(label_state, (int32_t)(cur - 1u), label_need) &&
             table[cur] == p);
        if (settled && cur <= me) return;
        const uint32_t seen = atomicCAS(at, cur, me);
        if (seen == cur) return;
        cur = seen;
    }
}

// The single-launch old-position index of an XY dJFA step: one 32-bit entry
// per pixel, (epoch << 29) | (label << 8) | move code, built by atomic
// minima.  Epochs count down from kIndexEpochs - 1 over the builds since
// the index was last filled with all ones, so this build's entries are
// below every earlier one and below all ones.  At one old position the
// lowest kept label wins and brings its move along: code = (dy + 8) << 4 |
// (dx + 8), the new position minus the old, at most kIndexMaxReach per
// axis.  A seed that is not kept offers the label kIndexNoLabel, which any
// kept seed's entry beats and which reads as unclaimed.  (old_pos,
// new_pos: seed i's position in the diagram and now.)
__device__ __forceinline__ void index_mark_seed(uint32_t *idx, uint32_t old_pos,
                                                uint32_t new_pos, int32_t i, int32_t W, bool kept,
                                                uint32_t epoch)
{
    const uint32_t dx = (new_pos & 0xFFFFu) + 8u - (old_pos & 0xFFFFu);
    const uint32_t dy = (new_pos >> 16) + 8u - (old_pos >> 16);
    const uint32_t e = (epoch << 29) |
                       (kept ? ((uint32_t)(i + 1) << 8) | (dy << 4) | dx : kIndexNoLabel << 8);
    __hip_atomic_fetch_min(&idx[pixel_of(old_pos, W)], e, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// After splat_swap_seed of every seed on the old positions (old_table) into
// idx, idx[old position] holds the lowest kept seed label (index + 1)
// sitting there, or all ones.  That seed writes its new position (table)
// over it; positions are >= (kOff << 16 | kOff), above every label, so no
// other seed of the same old position can mistake the overwritten entry for
// its own label.
__device__ __forceinline__ void index_resolve_seed(uint32_t *idx, const uint32_t *old_table,
                                                   const uint32_t *table, int32_t i, int32_t W)
{
    uint32_t *e = &idx[pixel_of(old_table[i + 1], W)];
    if (*e == (uint32_t)(i + 1)) *e = table[i + 1];
}

// An XY label (an old position) relabelled through the resolved index: the
// moved position of the lowest kept seed that sat there, else unclaimed (the
// entry then holds a leftover label or all ones, both below every
// position); label 0 stays unclaimed.
__device__ __forceinline__ uint32_t relabel_one(uint32_t l, const uint32_t *idx, int32_t W,
                                                int32_t H)
{
    if (l == kEmpty) return kEmpty;
    const int32_t lx = (int32_t)(l & 0xFFFFu) - (int32_t)kOff;
    const int32_t ly = (int32_t)(l >> 16) - (int32_t)kOff;
    const uint32_t np = (lx >= 0 && lx < W && ly >= 0 && ly < H) ? idx[(int64_t)ly * W + lx] : 0u;
    return (int32_t)np >= (int32_t)((kOff << 16) | kOff) ? np : kEmpty;
}

// ---------------------------------------------------------------------------
// Flood pass.
//
// Residue-chain schedule.  At step k, output row y reads input rows y - k,
// y and y + k, which all lie on the chain of rows congruent to y mod k.  A
// workgroup owns 256 adjacent columns of a segment of one chain and walks it
// downwards with a window of three input rows held in registers, so each
// input row is fetched once per segment (plus two rows of overlap between
// segments) whatever k is.  Rows are requested P + 1 rows ahead of use.
// Horizontal neighbours (x - k, x + k) are separate loads of the same row;
// for k < 256 they fall in lines the workgroup fetches anyway, for larger k
// in lines the workgroups of the neighbouring column tiles fetch.
//
// Buffer addressing.  Each row is read through its own buffer descriptor
// (base = row start, size = one row; size 0 for a row off the grid), with
// per-lane byte offsets 4(x - k), 4x, 4(x + k) fixed for the whole walk.
// The hardware returns 0 -- the unclaimed label -- for any offset outside
// the row, so off-grid neighbours need no compare, and stores from lanes
// past the right edge are dropped the same way.  ID labels fetch their
// position with an indexed buffer load from the seed table (stride 4).
//
// XCD-aware block order.  Workgroups are dispatched round-robin over the 8
// XCDs (block b goes to XCD b % 8).  Block b is given logical tile
// xcd * (blocks / 8) + b / 8, so each XCD walks one contiguous run of
// logical tiles (chain-major, column-minor): horizontal neighbours and the
// overlap rows of consecutive segments are then fetched by the same XCD,
// close in time, and hit its L2.
// ---------------------------------------------------------------------------
struct Ent {
    uint32_t l;   // label
    uint32_t s;   // its seed's packed position
};

struct Row {
    Ent w, c, e;  // columns x - k, x, x + k
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const uint32_t *base, int32_t y,
                                                           int32_t W, int32_t H)
{
    const bool in = y >= 0 && y < H;
    const uint32_t *p = base + (in ? (int64_t)y * W : 0);
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, 0, in ? W * 4 : 0, kRsrcWord3);
}

// A row of a chain walk addressed incrementally: `addr` is the byte address
// of the row's first pixel and moves on by k rows per step, so a step costs
// two scalar adds instead of a 64-bit multiply.  Rows the walk reaches are
// never above the grid; a row below it gets an empty descriptor.
struct Cursor {
    uint64_t addr;
    int32_t y;
};

__device__ __forceinline__ Cursor cursor_at(const uint32_t *base, int32_t y, int32_t W)
{
    return Cursor{(uint64_t)base + 4ull * (uint64_t)((int64_t)y * W), y};
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t cursor_rsrc(const Cursor &c, int32_t W,
                                                              int32_t H)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)c.addr, 0, c.y < H ? W * 4 : 0, kRsrcWord3);
}

__device__ __forceinline__ void advance(Cursor &c, uint32_t step_bytes, int32_t k)
{
    c.addr += step_bytes;
    c.y += k;
}

// Labels of one row (columns x - k, x, x + k); off-grid reads return 0.
__device__ __forceinline__ void load_labels(Row &row, __amdgpu_buffer_rsrc_t r, int32_t ow,
                                            int32_t oc, int32_t oe)
{
    row.w.l = __builtin_amdgcn_raw_buffer_load_b32(r, ow, 0, 0);
    row.c.l = __builtin_amdgcn_raw_buffer_load_b32(r, oc, 0, 0);
    row.e.l = __builtin_amdgcn_raw_buffer_load_b32(r, oe, 0, 0);
}

// Position of an ID label: an indexed load from the seed table (entry 0,
// the unclaimed label, is the sentinel) -- unless the same column k rows
// up carried the same label, whose position is reused.  In a converged map
// most labels repeat down a column.  A lane that reuses sends the load an
// index past the table, which the hardware answers with 0 without touching
// memory; this keeps the lookup free of exec-mask branches.
__device__ __forceinline__ uint32_t seed_pos(uint32_t l, uint32_t prev_l, uint32_t prev_s,
                                             i32x4 tab)
{
    const bool fresh = l != prev_l;
    const uint32_t v = vd_struct_buffer_load(tab, fresh ? (int32_t)l : -1, 0, 0, 0);
    return fresh ? v : prev_s;
}

// Seed positions of a row's labels; `up` is the row k above on the chain
// (or a row of unclaimed labels).  XY labels are positions already.
template <int LABEL>
__device__ __forceinline__ void lookup_positions(Row &row, const Row &up, i32x4 tab)
{
    if (LABEL == kLabelId) {
        row.w.s = seed_pos(row.w.l, up.w.l, up.w.s, tab);
        row.c.s = seed_pos(row.c.l, up.c.l, up.c.s, tab);
        row.e.s = seed_pos(row.e.l, up.e.l, up.e.s, tab);
    } else {
        row.w.s = row.w.l;
        row.c.s = row.c.l;
        row.e.s = row.e.l;
    }
}

// f(integral_constant<int, 0>, ..., integral_constant<int, N - 1>): a loop
// body instantiated N times with compile-time indices.
template <class F, int... I>
__device__ __forceinline__ bool expand_impl(F &f, std::integer_sequence<int, I...>)
{
    return f(std::integral_constant<int, I>{}...);
}

template <int N, class F>
__device__ __forceinline__ bool expand(F &f)
{
    return expand_impl(f, std::make_integer_sequence<int, N>{});
}

template <int METRIC>
__device__ __forceinline__ double cand_key(uint32_t p, const Ent &e)
{
    int32_t d;
    if (METRIC == kEuclid) {
        // The clamped form cannot saturate (d < 2^31, see above); it makes
        // the compiler emit the three-operand v_dot2 with an inline zero
        // rather than the accumulating form plus a move of zero into the
        // accumulator.
        short2_t dv = __builtin_bit_cast(short2_t, p) - __builtin_bit_cast(short2_t, e.s);
        d = __builtin_amdgcn_sdot2(dv, dv, 0, true);
    } else {
        // v_sad_u16 sums the absolute differences of both 16-bit halves, and
        // both halves of a packed position are a coordinate plus 16384, so
        // one instruction gives |dx| + |dy| exactly.
        d = (int32_t)__builtin_amdgcn_sad_u16(p, e.s, 0);
    }
    return __hiloint2double(d, (int32_t)e.l);
}

// Output pixel p (packed position) from the window a (row y - k), b (row
// y), c (row y + k), stored through `out` at byte offset oc.  A row off the
// grid reads as unclaimed labels, whose sentinel keys lose to every claimed
// candidate and tie with each other, so the edge rows need no special case.
template <int METRIC, int VN, int ST>
__device__ __forceinline__ void emit(__amdgpu_buffer_rsrc_t out, const Row &a, const Row &b,
                                     const Row &c, uint32_t p, int32_t oc)
{
    double best = cand_key<METRIC>(p, b.c);
    best = __builtin_fmin(best, cand_key<METRIC>(p, b.w));
    best = __builtin_fmin(best, cand_key<METRIC>(p, b.e));
    best = __builtin_fmin(best, cand_key<METRIC>(p, a.c));
    best = __builtin_fmin(best, cand_key<METRIC>(p, c.c));
    if (!VN) {
        best = __builtin_fmin(best, cand_key<METRIC>(p, a.w));
        best = __builtin_fmin(best, cand_key<METRIC>(p, a.e));
        best = __builtin_fmin(best, cand_key<METRIC>(p, c.w));
        best = __builtin_fmin(best, cand_key<METRIC>(p, c.e));
    }
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)__double2loint(best), out, oc, 0, ST);
}

struct Tile {
    int32_t x0;        // first column
    int32_t y0;        // first output row
    int32_t j0, jend;  // chain indices of the segment's rows
};

__device__ __forceinline__ Tile decode_tile(uint32_t logical, const FloodGrid &g, int32_t k,
                                            int32_t H)
{
    // The integer divisions run on the vector unit; readfirstlane tells
    // the compiler the results are wave-uniform, so every row address and
    // buffer descriptor derived from them stays scalar.
    const uint32_t col = __builtin_amdgcn_readfirstlane(logical % g.ncol);
    const uint32_t rs = logical / g.ncol;
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(rs % g.nseg));
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)(rs / g.nseg));   // rows r, r + k, ...
    const int32_t nj = (H - 1 - r) / k + 1;                                      // rows on the chain
    Tile t;
    t.x0 = (int32_t)col * kTW;
    t.j0 = seg * g.L;
    t.jend = min(t.j0 + g.L, nj);
    t.y0 = r + t.j0 * k;
    return t;
}

// Block b of a launch -> logical tile: each XCD (block b runs on XCD b % 8)
// gets one contiguous run of tiles.
__device__ __forceinline__ uint32_t xcd_logical(uint32_t b, uint32_t nblocks)
{
    const uint32_t q = nblocks >> 3, rem = nblocks & 7u, xcd = b & 7u;
    return xcd * q + min(xcd, rem) + (b >> 3);
}

// Indexed descriptor of a seed table with S + 1 entries of 4 bytes.
__device__ __forceinline__ i32x4 table_rsrc(const uint32_t *table, uint32_t S)
{
    const uint64_t ta = (uint64_t)table;
    return i32x4{(int32_t)(uint32_t)ta, (int32_t)(((uint32_t)(ta >> 32) & 0xFFFFu) | (4u << 16)),
                 (int32_t)(S + 1), kRsrcWord3};
}

// One tile of a pass: 256 columns of one segment of one chain, walked with
// a three-row register window (see the note above).
template <int LABEL, int METRIC, int VN, int P, int ST = 0>
__device__ __forceinline__ void flood_chain_tile(const uint32_t *src, uint32_t *dst, i32x4 tab,
                                                 int32_t W, int32_t H, int32_t k,
                                                 const FloodGrid &g, uint32_t logical)
{
    const Tile tl = decode_tile(logical, g, k, H);
    int32_t j = tl.j0;
    if (j >= tl.jend) return;
    const int32_t jend = tl.jend;
    const int32_t x = tl.x0 + (int32_t)threadIdx.x;
    const uint32_t px = (uint32_t)(x + (int32_t)kOff);
    const int32_t ow = 4 * (x - k), oc = 4 * x, oe = 4 * (x + k);
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;   // < 2^31 for sides <= 16368
    // packed position of the output pixel; the row field moves on by k per step
    uint32_t p = ((uint32_t)(tl.y0 + (int32_t)kOff) << 16) | px;
    const uint32_t p_step = (uint32_t)k << 16;

    // NR row registers rotate through the roles: at unrolled step u, slot
    // (u + m + 1) % NR holds row y + m*k for m = -1 .. P.  Labels are
    // requested P + 1 rows ahead of the output row and their positions P
    // rows ahead, so neither load is waited for in the step that issues it.
    // The loop is unrolled NR times, so no row is ever copied.
    constexpr int NR = P + 3;
    Row R[NR];
#pragma unroll
    for (int m = -1; m <= P; ++m)
        load_labels(R[m + 1], row_rsrc(src, tl.y0 + m * k, W, H), ow, oc, oe);
    const Row none = {{kEmpty, 0u}, {kEmpty, 0u}, {kEmpty, 0u}};   // label 0 -> sentinel 0
    lookup_positions<LABEL>(R[0], none, tab);
#pragma unroll
    for (int m = 0; m < P; ++m) lookup_positions<LABEL>(R[m + 1], R[m], tab);
    Cursor in = cursor_at(src, tl.y0 + (P + 1) * k, W);   // next row to load
    Cursor out = cursor_at(dst, tl.y0, W);                // next row to store (always on the grid)
    // One output row with the slots of unrolled step U; false once the
    // segment is done.
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        if (j >= jend) return false;
        load_labels(R[(u + NR - 1) % NR], cursor_rsrc(in, W, H), ow, oc, oe);
        lookup_positions<LABEL>(R[(u + NR - 2) % NR], R[(u + NR - 3) % NR], tab);
        emit<METRIC, VN, ST>(cursor_rsrc(out, W, H), R[u % NR], R[(u + 1) % NR], R[(u + 2) % NR], p,
                         oc);
        advance(in, step_bytes, k);
        advance(out, step_bytes, k);
        p += p_step;
        ++j;
        return true;
    };
    auto round = [&](auto... U) -> bool { return (step(U) && ...); };
    while (expand<NR>(round)) {
    }
}

// Shared-row variant (steps k <= kMaxLdsStep).  The same chain walk, but the
// 256 + 2k entries of each row that a workgroup needs (its columns plus k on
// either side) are fetched once, one or two per thread, and exchanged
// through LDS, where each thread reads its three (x - k, x, x + k).  A
// thread therefore issues one or two label loads and, for ID labels, one or
// two seed-table lookups per row instead of three of each.  Two LDS row
// buffers alternate; the barrier of each exchange also orders the reuse of
// the buffer written two exchanges earlier.
struct Raw {
    uint32_t l1, l2;   // labels of this thread's entries t and kTW + t
    uint32_t s1, s2;   // their positions
};

struct Slot {
    Raw raw;
    Row win;
};

// One tile of a pass with shared rows; `lds` holds two rows of kLdsRow
// entries.  Callers must not let a previous use of `lds` overlap the first
// exchange (a barrier between tiles suffices).
template <int LABEL, int METRIC, int VN, int P, int ST = 0>
__device__ __forceinline__ void flood_lds_tile(const uint32_t *src, uint32_t *dst, i32x4 tab,
                                               int32_t W, int32_t H, int32_t k,
                                               const FloodGrid &g, uint32_t logical,
                                               uint2 (*lds)[kLdsRow])
{
    const Tile tl = decode_tile(logical, g, k, H);
    int32_t j = tl.j0;
    if (j >= tl.jend) return;
    const int32_t jend = tl.jend;
    const int32_t t = (int32_t)threadIdx.x;
    const int32_t x0 = tl.x0;
    const int32_t x = x0 + t;
    const uint32_t px = (uint32_t)(x + (int32_t)kOff);
    const int32_t oc = 4 * x;
    // entry t is column x0 - k + t; entry kTW + t (only read for t < 2k) is
    // column x0 + kTW - k + t; an unused second entry reads out of range
    const int32_t o1 = 4 * (x0 - k + t);
    const int32_t o2 = t < 2 * k ? 4 * (x0 + kTW - k + t) : INT32_MIN;
    const bool wave2 = __builtin_amdgcn_readfirstlane(t & ~63) < 2 * k;   // any lane of the wave
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;
    uint32_t p = ((uint32_t)(tl.y0 + (int32_t)kOff) << 16) | px;
    const uint32_t p_step = (uint32_t)k << 16;
    // byte offset of the LDS row written next; the two rows alternate
    uint32_t lds_sel = 0;

    auto load = [&](Slot &sl, __amdgpu_buffer_rsrc_t rr) {
        sl.raw.l1 = __builtin_amdgcn_raw_buffer_load_b32(rr, o1, 0, 0);
        sl.raw.l2 = wave2 ? __builtin_amdgcn_raw_buffer_load_b32(rr, o2, 0, 0) : 0u;
    };
    // `up` holds the row k above on the chain; its positions are reused
    // where the label repeats.
    auto lookup = [&](Slot &sl, const Raw &up) {
        if (LABEL == kLabelId) {
            sl.raw.s1 = seed_pos(sl.raw.l1, up.l1, up.s1, tab);
            // Only the load sits under the wave-uniform branch: a select
            // inside it would wait for the load on the spot.  Waves without
            // second entries carry label 0 there, so they always reuse.
            const bool fresh2 = sl.raw.l2 != up.l2;
            uint32_t v2 = 0;
            if (wave2) v2 = vd_struct_buffer_load(tab, fresh2 ? (int32_t)sl.raw.l2 : -1, 0, 0, 0);
            sl.raw.s2 = fresh2 ? v2 : up.s2;
        } else {
            sl.raw.s1 = sl.raw.l1;
            sl.raw.s2 = sl.raw.l2;
        }
    };
    // Every thread writes both of its entries (entries past 256 + 2k are
    // never read), so the writes need no exec mask.
    auto exchange = [&](Slot &sl) {
        uint2 *row = (uint2 *)((char *)lds + lds_sel);
        lds_sel ^= (uint32_t)sizeof(lds[0]);
        row[t] = make_uint2(sl.raw.l1, sl.raw.s1);
        row[kTW + t] = make_uint2(sl.raw.l2, sl.raw.s2);
        __syncthreads();
        const uint2 w = row[t], c = row[t + k], e = row[t + 2 * k];
        sl.win.w.l = w.x;
        sl.win.w.s = w.y;
        sl.win.c.l = c.x;
        sl.win.c.s = c.y;
        sl.win.e.l = e.x;
        sl.win.e.s = e.y;
    };

    // Ring of NR slots as in k_flood: slot (u + m + 1) % NR holds row
    // y + m*k; labels are requested P + 1 rows ahead, positions P rows
    // ahead, and the row entering the window (m = 1) is exchanged.
    constexpr int NR = P + 3;
    Slot R[NR];
#pragma unroll
    for (int m = -1; m <= P; ++m) load(R[m + 1], row_rsrc(src, tl.y0 + m * k, W, H));
    const Raw none = {kEmpty, kEmpty, 0u, 0u};   // label 0 -> sentinel position 0
    lookup(R[0], none);
#pragma unroll
    for (int m = 0; m < P; ++m) lookup(R[m + 1], R[m].raw);
    exchange(R[0]);
    exchange(R[1]);
    Cursor in = cursor_at(src, tl.y0 + (P + 1) * k, W);
    Cursor out = cursor_at(dst, tl.y0, W);
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        if (j >= jend) return false;
        load(R[(u + NR - 1) % NR], cursor_rsrc(in, W, H));
        lookup(R[(u + NR - 2) % NR], R[(u + NR - 3) % NR].raw);
        exchange(R[(u + 2) % NR]);
        emit<METRIC, VN, ST>(cursor_rsrc(out, W, H), R[u % NR].win, R[(u + 1) % NR].win,
                         R[(u + 2) % NR].win, p, oc);
        advance(in, step_bytes, k);
        advance(out, step_bytes, k);
        p += p_step;
        ++j;
        return true;
    };
    auto round = [&](auto... U) -> bool { return (step(U) && ...); };
    while (expand<NR>(round)) {
    }
}

}  // namespace

}  // namespace vd
