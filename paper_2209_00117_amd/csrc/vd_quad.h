// Flood pass with four columns per lane (grids whose width is a multiple of
// four).  Same pass as the tiles in vd_device.h (Sec. III, Table I; Sec.
// V-B, Alg. 1) and the same residue-chain walk, but each lane owns four
// adjacent columns, so every row costs a lane one 16-byte load and one
// 16-byte store, and the per-row scalar work (descriptors, loop control,
// barrier) is shared by four pixels.  A workgroup covers 1024 columns.
//
// Groups.  A lane with columns x .. x+3 needs, from each input row, the
// groups at x - h, x and x + h, where h = k for k >= 4 (whole groups, since
// k is a power of two) and h = 4 for k = 1, 2 (the neighbouring groups,
// from which the columns x - k .. x + 3 + k are picked at compile time).
// With the width a multiple of four a group lies wholly inside or wholly
// outside a row, so the buffer range check returns 0 -- the unclaimed
// label -- for groups off the grid, exactly as for single columns.
//
// Rolling accumulators.  Input row y (chain index s) is a candidate row of
// the outputs y - k (as the row below), y (same row) and y + k (as the row
// above).  Each lane keeps the running best key of those three output rows
// and folds every input row into all three as soon as it arrives, so an
// input row is consumed once and no three-row window is held; the output
// y - k is then complete and is stored.  The accumulators rotate through
// three registers sets, which the unrolling by three makes static.
#pragma once

#include "vd_device.h"

namespace vd {

namespace {

constexpr int kQuad = 4;                             // columns per lane
constexpr int kTWQ = kBlock * kQuad;                 // columns per workgroup
constexpr int kQuadLdsRow = kTWQ + 2 * kMaxLdsStep;  // entries of one shared row
constexpr int kQuadLdsRowWide = kTWQ + 2 * kMaxQuadLdsStep;   // the same for k <= 512

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Labels and positions of one group of four columns.
struct G4 {
    u32x4 l, s;
};

// Columns a lane reads from one input row: groups at x - h, x, x + h.
struct Three {
    G4 a, b, c;
};

// Candidate j (0: west, 1: centre, 2: east) of pixel i of the lane, as
// (label, position).  KC = 0: k >= 4; KC = 1, 2: k = KC, picked from the
// twelve columns x - 4 .. x + 7.
template <int KC>
__device__ __forceinline__ Ent cand(const Three &t, int i, int j)
{
    int g, e;
    if (KC == 0) {
        g = j;
        e = i;
    } else {
        const int col = 4 + i + (j - 1) * KC;   // 0 .. 11
        g = col >> 2;
        e = col & 3;
    }
    const G4 &q = g == 0 ? t.a : (g == 1 ? t.b : t.c);
    return Ent{q.l[e], q.s[e]};
}

// Folds the three candidates (or the centre only) of input row t into the
// best keys of the lane's four pixels of one output row.
template <int METRIC, int KC, bool CENTRE_ONLY, bool INIT>
__device__ __forceinline__ void fold(double (&best)[4], const u32x4 &p, const Three &t)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double b = cand_key<METRIC>(p[i], cand<KC>(t, i, 1));
        if (!INIT) b = __builtin_fmin(best[i], b);
        if (!CENTRE_ONLY) {
            b = __builtin_fmin(b, cand_key<METRIC>(p[i], cand<KC>(t, i, 0)));
            b = __builtin_fmin(b, cand_key<METRIC>(p[i], cand<KC>(t, i, 2)));
        }
        best[i] = b;
    }
}

__device__ __forceinline__ u32x4 labels_of(const double (&best)[4])
{
    return u32x4{(uint32_t)__double2loint(best[0]), (uint32_t)__double2loint(best[1]),
                 (uint32_t)__double2loint(best[2]), (uint32_t)__double2loint(best[3])};
}

__device__ __forceinline__ u32x4 load4(__amdgpu_buffer_rsrc_t r, int32_t off)
{
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <int ST>
__device__ __forceinline__ void store4(u32x4 v, __amdgpu_buffer_rsrc_t r, int32_t off)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, v), r, off, 0, ST);
}

// Seed positions of four ID labels, reusing that of the left neighbour in
// the group or of the same column k rows up where the label repeats (a
// Voronoi cell spans several pixels of a row); only the other lanes send
// the table an index (see seed_pos).
__device__ __forceinline__ u32x4 seed_pos4(u32x4 l, const G4 &up, i32x4 tab)
{
    u32x4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool left = e > 0 && l[e] == l[e > 0 ? e - 1 : 0];
        const bool fresh = !left && l[e] != up.l[e];
        const uint32_t v = vd_struct_buffer_load(tab, fresh ? (int32_t)l[e] : -1, 0, 0, 0);
        r[e] = fresh ? v : (left ? r[e > 0 ? e - 1 : 0] : up.s[e]);
    }
    return r;
}

struct TileQ {
    int32_t x0;        // first column
    int32_t y0;        // first output row
    int32_t j0, jend;  // chain indices of the segment's output rows
};

__device__ __forceinline__ TileQ decode_tile_q(uint32_t logical, const FloodGrid &g, int32_t k,
                                               int32_t H)
{
    const uint32_t col = __builtin_amdgcn_readfirstlane(logical % g.ncol);
    const uint32_t rs = logical / g.ncol;
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(rs % g.nseg));
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)(rs / g.nseg));
    const int32_t nj = (H - 1 - r) / k + 1;
    TileQ t;
    t.x0 = (int32_t)col * kTWQ;
    t.j0 = seg * g.L;
    t.jend = min(t.j0 + g.L, nj);
    t.y0 = r + t.j0 * k;
    return t;
}

// Tile t of a segment-major order, as the chain-major number the tile
// functions decode: consecutive tiles (and so each XCD's run of them) are
// the segments of all residue chains that cover one band of rows, so what
// the labels of that band look up -- seed-table entries, index lines --
// stays in one L2.
__device__ __forceinline__ uint32_t seg_major(uint32_t t, const FloodGrid &g)
{
    const uint32_t nres = g.nblocks / (g.ncol * g.nseg);
    const uint32_t col = t % g.ncol, rs = t / g.ncol;
    return ((rs % nres) * g.nseg + rs / nres) * g.ncol + col;
}

template <int N>
using IC = std::integral_constant<int, N>;

// Request phase of input row s: the first two rows may lie above the grid
// (phase 0 and 1 address them directly); later rows come from the cursor.
// Rows requested in the prologue carry their index (for the lookups that
// trail the requests); rows requested in the loop carry kSteady.
constexpr int kSteady = 1 << 20;

// The walk shared by all quad tiles.  Input row s of the segment is grid
// row y0 + (s - 1) k, and output row j (grid row y0 + j k) takes input rows
// j, j + 1 and j + 2.  Input rows rotate through NS slots (row s in slot
// s % NS) and are requested NS - 1 rows ahead of their use:
// `request(s, Slot, Phase)` starts fetching row s into its slot, and
// `fetch(Slot)` returns the row in a slot as a Three.  The loop is unrolled
// lcm(3, NS) times, so every slot and accumulator index is a compile-time
// constant and the ring lives in registers.
template <int METRIC, int VN, int KC, int NS, int ST, class Request, class Fetch>
__device__ __forceinline__ void quad_walk(uint32_t *dst, int32_t W, int32_t H, int32_t k,
                                          const TileQ &tl, int32_t oc, Request &request,
                                          Fetch &fetch)
{
    static_assert(NS == 3 || NS == 4, "ring of 3 or 4 rows");
    constexpr int A = NS - 1;                 // rows requested ahead of use
    constexpr int U = NS == 3 ? 3 : 12;       // lcm(3, NS)
    const int32_t nout = tl.jend - tl.j0;
    const int32_t x = tl.x0 + kQuad * (int32_t)threadIdx.x;
    const uint32_t pk = (uint32_t)k << 16;
    // packed positions of the lane's four pixels in output row 0
    const uint32_t p0 = ((uint32_t)(tl.y0 + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff);
    u32x4 prow[3];   // pixel positions of the output rows held in acc[]
    double acc[3][4];
    Cursor out = cursor_at(dst, tl.y0, W);
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;

    auto pre = [&](auto M) { request(decltype(M)::value, IC<decltype(M)::value % NS>{}, M); };
    pre(IC<0>{});
    pre(IC<1>{});
    pre(IC<2>{});
    if constexpr (A >= 3) pre(IC<3>{});
    // input rows 0 and 1 open output rows 0 and 1
    {
        prow[0] = u32x4{p0, p0 + 1, p0 + 2, p0 + 3};
        const Three t = fetch(IC<0>{});
        fold<METRIC, KC, VN != 0, true>(acc[0], prow[0], t);
    }
    pre(IC<A + 1>{});
    {
        prow[1] = prow[0] + pk;
        const Three t = fetch(IC<1>{});
        fold<METRIC, KC, false, false>(acc[0], prow[0], t);
        fold<METRIC, KC, VN != 0, true>(acc[1], prow[1], t);
    }
    // Input row s (s >= 2) closes output row s - 2, continues s - 1 and
    // opens s (rows opened past the segment are never stored).
    int32_t s = 2;
    auto step = [&](auto I) -> bool {
        constexpr int u = (decltype(I)::value + 2) % U;   // s mod U
        constexpr int c0 = (u + 1) % 3, c1 = (u + 2) % 3, c2 = u % 3;
        if (s - 2 >= nout) return false;
        request(s + A, IC<(u + A) % NS>{}, IC<kSteady>{});
        prow[c2] = prow[c1] + pk;
        const Three t = fetch(IC<u % NS>{});
        fold<METRIC, KC, VN != 0, false>(acc[c0], prow[c0], t);
        store4<ST>(labels_of(acc[c0]), cursor_rsrc(out, W, H), oc);
        fold<METRIC, KC, false, false>(acc[c1], prow[c1], t);
        fold<METRIC, KC, VN != 0, true>(acc[c2], prow[c2], t);
        advance(out, step_bytes, k);
        ++s;
        return true;
    };
    auto round = [&](auto... I) -> bool { return (step(I) && ...); };
    while (expand<U>(round)) {
    }
}

// XY labels: positions are the labels, so a lane loads its three groups of
// each row directly (the neighbouring groups come from L2) and needs no
// exchange.  Input rows are requested NS - 1 rows ahead into a ring of NS.
template <int METRIC, int VN, int KC, int NS, int ST>
__device__ __forceinline__ void flood_quad_xy_tile(const uint32_t *src, uint32_t *dst,
                                                   int32_t W, int32_t H, int32_t k,
                                                   const FloodGrid &g, uint32_t logical)
{
    const TileQ tl = decode_tile_q(logical, g, k, H);
    if (tl.j0 >= tl.jend) return;
    const int32_t h = KC == 0 ? k : 4;
    const int32_t x = tl.x0 + kQuad * (int32_t)threadIdx.x;
    const int32_t oc = 4 * x, oa = 4 * (x - h), ob = 4 * (x + h);
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;
    u32x4 ring[NS][3];
    // input row s of the segment is grid row y0 + (s - 1) k; rows above the
    // grid only occur among the first two
    Cursor in = cursor_at(src, tl.y0 + k, W);   // input row 2
    // input rows past the segment's last output row + 1 are requested with
    // an empty descriptor (no memory access): short segments need not fetch
    // the rows their ring would hold next
    const int32_t last_in = tl.jend - tl.j0 + 1;
    auto request = [&](int32_t s, auto Slot, auto Phase) {
        __amdgpu_buffer_rsrc_t r;
        if (decltype(Phase)::value < 2) {
            r = row_rsrc(src, tl.y0 + (s - 1) * k, W, H);
        } else {
            r = cursor_rsrc(in, W, s <= last_in ? H : 0);
            advance(in, step_bytes, k);
        }
        u32x4 *q = ring[decltype(Slot)::value];
        q[0] = load4(r, oa);
        q[1] = load4(r, oc);
        q[2] = load4(r, ob);
    };
    auto fetch = [&](auto Slot) -> Three {
        const u32x4 *q = ring[decltype(Slot)::value];
        return Three{{q[0], q[0]}, {q[1], q[1]}, {q[2], q[2]}};
    };
    quad_walk<METRIC, VN, KC, NS, ST>(dst, W, H, k, tl, oc, request, fetch);
}

// ID labels at large steps (k > kMaxLdsStep, a multiple of 4): the groups
// at x - k and x + k belong to other workgroups' columns, so each lane loads
// its three groups itself and looks up all twelve positions (each reused
// where the label repeats k rows up).  Labels are requested NS - 1 rows
// ahead of use and looked up one row ahead of use.
template <int METRIC, int VN, int NS, int ST>
__device__ __forceinline__ void flood_quad_id_direct_tile(const uint32_t *src, uint32_t *dst,
                                                          i32x4 tab, int32_t W, int32_t H,
                                                          int32_t k, const FloodGrid &g,
                                                          uint32_t logical)
{
    constexpr int D = NS - 2;   // rows between a row's label request and its lookups
    const TileQ tl = decode_tile_q(logical, g, k, H);
    if (tl.j0 >= tl.jend) return;
    const int32_t x = tl.x0 + kQuad * (int32_t)threadIdx.x;
    const int32_t oc = 4 * x, oa = 4 * (x - k), ob = 4 * (x + k);
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;
    Three ring[NS];
    const Three none = {};   // labels 0 -> sentinel position 0
    Cursor in = cursor_at(src, tl.y0 + k, W);   // input row 2
    auto request = [&](int32_t s, auto Slot, auto Phase) {
        constexpr int slot = decltype(Slot)::value, phase = decltype(Phase)::value;
        __amdgpu_buffer_rsrc_t r;
        if (phase < 2) {
            r = row_rsrc(src, tl.y0 + (s - 1) * k, W, H);
        } else {
            r = cursor_rsrc(in, W, H);
            advance(in, step_bytes, k);
        }
        Three &q = ring[slot];
        q.a.l = load4(r, oa);
        q.b.l = load4(r, oc);
        q.c.l = load4(r, ob);
        if (phase >= D) {   // positions of row s - D, reusing row s - D - 1's
            Three &n = ring[(slot + NS - D) % NS];
            const Three &up = phase >= D + 1 ? ring[(slot + NS - D - 1) % NS] : none;
            n.a.s = seed_pos4(n.a.l, up.a, tab);
            n.b.s = seed_pos4(n.b.l, up.b, tab);
            n.c.s = seed_pos4(n.c.l, up.c, tab);
        }
    };
    auto fetch = [&](auto Slot) -> Three { return ring[decltype(Slot)::value]; };
    quad_walk<METRIC, VN, 0, NS, ST>(dst, W, H, k, tl, oc, request, fetch);
}

// How a shared-row tile finds the position of each label it loads.
//
// TableLookup: ID labels; the position comes from the seed table (entry 0,
// the unclaimed label, is the sentinel), reused where the label repeats k
// rows up.
struct TableLookup {
    i32x4 tab;
    static constexpr bool kLabelIsPos = false;
    __device__ __forceinline__ u32x4 pos4(u32x4 l, const G4 &up) const
    {
        return seed_pos4(l, up, tab);
    }
    __device__ __forceinline__ uint32_t pos1(uint32_t l) const
    {
        return vd_struct_buffer_load(tab, (int32_t)l, 0, 0, 0);
    }
};

// RelabelLookup: the XY labels of the previous diagram, read by a dJFA
// step's first pass.  A label is an old position, which stands for the
// moved position of the lowest kept seed that sat there (the old position
// plus the move code of the index entry there, see index_mark_seed; the
// label field kIndexNoLabel: no such seed, unclaimed), or a seed pixel
// claimed by this step's splat, marked with the top bit, which stands for
// itself; 0 stays unclaimed.  The translated value is both the label and
// the position.  Where the label repeats that of the left neighbour in the
// group or k rows up, that result is reused, and the lane's gather goes to
// an offset past the map, which the hardware answers without a memory
// access.
constexpr uint32_t kMarked = 0x80000000u;

struct RelabelLookup {
    __amdgpu_buffer_rsrc_t idx;
    int32_t W;
    static constexpr bool kLabelIsPos = true;
    __device__ __forceinline__ uint32_t one(uint32_t l, bool fresh) const
    {
        const bool marked = (l & kMarked) != 0u;
        const int32_t x = (int32_t)(l & 0xFFFFu) - (int32_t)kOff;
        const int32_t y = (int32_t)(l >> 16) - (int32_t)kOff;
        const int32_t at = (fresh && !marked && l != kEmpty) ? 4 * (y * W + x) : -1;
        const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(idx, at, 0, 0);
        const bool kept = l != kEmpty && ((v >> 8) & kIndexNoLabel) != kIndexNoLabel;
        const uint32_t moved =
            kept ? l + ((((v >> 4) & 15u) << 16) | (v & 15u)) - 0x00080008u : kEmpty;
        return marked ? (l & ~kMarked) : moved;
    }
    __device__ __forceinline__ u32x4 pos4(u32x4 l, const G4 &up) const
    {
        u32x4 r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool left = e > 0 && l[e] == l[e > 0 ? e - 1 : 0];
            const bool fresh = !left && l[e] != up.l[e];
            const uint32_t v = one(l[e], fresh);
            r[e] = fresh ? v : (left ? r[e > 0 ? e - 1 : 0] : up.s[e]);
        }
        return r;
    }
    __device__ __forceinline__ uint32_t pos1(uint32_t l) const { return one(l, true); }
};

// XY labels of a JFA step's first pass read straight from the previous
// diagram: only this step's seed pixels, marked with the top bit by the
// splat, are claimed (by themselves); every other label is left from the
// previous diagram and counts as unclaimed, as on a filled map.  A pass
// writes no marked label, so a diagram holds none.
struct SeedMarks {
    static constexpr bool kLabelIsPos = true;
    __device__ __forceinline__ u32x4 pos4(u32x4 l, const G4 &) const
    {
        u32x4 r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = (l[e] & kMarked) ? (l[e] & ~kMarked) : kEmpty;
        return r;
    }
};

// Shared rows of the ID tile, in groups of four entries: entry e is column
// x0 - h + e.  Labels and positions are kept apart so that a lane moves 16
// contiguous bytes of each array per group.
template <int ROW>
struct QuadRowT {
    u32x4 l[ROW / kQuad];
    u32x4 s[ROW / kQuad];
};
using QuadRow = QuadRowT<kQuadLdsRow>;           // steps up to kMaxLdsStep: 20 KiB for two
using QuadRowWide = QuadRowT<kQuadLdsRowWide>;   // steps up to kMaxQuadLdsStep: 32 KiB

// ID labels (steps k <= kMaxLdsStep): the 1024 + 2h columns a workgroup
// needs are fetched once -- group t by lane t, the 2h / 4 groups past the
// end by the first lanes of wave 0 -- their positions looked up once, and
// the three groups each lane needs are read back from LDS.  Labels are
// requested NS - 1 rows ahead and looked up one row ahead; two LDS rows
// alternate, and the barrier of each exchange also orders the reuse of the
// row written two exchanges earlier.  Callers must not let a previous use
// of `lds` overlap the first exchange (a barrier between tiles suffices).
// DL (0: NS - 2) is the number of rows between a row's label request and
// its lookups; the lookups then have NS - 1 - DL rows to arrive.
template <int METRIC, int VN, int KC, int NS, int ST, class Q, class LK, int DL = 0>
__device__ __forceinline__ void flood_quad_id_tile(const uint32_t *src, uint32_t *dst,
                                                   const LK &lk, int32_t W, int32_t H,
                                                   int32_t k, const FloodGrid &g,
                                                   uint32_t logical, Q *lds)
{
    const TileQ tl = decode_tile_q(logical, g, k, H);
    if (tl.j0 >= tl.jend) return;
    const int32_t h = KC == 0 ? k : 4;
    const int32_t t = (int32_t)threadIdx.x;
    const int32_t oc = 4 * (tl.x0 + kQuad * t);
    const int32_t o1 = 4 * (tl.x0 - h + kQuad * t);
    const int32_t o2 = t < h / 2 ? 4 * (tl.x0 - h + kTWQ + kQuad * t) : INT32_MIN;
    const bool wave2 = __builtin_amdgcn_readfirstlane(t & ~63) < h / 2;   // any lane of the wave
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;
    constexpr int D = DL > 0 ? DL : NS - 2;   // rows between a row's label request and its lookups
    static_assert(D >= 1 && D <= NS - 2, "lookups need one row after the labels, one before use");
    struct Slot_ {
        G4 g1, g2;   // groups t and 256 + t
    };
    Slot_ ring[NS];
    const G4 none = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};   // label 0 -> sentinel 0
    Cursor in = cursor_at(src, tl.y0 + k, W);   // input row 2
    uint32_t lds_sel = 0;

    // Labels of input row s, and positions of input row s - D.
    auto request = [&](int32_t s, auto Slot, auto Phase) {
        constexpr int slot = decltype(Slot)::value, phase = decltype(Phase)::value;
        __amdgpu_buffer_rsrc_t r;
        if (phase < 2) {
            r = row_rsrc(src, tl.y0 + (s - 1) * k, W, H);
        } else {
            r = cursor_rsrc(in, W, H);
            advance(in, step_bytes, k);
        }
        Slot_ &q = ring[slot];
        q.g1.l = load4(r, o1);
        q.g2.l = wave2 ? load4(r, o2) : u32x4{0u, 0u, 0u, 0u};
        if (phase >= D) {
            Slot_ &n = ring[(slot + NS - D) % NS];
            const G4 &up1 = phase >= D + 1 ? ring[(slot + NS - D - 1) % NS].g1 : none;
            n.g1.s = lk.pos4(n.g1.l, up1);
            // The few halo groups are looked up without reuse: their loads
            // then write the positions directly under the wave-uniform
            // branch, with no select that would wait for them there.
            if (wave2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) n.g2.s[e] = lk.pos1(n.g2.l[e]);
            }
        }
    };
    auto fetch = [&](auto Slot) -> Three {
        const Slot_ &q = ring[decltype(Slot)::value];
        Q *row = (Q *)((char *)lds + lds_sel);
        lds_sel ^= (uint32_t)sizeof(Q);
        if (!LK::kLabelIsPos) row->l[t] = q.g1.l;
        row->s[t] = q.g1.s;
        if (wave2) {
            if (!LK::kLabelIsPos) row->l[kBlock + t] = q.g2.l;
            row->s[kBlock + t] = q.g2.s;
        }
        __syncthreads();
        // groups of columns x - h, x and x + h
        const int32_t ga = t, gb = t + h / kQuad, gc = t + 2 * (h / kQuad);
        Three th;
        th.a.s = row->s[ga];
        th.b.s = row->s[gb];
        th.c.s = row->s[gc];
        if (LK::kLabelIsPos) {
            th.a.l = th.a.s;
            th.b.l = th.b.s;
            th.c.l = th.c.s;
        } else {
            th.a.l = row->l[ga];
            th.b.l = row->l[gb];
            th.c.l = row->l[gc];
        }
        return th;
    };
    quad_walk<METRIC, VN, KC, NS, ST>(dst, W, H, k, tl, oc, request, fetch);
}

// Passes at a step k of at least a quarter of both sides (a JFA step's first
// two passes, k = k1 and k1 / 2, and a dJFA step's first ones when delta_1
// is that large).  Then the columns congruent to x0 mod k (x0 < k) number
// at most NB = 2 or 4 on the grid, x0 + m k for m < NB, and likewise the
// rows, so the NB x NB pixels {x0 + m k} x {y0 + n k} hold each other's
// candidates and nothing else: a lane owns one such block of four-column
// groups, loads its NB x NB groups once, folds every pixel's candidates
// from the block (the same column of each group, since k is a multiple of
// 4) and stores the groups.  The map streams through once, with no row or
// group read twice.  Groups off the grid read as unclaimed and are not
// stored (buffer range checks), exactly as in the walks above.
__host__ __device__ __forceinline__ int32_t block_span(int32_t W, int32_t H, int32_t k)
{
    if (W % kQuad != 0 || k % kQuad != 0) return 0;
    if (W <= 2 * k && H <= 2 * k) return 2;
    if (W <= 4 * k && H <= 4 * k) return 4;
    return 0;
}
__host__ __device__ __forceinline__ bool block_ok(int32_t W, int32_t H, int32_t k)
{
    return block_span(W, H, k) != 0;
}

// XY labels: the label is the position.
struct PosLabels {
    static constexpr bool kLabelIsPos = true;
    __device__ __forceinline__ u32x4 pos4(u32x4 l, const G4 &) const { return l; }
};

template <int NB, int METRIC, int VN, int ST, class LK>
__device__ __forceinline__ void flood_block_tile(const uint32_t *src, uint32_t *dst,
                                                 const LK &lk, int32_t W, int32_t H, int32_t k,
                                                 int32_t gx, int32_t y0)
{
    const int32_t x0 = kQuad * gx;
    const G4 none = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
    G4 q[NB][NB];   // [row m][column n]: the group at (x0 + n k, y0 + m k)
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const __amdgpu_buffer_rsrc_t r = row_rsrc(src, y0 + m * k, W, H);
#pragma unroll
        for (int n = 0; n < NB; ++n) q[m][n].l = load4(r, 4 * (x0 + n * k));
    }
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            q[m][n].s = lk.pos4(q[m][n].l, none);
            if (LK::kLabelIsPos) q[m][n].l = q[m][n].s;   // the translated label
        }
    const uint32_t p0 = ((uint32_t)(y0 + (int32_t)kOff) << 16) | (uint32_t)(x0 + (int32_t)kOff);
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const __amdgpu_buffer_rsrc_t out = row_rsrc(dst, y0 + m * k, W, H);
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const uint32_t pb = p0 + (uint32_t)(n * k) + ((uint32_t)(m * k) << 16);
            double best[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t p = pb + (uint32_t)e;
                double v = cand_key<METRIC>(p, Ent{q[m][n].l[e], q[m][n].s[e]});
#pragma unroll
                for (int dm = -1; dm <= 1; ++dm)
#pragma unroll
                    for (int dn = -1; dn <= 1; ++dn) {
                        const int mm = m + dm, nn = n + dn;
                        if ((dm == 0 && dn == 0) || mm < 0 || mm >= NB || nn < 0 || nn >= NB)
                            continue;
                        if (VN && dm != 0 && dn != 0) continue;
                        v = __builtin_fmin(v, cand_key<METRIC>(p, Ent{q[mm][nn].l[e],
                                                                      q[mm][nn].s[e]}));
                    }
                best[e] = v;
            }
            store4<ST>(labels_of(best), out, 4 * (x0 + n * k));
        }
    }
}

// The first two passes of a step, k and kh = k / 2, where both sides are at
// most 2 k (pair_ok): the 4 x 4 block of groups {x0 + n kh} x {y0 + m kh}
// (x0, y0 < kh) holds every candidate of both passes for its pixels (the
// first pass's partners lie two groups away, the second's one), so a lane
// loads its 16 groups once, runs the first pass into registers (pixels off
// the grid stay unclaimed, as the map would hold them between the passes),
// takes the positions of the labels it produced (ID: from the seed table)
// and runs the second pass.  Both passes take the Moore neighbourhood (the
// first two passes of a JFA step).
__host__ __device__ __forceinline__ bool pair_ok(int32_t W, int32_t H, int32_t k)
{
    return W % kQuad == 0 && k % (2 * kQuad) == 0 && W <= 2 * k && H <= 2 * k;
}

template <int METRIC, int ST, class LK>
__device__ __forceinline__ void flood_block_pair_tile(const uint32_t *src, uint32_t *dst,
                                                      const LK &lk, int32_t W, int32_t H,
                                                      int32_t kh, int32_t gx, int32_t y0)
{
    constexpr bool POS = LK::kLabelIsPos;   // positions are the labels: one array per level
    const int32_t x0 = kQuad * gx;
    const G4 none = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
    const uint32_t p0 = ((uint32_t)(y0 + (int32_t)kOff) << 16) | (uint32_t)(x0 + (int32_t)kOff);
    auto ent = [](const G4 &g, int e) { return Ent{g.l[e], POS ? g.l[e] : g.s[e]}; };
    G4 q[4][4];   // [row m][column n]: the group at (x0 + n kh, y0 + m kh)
    G4 h[4][4];   // the first pass's labels (and positions) there
    // The first pass pairs rows 0 with 2 and 1 with 3, so it runs on rows 0
    // and 2, then on rows 1 and 3: each pair of input rows is dead once its
    // outputs exist, which bounds the registers in use.
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const int m = half + 2 * mi;
            const __amdgpu_buffer_rsrc_t r = row_rsrc(src, y0 + m * kh, W, H);
#pragma unroll
            for (int n = 0; n < 4; ++n) q[m][n].l = load4(r, 4 * (x0 + n * kh));
        }
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int m = half + 2 * mi;
                if (POS)
                    q[m][n].l = lk.pos4(q[m][n].l, none);   // the translated label
                else
                    q[m][n].s = lk.pos4(q[m][n].l, none);
            }
        // first pass (step 2 kh): partners two groups away
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int m = half + 2 * mi;
                const uint32_t pb = p0 + (uint32_t)(n * kh) + ((uint32_t)(m * kh) << 16);
                double best[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t p = pb + (uint32_t)e;
                    double v = cand_key<METRIC>(p, ent(q[m][n], e));
#pragma unroll
                    for (int dm = -2; dm <= 2; dm += 2)
#pragma unroll
                        for (int dn = -2; dn <= 2; dn += 2) {
                            const int mm = m + dm, nn = n + dn;
                            if ((dm == 0 && dn == 0) || mm < 0 || mm >= 4 || nn < 0 || nn >= 4)
                                continue;
                            v = __builtin_fmin(v, cand_key<METRIC>(p, ent(q[mm][nn], e)));
                        }
                    best[e] = v;
                }
                u32x4 l = labels_of(best);
                const bool row_in = y0 + m * kh < H;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!row_in || x0 + n * kh + e >= W) l[e] = kEmpty;
                h[m][n].l = l;
            }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (!POS) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n) h[m][n].s = lk.pos4(h[m][n].l, none);
    }
    // second pass (step kh): partners one group away
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const __amdgpu_buffer_rsrc_t out = row_rsrc(dst, y0 + m * kh, W, H);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const uint32_t pb = p0 + (uint32_t)(n * kh) + ((uint32_t)(m * kh) << 16);
            double best[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t p = pb + (uint32_t)e;
                double v = cand_key<METRIC>(p, ent(h[m][n], e));
#pragma unroll
                for (int dm = -1; dm <= 1; ++dm)
#pragma unroll
                    for (int dn = -1; dn <= 1; ++dn) {
                        const int mm = m + dm, nn = n + dn;
                        if ((dm == 0 && dn == 0) || mm < 0 || mm >= 4 || nn < 0 || nn >= 4)
                            continue;
                        v = __builtin_fmin(v, cand_key<METRIC>(p, ent(h[mm][nn], e)));
                    }
                best[e] = v;
            }
            store4<ST>(labels_of(best), out, 4 * (x0 + n * kh));
        }
    }
}

// Column-class tile (steps of k >= 4 where a class fits one DPP row, see
// class_lanes).  The columns congruent to x0 mod k, x0 + m k, are the only
// ones a pixel of column x0 + m k takes candidates from, so lanes are given
// whole classes instead of adjacent columns: lane j of a class (C lanes per
// class, C a power of two up to 16, classes aligned to C lanes) owns the
// G groups m = G j .. G j + G - 1 (G = 2 or 4).  A group's
// neighbours at x -+ k are then the lane's own next groups, or for its
// first and last group the last group of lane j - 1 and the first of lane
// j + 1, which come over one DPP row shift each -- no shared rows, no halo,
// and each label is loaded and (ID labels) looked up once per row.  Rows
// are walked down the residue chain with quad_walk's rolling accumulators,
// one set per group.  Lanes whose class lies past k address offsets past
// the row (no memory access), so they neither read nor write.
constexpr int kClassMaxC = 16;      // lanes per class: one DPP row
constexpr int kClassMinStep = 128;  // below, the shared-row tiles' halo is small

// Lanes per class with G groups per lane, 0 if a class does not fit.
__host__ __device__ __forceinline__ int32_t class_lanes(int32_t W, int32_t k, int32_t G)
{
    if (W % kQuad != 0 || k % kQuad != 0 || k < kQuad) return 0;
    const int32_t members = (W + k - 1) / k;   // columns of class 0 on the grid
    const int32_t need = (members + G - 1) / G;
    int32_t c = 1;
    while (c < need) c <<= 1;
    return c <= kClassMaxC ? c : 0;
}

// Groups per lane of the column-class tile for a pass: 2 where a class fits
// 16 lanes of two, else 4 where it fits 16 of four, else 0 (not available).
__host__ __device__ __forceinline__ int32_t class_groups(int32_t W, int32_t k)
{
    return class_lanes(W, k, 2) ? 2 : (class_lanes(W, k, 4) ? 4 : 0);
}

// Grid of the column-class tile: ncol blocks of kBlock / C classes x
// min(k, H) chains x segments of at most L rows (chain-major, class-block
// minor, as flood_grid_quad numbers its tiles).
__host__ __device__ __forceinline__ int32_t class_blocks(int32_t k, int32_t C)
{
    const int32_t per = kBlock / C;   // classes per workgroup
    return (k / kQuad + per - 1) / per;
}

// Value of lane - 1 (east == false) or lane + 1 (east == true) within the
// lane's DPP row of 16 (row_shr:1 / row_shl:1); 0 for the lanes the shift
// leaves without one.  (Whole-wave shifts, which would let a class span 64
// lanes, measured slower.)
__device__ __forceinline__ uint32_t dpp_shift(uint32_t v, bool east)
{
    return east ? (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x101, 0xF, 0xF, true)
                : (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
}
__device__ __forceinline__ u32x4 dpp_shift4(u32x4 v, bool east)
{
    return u32x4{dpp_shift(v[0], east), dpp_shift(v[1], east), dpp_shift(v[2], east),
                 dpp_shift(v[3], east)};
}

template <int G, int METRIC, int VN, int NS, int ST, class LK>
__device__ __forceinline__ void flood_class_tile(const uint32_t *src, uint32_t *dst,
                                                 const LK &lk, int32_t W, int32_t H, int32_t k,
                                                 int32_t C, const FloodGrid &g, uint32_t logical)
{
    static_assert(NS == 3 || NS == 4, "ring of 3 or 4 rows");
    constexpr int A = NS - 1;                 // rows requested ahead of use
    constexpr int U = NS == 3 ? 3 : 12;       // lcm(3, NS)
    constexpr int D = NS - 2;                 // rows between a row's labels and its lookups
    // tile: class block, residue chain, segment
    const uint32_t cb = __builtin_amdgcn_readfirstlane(logical % g.ncol);
    const uint32_t rs = logical / g.ncol;
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(rs % g.nseg));
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)(rs / g.nseg));
    const int32_t nj = (H - 1 - r) / k + 1;
    const int32_t j0 = seg * g.L, jend = min(j0 + g.L, nj);
    if (j0 >= jend) return;
    const int32_t y0 = r + j0 * k;
    const int32_t nout = jend - j0;
    const int32_t t = (int32_t)threadIdx.x;
    const int32_t lane = t % C;   // lane of the class
    const int32_t x0 = kQuad * ((int32_t)cb * (kBlock / C) + t / C);
    const bool live = x0 < k;
    const bool first = lane == 0, last = lane == C - 1;
    int32_t oc[G];                // byte offsets of the lane's groups in a row
    uint32_t p0[G];               // packed position of each group's first pixel in row y0
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int32_t x = x0 + (G * lane + i) * k;
        oc[i] = live ? 4 * x : INT32_MIN;
        p0[i] = ((uint32_t)(y0 + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff);
    }
    const uint32_t step_bytes = 4u * (uint32_t)k * (uint32_t)W;
    const uint32_t pk = (uint32_t)k << 16;
    struct Slot_ {
        G4 q[G];
    };
    Slot_ ring[NS];
    const G4 none = {u32x4{0u, 0u, 0u, 0u}, u32x4{0u, 0u, 0u, 0u}};
    Cursor in = cursor_at(src, y0 + k, W);   // input row 2
    Cursor out = cursor_at(dst, y0, W);

    // Labels of input row s, and (ID labels) positions of input row s - D.
    auto request = [&](int32_t s, auto Slot, auto Phase) {
        constexpr int slot = decltype(Slot)::value, phase = decltype(Phase)::value;
        __amdgpu_buffer_rsrc_t rr;
        if (phase < 2) {
            rr = row_rsrc(src, y0 + (s - 1) * k, W, H);
        } else {
            rr = cursor_rsrc(in, W, H);
            advance(in, step_bytes, k);
        }
#pragma unroll
        for (int i = 0; i < G; ++i) ring[slot].q[i].l = load4(rr, oc[i]);
        if (!LK::kLabelIsPos && phase >= D) {
            Slot_ &n = ring[(slot + NS - D) % NS];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                const G4 &up = phase >= D + 1 ? ring[(slot + NS - D - 1) % NS].q[i] : none;
                n.q[i].s = lk.pos4(n.q[i].l, up);
            }
        }
    };
    // The row in a slot as one Three per group: the neighbours at x -+ k.
    auto fetch = [&](auto Slot, Three (&th)[G]) {
        const Slot_ &q = ring[decltype(Slot)::value];
        G4 grp[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            grp[i].l = q.q[i].l;
            grp[i].s = LK::kLabelIsPos ? q.q[i].l : q.q[i].s;
        }
        const u32x4 zero = {0u, 0u, 0u, 0u};
        G4 west, east;   // last group of lane - 1, first group of lane + 1
        west.l = dpp_shift4(grp[G - 1].l, false);
        east.l = dpp_shift4(grp[0].l, true);
        if (LK::kLabelIsPos) {
            west.s = west.l;
            east.s = east.l;
        } else {
            west.s = dpp_shift4(grp[G - 1].s, false);
            east.s = dpp_shift4(grp[0].s, true);
        }
        if (first) west = G4{zero, zero};
        if (last) east = G4{zero, zero};
#pragma unroll
        for (int i = 0; i < G; ++i) {
            th[i].a = i == 0 ? west : grp[i > 0 ? i - 1 : 0];
            th[i].b = grp[i];
            th[i].c = i == G - 1 ? east : grp[i < G - 1 ? i + 1 : 0];
        }
    };

    u32x4 prow[3][G];
    double acc[3][G][4];
    auto pre = [&](auto M) { request(decltype(M)::value, IC<decltype(M)::value % NS>{}, M); };
    pre(IC<0>{});
    pre(IC<1>{});
    pre(IC<2>{});
    if constexpr (A >= 3) pre(IC<3>{});
    {
        Three th[G];
        fetch(IC<0>{}, th);
#pragma unroll
        for (int i = 0; i < G; ++i) {
            prow[0][i] = u32x4{p0[i], p0[i] + 1, p0[i] + 2, p0[i] + 3};
            fold<METRIC, 0, VN != 0, true>(acc[0][i], prow[0][i], th[i]);
        }
    }
    pre(IC<A + 1>{});
    {
        Three th[G];
        fetch(IC<1>{}, th);
#pragma unroll
        for (int i = 0; i < G; ++i) {
            prow[1][i] = prow[0][i] + pk;
            fold<METRIC, 0, false, false>(acc[0][i], prow[0][i], th[i]);
            fold<METRIC, 0, VN != 0, true>(acc[1][i], prow[1][i], th[i]);
        }
    }
    int32_t s = 2;
    auto step = [&](auto I) -> bool {
        constexpr int u = (decltype(I)::value + 2) % U;   // s mod U
        constexpr int c0 = (u + 1) % 3, c1 = (u + 2) % 3, c2 = u % 3;
        if (s - 2 >= nout) return false;
        request(s + A, IC<(u + A) % NS>{}, IC<kSteady>{});
        Three th[G];
        fetch(IC<u % NS>{}, th);
        const __amdgpu_buffer_rsrc_t o = cursor_rsrc(out, W, H);
#pragma unroll
        for (int i = 0; i < G; ++i) {
            prow[c2][i] = prow[c1][i] + pk;
            fold<METRIC, 0, VN != 0, false>(acc[c0][i], prow[c0][i], th[i]);
            store4<ST>(labels_of(acc[c0][i]), o, oc[i]);
            fold<METRIC, 0, false, false>(acc[c1][i], prow[c1][i], th[i]);
            fold<METRIC, 0, VN != 0, true>(acc[c2][i], prow[c2][i], th[i]);
        }
        advance(out, step_bytes, k);
        ++s;
        return true;
    };
    auto round = [&](auto... I) -> bool { return (step(I) && ...); };
    while (expand<U>(round)) {
    }
}

// XY labels after a move (widths divisible by 4), one block of the map:
// each lane relabels four adjacent pixels in each of kRelabelRows rows at
// once -- all their label loads are requested, then all their gathers from
// the old-position index, then the results stored -- so the gathers of
// eight rows are in flight together.  A pixel whose label equals its left
// neighbour's in the group reuses that result (its gather goes to an offset
// past the map, which the hardware answers without a memory access); rows
// are independent of each other.  Block b covers 1024 columns of `rows`
// rows (a multiple of kRelabelRows); old positions lie near the pixels that
// carry them, so neighbouring rows share their index lines in L2.
constexpr int kRelabelRows = 8;

__device__ __forceinline__ void relabel_block(uint32_t *map, const uint32_t *idx, int32_t W,
                                              int32_t H, int32_t rows, uint32_t b)
{
    const int32_t strips = (W + kTWQ - 1) / kTWQ;
    const int32_t strip = (int32_t)(b % (uint32_t)strips);
    const int32_t y0 = (int32_t)(b / (uint32_t)strips) * rows;
    const int32_t y1 = min(y0 + rows, H);
    const int32_t off = 4 * (strip * kTWQ + kQuad * (int32_t)threadIdx.x);
    const __amdgpu_buffer_rsrc_t ir = __builtin_amdgcn_make_buffer_rsrc(
        (void *)idx, 0, (int32_t)min((int64_t)W * H * 4, (int64_t)0x7FFFFFFF), kRsrcWord3);
    const int32_t base = (int32_t)((kOff << 16) | kOff);
    for (int32_t y = y0; y < y1; y += kRelabelRows) {
        u32x4 l[kRelabelRows], v[kRelabelRows];
#pragma unroll
        for (int r = 0; r < kRelabelRows; ++r)   // rows past y1 read as unclaimed (size 0)
            l[r] = load4(row_rsrc(map, y + r < y1 ? y + r : H, W, H), off);
#pragma unroll
        for (int r = 0; r < kRelabelRows; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t le = l[r][e];
                const int32_t lx = (int32_t)(le & 0xFFFFu) - (int32_t)kOff;
                const int32_t ly = (int32_t)(le >> 16) - (int32_t)kOff;
                const bool valid = le != kEmpty && lx >= 0 && lx < W && ly >= 0 && ly < H;
                const bool reuse = e > 0 && le == l[r][e > 0 ? e - 1 : 0];
                const int32_t at = (valid && !reuse) ? 4 * (ly * W + lx) : -1;
                v[r][e] = __builtin_amdgcn_raw_buffer_load_b32(ir, at, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < kRelabelRows; ++r) {
            u32x4 n;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t le = l[r][e];
                const bool reuse = e > 0 && le == l[r][e > 0 ? e - 1 : 0];
                // a position, not a leftover label nor the all-ones of "no kept
                // seed" (label 0 and labels off the grid gathered nothing: 0)
                const uint32_t np = (int32_t)v[r][e] >= base ? v[r][e] : kEmpty;
                n[e] = reuse ? n[e > 0 ? e - 1 : 0] : np;
            }
            store4<0>(n, row_rsrc(map, y + r < y1 ? y + r : H, W, H), off);
        }
    }
}

// Blocks of relabel_block for a W x H map.
__host__ __device__ __forceinline__ int64_t relabel_blocks(int32_t W, int32_t H)
{
    return (int64_t)((W + kTWQ - 1) / kTWQ) * ((H + 4 * kRelabelRows - 1) / (4 * kRelabelRows));
}
constexpr int kRelabelBlockRows = 4 * kRelabelRows;

}  // namespace

}  // namespace vd
