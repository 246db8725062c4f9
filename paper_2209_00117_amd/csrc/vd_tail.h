// The last passes of a step fused into one launch (temporal blocking of the
// small-k tail).  A JFA or dJFA step ends with passes at k = 4, 2, 1 (plus
// JFA+1 / JFA+2's extra k = 1 or k = 2, 1); each is a Jacobi pass over the
// whole map (Sec. III, Table I; Sec. V-B).  Run separately, every one of
// them streams the map in and out.  Here a workgroup loads one tile of the
// input map with a halo of h = sum of the fused steps (at most kTailHalo)
// into LDS, as (label, seed position) pairs, and runs the passes on it in
// LDS: pass i computes the tile grown by the halo the later passes still
// need, reading the previous pass's buffer; the last pass writes the tile's
// output pixels to the map.  So the fused passes cost one read and one
// write of the map (plus the halo re-reads, from L2) and one seed-table
// lookup per loaded pixel and per label a pass changes, instead of a full
// read, write and lookups per pass.
//
// The result is the same map as the passes run one after another: every
// entry a pass computes sees exactly the candidates it would see in the
// full map, because the tile grows by k on each side per earlier pass.
// Pixels off the grid stay unclaimed (label 0, sentinel position) in every
// buffer, so a candidate off the grid loses to every claimed one, as in the
// single passes.
#pragma once

#include "vd_device.h"

namespace vd {

namespace {

constexpr int kTailTW = 48;                          // output columns per tile
constexpr int kTailBW = kTailTW + 2 * kTailHalo;     // 64 entries per LDS row

// A tile buffer for TH output rows (tile heights 16, 24 or 32 trade halo
// work for occupancy: two buffers take 32, 40 or 48 KiB of LDS).
template <int TH>
struct TailBuf {
    static constexpr int kRows = TH + 2 * kTailHalo;
    uint2 e[kRows][kTailBW];   // (label, seed position)
};

// Work layout.  A tile buffer row has 64 entries, one per lane of a wave:
// lane i always handles buffer column i (clamped into the rectangle a
// phase covers, so every LDS access stays inside the buffer; lanes past
// the rectangle compute a duplicate and do not write).  The load spreads
// rows over the four waves (wave w: rows w, w + 4, ...), requesting all of
// a lane's labels, then all their seed positions, before writing any.  A
// pass at step K walks the rows of each residue class mod K as a chain
// with a window of three rows in registers (rows y - K, y, y + K, each as
// the entries x - K, x, x + K), so an output row costs three LDS reads per
// lane; the K chains are cut into 4 / K segments, one per wave.
static_assert(kTailBW == 64, "one buffer column per lane");

// Loads the tile's input with halo h: entry (cx, cy) of `buf` is map pixel
// (x0 - kTailHalo + cx, y0 - kTailHalo + cy).
template <int LABEL, int TH>
__device__ __forceinline__ void tail_load(TailBuf<TH> &buf, __amdgpu_buffer_rsrc_t src,
                                          i32x4 tab, int32_t W, int32_t H, int32_t x0,
                                          int32_t y0, int32_t h)
{
    constexpr int kTailRowsPerWave = (TailBuf<TH>::kRows + 3) / 4;
    const int32_t lane = (int32_t)(threadIdx.x & 63u);
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t b0 = kTailHalo - h, w = kTailTW + 2 * h, nh = TH + 2 * h;
    const int32_t cx = b0 + min(lane, w - 1);
    const int32_t gx = x0 - kTailHalo + cx;
    const bool col_on = lane < w && (uint32_t)gx < (uint32_t)W;
    uint32_t l[kTailRowsPerWave], sp[kTailRowsPerWave];
#pragma unroll
    for (int i = 0; i < kTailRowsPerWave; ++i) {
        const int32_t cy = b0 + wave + 4 * i;
        const int32_t gy = y0 - kTailHalo + cy;
        const bool on = col_on && (wave + 4 * i) < nh && (uint32_t)gy < (uint32_t)H;
        // off the grid: an offset past the map, answered with 0 (unclaimed)
        l[i] = __builtin_amdgcn_raw_buffer_load_b32(src, on ? 4 * (gy * W + gx) : -1, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < kTailRowsPerWave; ++i)
        sp[i] = LABEL == kLabelId ? vd_struct_buffer_load(tab, l[i] ? (int32_t)l[i] : -1, 0, 0, 0)
                                  : l[i];
#pragma unroll
    for (int i = 0; i < kTailRowsPerWave; ++i)
        if (lane < w && wave + 4 * i < nh) buf.e[b0 + wave + 4 * i][cx] = make_uint2(l[i], sp[i]);
}

// One fused pass at step K over the tile grown by r (the halo the later
// passes still need).  LAST: the tile's own pixels go to the map.  The
// three window rows rotate through three register slots; the walk is
// unrolled by three so that the rotation is static (no row is copied).
template <int LABEL, int METRIC, int K, int VN, bool LAST, int ST, int TH>
__device__ __forceinline__ void tail_pass(const TailBuf<TH> &in, TailBuf<TH> &out,
                                          __amdgpu_buffer_rsrc_t dst, i32x4 tab, int32_t W,
                                          int32_t H, int32_t x0, int32_t y0, int32_t r)
{
    const int32_t lane = (int32_t)(threadIdx.x & 63u);
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t b0 = kTailHalo - r, w = kTailTW + 2 * r, nh = TH + 2 * r;
    const int32_t cx = b0 + min(lane, w - 1);
    const int32_t gx = x0 - kTailHalo + cx;
    // gx_on is a property of the (clamped) column, so a duplicating lane
    // computes exactly what the lane it duplicates computes
    const bool gx_on = (uint32_t)gx < (uint32_t)W;
    const bool mine = lane < w;
    // this wave's segment of chain c (rows b0 + c + K*j, j in [j0, j1))
    constexpr int NSEG = 4 / K;
    const int32_t c = wave % K, seg = wave / K;
    const int32_t len = (nh - c + K - 1) / K;
    const int32_t L = (len + NSEG - 1) / NSEG;
    const int32_t j0 = seg * L, j1 = min(j0 + L, len);
    const int32_t n = j1 - j0;   // wave-uniform
    if (n <= 0) return;
    const int32_t cy = b0 + c + K * j0;
    constexpr int RS = kTailBW;   // entries per buffer row
    // Lanes past the rectangle duplicate its last column: their LDS writes
    // repeat that column's value at the same address, which is harmless;
    // their map stores are dropped.
    const uint2 *q = &in.e[cy][cx];
    uint2 *o = &out.e[cy][cx];
    int32_t gy = y0 - kTailHalo + cy;
    uint32_t p = ((uint32_t)(gy + (int32_t)kOff) << 16) | (uint32_t)(gx + (int32_t)kOff);
    auto ld = [](Row &R, const uint2 *at) {
        const uint2 a = at[-K], m = at[0], e = at[K];
        R = Row{Ent{a.x, a.y}, Ent{m.x, m.y}, Ent{e.x, e.y}};
    };
    Row R[3];
    ld(R[0], q - K * RS);
    ld(R[1], q);
    int32_t i = 0;
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        if (i >= n) return false;
        const Row &A = R[u % 3], &B = R[(u + 1) % 3];
        Row &C = R[(u + 2) % 3];
        ld(C, q + K * RS);
        double best = cand_key<METRIC>(p, B.c);
        best = __builtin_fmin(best, cand_key<METRIC>(p, B.w));
        best = __builtin_fmin(best, cand_key<METRIC>(p, B.e));
        best = __builtin_fmin(best, cand_key<METRIC>(p, A.c));
        best = __builtin_fmin(best, cand_key<METRIC>(p, C.c));
        if (!VN) {
            best = __builtin_fmin(best, cand_key<METRIC>(p, A.w));
            best = __builtin_fmin(best, cand_key<METRIC>(p, A.e));
            best = __builtin_fmin(best, cand_key<METRIC>(p, C.w));
            best = __builtin_fmin(best, cand_key<METRIC>(p, C.e));
        }
        const uint32_t l = (uint32_t)__double2loint(best);
        const bool on = gx_on && (uint32_t)gy < (uint32_t)H;
        if (LAST) {
            // the tile's pixels; lanes past it and pixels off the grid are dropped
            __builtin_amdgcn_raw_buffer_store_b32(l, dst, on && mine ? 4 * (gy * W + gx) : -1, 0,
                                                  ST);
        } else {
            // a label the pass did not change keeps its position
            const uint32_t sp = LABEL == kLabelId ? seed_pos(l, B.c.l, B.c.s, tab) : l;
            *o = on ? make_uint2(l, sp) : make_uint2(0u, 0u);
        }
        q += K * RS;
        o += K * RS;
        gy += K;
        p += (uint32_t)K << 16;
        ++i;
        return true;
    };
    auto round = [&](auto... U) -> bool { return (step(U) && ...); };
    while (expand<3>(round)) {
    }
}

// Runtime (k, vn) of a fused pass -> its compiled form.
template <int LABEL, int METRIC, bool LAST, int ST, int TH>
__device__ __forceinline__ void tail_pass_rt(int32_t k, int32_t vn, const TailBuf<TH> &in,
                                             TailBuf<TH> &out, __amdgpu_buffer_rsrc_t dst,
                                             i32x4 tab, int32_t W, int32_t H, int32_t x0,
                                             int32_t y0, int32_t r)
{
#define VD_TAIL_PASS(K, V) \
    tail_pass<LABEL, METRIC, K, V, LAST, ST, TH>(in, out, dst, tab, W, H, x0, y0, r)
    switch (2 * k + (vn ? 1 : 0)) {
    case 2: VD_TAIL_PASS(1, 0); break;
    case 3: VD_TAIL_PASS(1, 1); break;
    case 4: VD_TAIL_PASS(2, 0); break;
    case 5: VD_TAIL_PASS(2, 1); break;
    case 8: VD_TAIL_PASS(4, 0); break;
    default: VD_TAIL_PASS(4, 1); break;
    }
#undef VD_TAIL_PASS
}

// One tile of the fused passes (the plan's steps are 1, 2 or 4 and sum to
// at most kTailHalo; the launcher checks).
template <int LABEL, int METRIC, int ST, int TH>
__device__ __forceinline__ void flood_tail_tile(const uint32_t *src, uint32_t *dst,
                                                const uint32_t *table, uint32_t S, int32_t W,
                                                int32_t H, const TailPlan &plan,
                                                uint32_t logical, TailBuf<TH> (&buf)[2])
{
    const uint32_t tx = __builtin_amdgcn_readfirstlane(logical % plan.ntx);
    const uint32_t ty = __builtin_amdgcn_readfirstlane(logical / plan.ntx);
    const int32_t x0 = (int32_t)tx * kTailTW, y0 = (int32_t)ty * TH;
    const int32_t bytes = (int32_t)min((int64_t)W * H * 4, (int64_t)0x7FFFFFFF);
    const __amdgpu_buffer_rsrc_t sr = __builtin_amdgcn_make_buffer_rsrc((void *)src, 0, bytes,
                                                                        kRsrcWord3);
    const __amdgpu_buffer_rsrc_t dr = __builtin_amdgcn_make_buffer_rsrc((void *)dst, 0, bytes,
                                                                        kRsrcWord3);
    const i32x4 tab = table_rsrc(table, S);
    int32_t r = plan.halo;
    tail_load<LABEL, TH>(buf[0], sr, tab, W, H, x0, y0, r);
    __syncthreads();
    for (int32_t i = 0; i < plan.n; ++i) {
        r -= plan.k[i];
        const TailBuf<TH> &in = buf[i & 1];
        TailBuf<TH> &out = buf[(i + 1) & 1];
        if (i + 1 < plan.n) {
            tail_pass_rt<LABEL, METRIC, false, ST, TH>(plan.k[i], plan.vn[i], in, out, dr, tab,
                                                       W, H, x0, y0, r);
            __syncthreads();
        } else {
            tail_pass_rt<LABEL, METRIC, true, ST, TH>(plan.k[i], plan.vn[i], in, out, dr, tab, W,
                                                      H, x0, y0, r);
        }
    }
}

}  // namespace

}  // namespace vd
