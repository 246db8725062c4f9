// vdflood kernels for gfx950 (CDNA4, wave64).
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
#include "vd_kernels.h"

#include <utility>

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
constexpr int kMaxLdsK = 128;      // flood pass, shared-row variant: largest step
constexpr int kLdsRow = kTW + 2 * kMaxLdsK;   // entries of one shared row
constexpr int32_t kRsrcWord3 = 0x00020000;   // buffer descriptor word 3 on gfx9 parts

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef vd_i32x4 i32x4;


__global__ void __launch_bounds__(kBlock) k_fill(uint32_t *__restrict__ map, int64_t n,
                                                 uint32_t value)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        map[i] = value;
}

__device__ __forceinline__ int64_t pixel_of(uint32_t p, int32_t W)
{
    return (int64_t)((int32_t)(p >> 16) - (int32_t)kOff) * W +
           ((int32_t)(p & 0xFFFFu) - (int32_t)kOff);
}

__global__ void __launch_bounds__(kBlock) k_splat_reset(uint32_t *__restrict__ map,
                                                        const uint32_t *__restrict__ table,
                                                        int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) map[pixel_of(table[i + 1], W)] = 0xFFFFFFFFu;
}

__global__ void __launch_bounds__(kBlock) k_splat_min(uint32_t *__restrict__ map,
                                                      const uint32_t *__restrict__ table,
                                                      int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) atomicMin(&map[pixel_of(table[i + 1], W)], (uint32_t)(i + 1));
}

__global__ void __launch_bounds__(kBlock) k_splat_xy(uint32_t *__restrict__ map,
                                                     const uint32_t *__restrict__ table,
                                                     int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) {
        uint32_t p = table[i + 1];
        map[pixel_of(p, W)] = p;
    }
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

__global__ void __launch_bounds__(kBlock) k_move(uint32_t *__restrict__ table, int32_t S,
                                                 int32_t W, int32_t H, uint64_t move_seed,
                                                 uint64_t t, int32_t lo, uint32_t span)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    uint64_t n = ((t - 1) * (uint64_t)S + (uint64_t)i) * 2u;
    uint32_t p = table[i + 1];
    int32_t x = (int32_t)(p & 0xFFFFu) - (int32_t)kOff + draw(move_seed, n + 0, lo, span);
    int32_t y = (int32_t)(p >> 16) - (int32_t)kOff + draw(move_seed, n + 1, lo, span);
    x = min(max(x, 0), W - 1);
    y = min(max(y, 0), H - 1);
    table[i + 1] = ((uint32_t)(y + (int32_t)kOff) << 16) | (uint32_t)(x + (int32_t)kOff);
}

__global__ void __launch_bounds__(kBlock) k_relabel(uint32_t *__restrict__ map,
                                                    const uint32_t *__restrict__ idx,
                                                    const uint32_t *__restrict__ table,
                                                    int32_t S, int32_t W, int32_t H)
{
    int64_t n = (int64_t)W * H;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t l = map[p];
        if (l == kEmpty) continue;
        int32_t lx = (int32_t)(l & 0xFFFFu) - (int32_t)kOff;
        int32_t ly = (int32_t)(l >> 16) - (int32_t)kOff;
        uint32_t i = (lx >= 0 && lx < W && ly >= 0 && ly < H) ? idx[(int64_t)ly * W + lx] : 0u;
        map[p] = (i >= 1 && i <= (uint32_t)S) ? table[i] : kEmpty;
    }
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

// ---------------------------------------------------------------------------
// Flood pass.
//
// Residue-chain schedule.  At step k, output row y reads input rows y - k,
// y and y + k, which all lie on the chain of rows congruent to y mod k.  A
// workgroup owns 256 adjacent columns of a segment of one chain and walks it
// downwards with a window of three input rows held in registers, so each
// input row is fetched once per segment (plus two rows of overlap between
// segments) whatever k is.  The next row is requested one iteration ahead.
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

// Labels of one row (columns x - k, x, x + k); off-grid reads return 0.
__device__ __forceinline__ void load_labels(Row &row, const uint32_t *src, int32_t y, int32_t W,
                                            int32_t H, int32_t ow, int32_t oc, int32_t oe)
{
    __amdgpu_buffer_rsrc_t r = row_rsrc(src, y, W, H);
    row.w.l = __builtin_amdgcn_raw_buffer_load_b32(r, ow, 0, 0);
    row.c.l = __builtin_amdgcn_raw_buffer_load_b32(r, oc, 0, 0);
    row.e.l = __builtin_amdgcn_raw_buffer_load_b32(r, oe, 0, 0);
}

// Seed positions of a row's labels: ID labels index the seed table (entry 0,
// the unclaimed label, is the sentinel); XY labels are positions already.
template <int LABEL>
__device__ __forceinline__ void lookup_positions(Row &row, i32x4 tab)
{
    if (LABEL == kLabelId) {
        row.w.s = vd_struct_buffer_load(tab, (int32_t)row.w.l, 0, 0, 0);
        row.c.s = vd_struct_buffer_load(tab, (int32_t)row.c.l, 0, 0, 0);
        row.e.s = vd_struct_buffer_load(tab, (int32_t)row.e.l, 0, 0, 0);
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
    short2_t dv = __builtin_bit_cast(short2_t, p) - __builtin_bit_cast(short2_t, e.s);
    int32_t d;
    if (METRIC == kEuclid)
        d = __builtin_amdgcn_sdot2(dv, dv, 0, false);
    else
        d = abs((int32_t)dv.x) + abs((int32_t)dv.y);
    return __hiloint2double(d, (int32_t)e.l);
}

// Output row y from the window a (row y - k), b (row y), c (row y + k).
template <int METRIC, int VN>
__device__ __forceinline__ void emit(uint32_t *dst, const Row &a, const Row &b, const Row &c,
                                     int32_t y, int32_t k, int32_t W, int32_t H, uint32_t px,
                                     int32_t oc)
{
    uint32_t p = ((uint32_t)(y + (int32_t)kOff) << 16) | px;
    double best = cand_key<METRIC>(p, b.c);
    best = __builtin_fmin(best, cand_key<METRIC>(p, b.w));
    best = __builtin_fmin(best, cand_key<METRIC>(p, b.e));
    if (y >= k) {
        best = __builtin_fmin(best, cand_key<METRIC>(p, a.c));
        if (!VN) {
            best = __builtin_fmin(best, cand_key<METRIC>(p, a.w));
            best = __builtin_fmin(best, cand_key<METRIC>(p, a.e));
        }
    }
    if (y + k < H) {
        best = __builtin_fmin(best, cand_key<METRIC>(p, c.c));
        if (!VN) {
            best = __builtin_fmin(best, cand_key<METRIC>(p, c.w));
            best = __builtin_fmin(best, cand_key<METRIC>(p, c.e));
        }
    }
    __builtin_amdgcn_raw_buffer_store_b32((uint32_t)__double2loint(best), row_rsrc(dst, y, W, H),
                                          oc, 0, 0);
}

template <int LABEL, int METRIC, int VN, int P>
__global__ void __launch_bounds__(kTW) k_flood(const uint32_t *__restrict__ src,
                                               uint32_t *__restrict__ dst,
                                               const uint32_t *__restrict__ table, uint32_t S,
                                               int32_t W, int32_t H, int32_t k, uint32_t ncol,
                                               uint32_t nseg, int32_t L, uint32_t nblocks)
{
    // The integer divisions below run on the vector unit; readfirstlane
    // tells the compiler their results are wave-uniform, so every row
    // address and buffer descriptor derived from them stays scalar.
    const uint32_t b = blockIdx.x;
    const uint32_t q = nblocks >> 3, rem = nblocks & 7u, xcd = b & 7u;
    const uint32_t logical = xcd * q + min(xcd, rem) + (b >> 3);
    const uint32_t col = __builtin_amdgcn_readfirstlane(logical % ncol);
    const uint32_t rs = logical / ncol;
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(rs % nseg));
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)(rs / nseg));   // chain: rows r, r + k, ...
    const int32_t nj = (H - 1 - r) / k + 1;             // rows on this chain
    int32_t j = seg * L;
    if (j >= nj) return;
    const int32_t jend = min(j + L, nj);
    const int32_t x = (int32_t)(col * kTW + threadIdx.x);
    const uint32_t px = (uint32_t)(x + (int32_t)kOff);
    const int32_t ow = 4 * (x - k), oc = 4 * x, oe = 4 * (x + k);
    const uint64_t ta = (uint64_t)table;
    const i32x4 tab = {(int32_t)(uint32_t)ta, (int32_t)(((uint32_t)(ta >> 32) & 0xFFFFu) | (4u << 16)),
                       (int32_t)(S + 1), kRsrcWord3};
    int32_t y = r + j * k;

    // NR row registers rotate through the roles: at unrolled step u, slot
    // (u + m + 1) % NR holds row y + m*k for m = -1 .. P.  Labels are
    // requested P + 1 rows ahead of the output row and their positions P
    // rows ahead, so neither load is waited for in the step that issues it.
    // The loop is unrolled NR times, so no row is ever copied.
    constexpr int NR = P + 3;
    Row R[NR];
#pragma unroll
    for (int m = -1; m <= P; ++m) load_labels(R[m + 1], src, y + m * k, W, H, ow, oc, oe);
#pragma unroll
    for (int m = -1; m < P; ++m) lookup_positions<LABEL>(R[m + 1], tab);
    // One output row with the slots of unrolled step U; false once the
    // segment is done.
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        if (j >= jend) return false;
        load_labels(R[(u + NR - 1) % NR], src, y + (P + 1) * k, W, H, ow, oc, oe);
        lookup_positions<LABEL>(R[(u + NR - 2) % NR], tab);
        emit<METRIC, VN>(dst, R[u % NR], R[(u + 1) % NR], R[(u + 2) % NR], y, k, W, H, px, oc);
        ++j;
        y += k;
        return true;
    };
    auto round = [&](auto... U) -> bool { return (step(U) && ...); };
    while (expand<NR>(round)) {
    }
}

// Shared-row variant (steps k <= kMaxLdsK).  The same chain walk, but the
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

template <int LABEL, int METRIC, int VN, int P>
__global__ void __launch_bounds__(kTW) k_flood_lds(const uint32_t *__restrict__ src,
                                                   uint32_t *__restrict__ dst,
                                                   const uint32_t *__restrict__ table,
                                                   uint32_t S, int32_t W, int32_t H, int32_t k,
                                                   uint32_t ncol, uint32_t nseg, int32_t L,
                                                   uint32_t nblocks)
{
    __shared__ uint2 lds[2][kLdsRow];
    const uint32_t b = blockIdx.x;
    const uint32_t q = nblocks >> 3, rem = nblocks & 7u, xcd = b & 7u;
    const uint32_t logical = xcd * q + min(xcd, rem) + (b >> 3);
    const uint32_t col = __builtin_amdgcn_readfirstlane(logical % ncol);
    const uint32_t rs = logical / ncol;
    const int32_t seg = __builtin_amdgcn_readfirstlane((int32_t)(rs % nseg));
    const int32_t r = __builtin_amdgcn_readfirstlane((int32_t)(rs / nseg));
    const int32_t nj = (H - 1 - r) / k + 1;
    int32_t j = seg * L;
    if (j >= nj) return;
    const int32_t jend = min(j + L, nj);
    const int32_t t = (int32_t)threadIdx.x;
    const int32_t x0 = (int32_t)col * kTW;
    const int32_t x = x0 + t;
    const uint32_t px = (uint32_t)(x + (int32_t)kOff);
    const int32_t oc = 4 * x;
    // entry t is column x0 - k + t; entry kTW + t (only for t < 2k) is
    // column x0 + kTW - k + t; an unused second entry reads out of range
    const int32_t o1 = 4 * (x0 - k + t);
    const bool has2 = t < 2 * k;
    const int32_t o2 = has2 ? 4 * (x0 + kTW - k + t) : INT32_MIN;
    const bool wave2 = __builtin_amdgcn_readfirstlane(t & ~63) < 2 * k;   // any lane of the wave
    const uint64_t ta = (uint64_t)table;
    const i32x4 tab = {(int32_t)(uint32_t)ta, (int32_t)(((uint32_t)(ta >> 32) & 0xFFFFu) | (4u << 16)),
                       (int32_t)(S + 1), kRsrcWord3};
    int32_t y = r + j * k;
    int32_t exchanges = 0;

    auto load = [&](Slot &sl, int32_t yy) {
        __amdgpu_buffer_rsrc_t rr = row_rsrc(src, yy, W, H);
        sl.raw.l1 = __builtin_amdgcn_raw_buffer_load_b32(rr, o1, 0, 0);
        sl.raw.l2 = wave2 ? __builtin_amdgcn_raw_buffer_load_b32(rr, o2, 0, 0) : 0u;
    };
    auto lookup = [&](Slot &sl) {
        if (LABEL == kLabelId) {
            sl.raw.s1 = vd_struct_buffer_load(tab, (int32_t)sl.raw.l1, 0, 0, 0);
            sl.raw.s2 = wave2 ? vd_struct_buffer_load(tab, (int32_t)sl.raw.l2, 0, 0, 0) : 0u;
        } else {
            sl.raw.s1 = sl.raw.l1;
            sl.raw.s2 = sl.raw.l2;
        }
    };
    auto exchange = [&](Slot &sl) {
        uint2 *row = lds[exchanges & 1];
        ++exchanges;
        row[t] = make_uint2(sl.raw.l1, sl.raw.s1);
        if (has2) row[kTW + t] = make_uint2(sl.raw.l2, sl.raw.s2);
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
    for (int m = -1; m <= P; ++m) load(R[m + 1], y + m * k);
#pragma unroll
    for (int m = -1; m < P; ++m) lookup(R[m + 1]);
    exchange(R[0]);
    exchange(R[1]);
    auto step = [&](auto U) -> bool {
        constexpr int u = decltype(U)::value;
        if (j >= jend) return false;
        load(R[(u + NR - 1) % NR], y + (P + 1) * k);
        lookup(R[(u + NR - 2) % NR]);
        exchange(R[(u + 2) % NR]);
        emit<METRIC, VN>(dst, R[u % NR].win, R[(u + 1) % NR].win, R[(u + 2) % NR].win, y, k, W,
                         H, px, oc);
        ++j;
        y += k;
        return true;
    };
    auto round = [&](auto... U) -> bool { return (step(U) && ...); };
    while (expand<NR>(round)) {
    }
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
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_reset, grid1d(S), dim3(kBlock), 0, s, map, table, S, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splat_min, grid1d(S), dim3(kBlock), 0, s, map, table, S, W);
    return hipGetLastError();
}

hipError_t launch_splat_xy(uint32_t *map, const uint32_t *table, int32_t S, int32_t W,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_xy, grid1d(S), dim3(kBlock), 0, s, map, table, S, W);
    return hipGetLastError();
}

hipError_t launch_move(uint32_t *table, int32_t S, int32_t W, int32_t H, uint64_t move_seed,
                       int64_t t, int32_t lo, int32_t hi, hipStream_t s)
{
    hipLaunchKernelGGL(k_move, grid1d(S), dim3(kBlock), 0, s, table, S, W, H, move_seed,
                       (uint64_t)t, lo, (uint32_t)(hi - lo + 1));
    return hipGetLastError();
}

hipError_t launch_index_old(uint32_t *idx, const uint32_t *old_table, int32_t S, int32_t W,
                            hipStream_t s)
{
    return launch_splat_id(idx, old_table, S, W, s);
}

hipError_t launch_relabel(uint32_t *map, const uint32_t *idx, const uint32_t *table,
                          int32_t S, int32_t W, int32_t H, hipStream_t s)
{
    hipLaunchKernelGGL(k_relabel, grid1d((int64_t)W * H, 8192), dim3(kBlock), 0, s, map, idx,
                       table, S, W, H);
    return hipGetLastError();
}

hipError_t launch_export(const uint32_t *map, uint32_t *out, int64_t n, int32_t label,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_export, grid1d(n, 8192), dim3(kBlock), 0, s, map, out, n, label);
    return hipGetLastError();
}

hipError_t launch_flood(const uint32_t *src, uint32_t *dst, const uint32_t *table, int32_t S,
                        int32_t W, int32_t H, int32_t k, int32_t vn, int32_t label,
                        int32_t metric, int32_t variant, hipStream_t s)
{
    // Segment length: long enough to amortise the two overlap rows, short
    // enough to give the 256 CUs about 2048 workgroups.
    int64_t npix = (int64_t)W * H;
    int32_t L = (int32_t)(npix / ((int64_t)kTW * 2048));
    L = L < 1 ? 1 : (L > kMaxSegRows ? kMaxSegRows : L);
    uint32_t ncol = (uint32_t)((W + kTW - 1) / kTW);
    uint32_t nres = (uint32_t)(k < H ? k : H);
    int32_t chain = (H + k - 1) / k;                      // rows on the longest chain
    uint32_t nseg = (uint32_t)((chain + L - 1) / L);
    uint64_t nblocks = (uint64_t)ncol * nres * nseg;
    if (k < 1 || nblocks == 0 || nblocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks), block(kTW);
    uint32_t nb = (uint32_t)nblocks, uS = (uint32_t)S;
#define VD_LAUNCH(LB, MT, V, P)                                                              \
    hipLaunchKernelGGL((k_flood<LB, MT, V, P>), grid, block, 0, s, src, dst, table, uS, W, H,  \
                       k, ncol, nseg, L, nb)
#define VD_LAUNCH_LDS(LB, MT, V, P)                                                           \
    hipLaunchKernelGGL((k_flood_lds<LB, MT, V, P>), grid, block, 0, s, src, dst, table, uS, W,  \
                       H, k, ncol, nseg, L, nb)
#define VD_LAUNCH_P(LB, MT, V)                                                                \
    do {                                                                                      \
        if (variant == 0) VD_LAUNCH(LB, MT, V, 1);                                            \
        else if (variant == 1 || (variant == 3 && k > kMaxLdsK)) VD_LAUNCH(LB, MT, V, 2);     \
        else if (variant == 2) VD_LAUNCH(LB, MT, V, 3);                                       \
        else VD_LAUNCH_LDS(LB, MT, V, 2);                                                     \
    } while (0)
    if (variant < 0 || variant >= kFloodVariants) return hipErrorInvalidValue;
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

}  // namespace vd
