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

template <int LABEL>
__device__ __forceinline__ Ent make_ent(uint32_t l, i32x4 tab)
{
    Ent e;
    e.l = l;
    e.s = LABEL == kLabelId ? vd_struct_buffer_load(tab, (int32_t)l, 0, 0, 0) : l;
    return e;
}

template <int LABEL>
__device__ __forceinline__ Row load_row(const uint32_t *src, int32_t y, int32_t W, int32_t H,
                                        i32x4 tab, int32_t ow, int32_t oc, int32_t oe)
{
    __amdgpu_buffer_rsrc_t r = row_rsrc(src, y, W, H);
    Row row;
    row.w = make_ent<LABEL>(__builtin_amdgcn_raw_buffer_load_b32(r, ow, 0, 0), tab);
    row.c = make_ent<LABEL>(__builtin_amdgcn_raw_buffer_load_b32(r, oc, 0, 0), tab);
    row.e = make_ent<LABEL>(__builtin_amdgcn_raw_buffer_load_b32(r, oe, 0, 0), tab);
    return row;
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

template <int LABEL, int METRIC, int VN>
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

    // Four row registers rotate through the roles (above, current, below,
    // prefetched); the loop is unrolled four times so no row is copied.
    Row r0 = load_row<LABEL>(src, y - k, W, H, tab, ow, oc, oe);
    Row r1 = load_row<LABEL>(src, y, W, H, tab, ow, oc, oe);
    Row r2 = load_row<LABEL>(src, y + k, W, H, tab, ow, oc, oe);
    Row r3;
#define VD_FLOOD_STEP(A, B, C, N)                                                       \
    {                                                                                   \
        if (j >= jend) break;                                                           \
        N = load_row<LABEL>(src, y + 2 * k, W, H, tab, ow, oc, oe);                       \
        emit<METRIC, VN>(dst, A, B, C, y, k, W, H, px, oc);                              \
        ++j;                                                                            \
        y += k;                                                                         \
    }
    for (;;) {
        VD_FLOOD_STEP(r0, r1, r2, r3)
        VD_FLOOD_STEP(r1, r2, r3, r0)
        VD_FLOOD_STEP(r2, r3, r0, r1)
        VD_FLOOD_STEP(r3, r0, r1, r2)
    }
#undef VD_FLOOD_STEP
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
                        int32_t metric, hipStream_t s)
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
#define VD_LAUNCH(LB, MT, V)                                                                 \
    hipLaunchKernelGGL((k_flood<LB, MT, V>), grid, block, 0, s, src, dst, table, uS, W, H, k, \
                       ncol, nseg, L, nb)
    if (label == kLabelId) {
        if (metric == kEuclid) {
            if (vn) VD_LAUNCH(kLabelId, kEuclid, 1); else VD_LAUNCH(kLabelId, kEuclid, 0);
        } else {
            if (vn) VD_LAUNCH(kLabelId, kManhattan, 1); else VD_LAUNCH(kLabelId, kManhattan, 0);
        }
    } else {
        if (metric == kEuclid) {
            if (vn) VD_LAUNCH(kLabelXy, kEuclid, 1); else VD_LAUNCH(kLabelXy, kEuclid, 0);
        } else {
            if (vn) VD_LAUNCH(kLabelXy, kManhattan, 1); else VD_LAUNCH(kLabelXy, kManhattan, 0);
        }
    }
#undef VD_LAUNCH
    return hipGetLastError();
}

}  // namespace vd
