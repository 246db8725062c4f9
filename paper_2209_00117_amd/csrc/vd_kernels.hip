// vdflood kernels for gfx950 (CDNA4, wave64).
//
// Flood pass (Sec. III, Table I; Sec. V-B, Alg. 1).  The paper's kernel has
// each pixel push its seed into its neighbours in place, which races when
// two pixels push into one.  Here each pixel gathers from the symmetric
// neighbourhood instead and the pass reads one buffer and writes the other,
// so the result is a function of the input map alone.
//
// Candidate order: (distance, label) compared lexicographically as one
// 64-bit key, distance in the high word.  A missing candidate (off the grid
// or EMPTY) never becomes the minimum; if every candidate is missing the key
// stays all ones and its low word is kEmpty.
#include "vd_kernels.h"

namespace vd {

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_fill(uint32_t *__restrict__ map, int64_t n,
                                                 uint32_t value)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        map[i] = value;
}

__device__ __forceinline__ int64_t pixel_of(uint32_t p, int32_t W)
{
    return (int64_t)(p >> 16) * W + (p & 0xFFFFu);
}

__global__ void __launch_bounds__(kBlock) k_splat_reset(uint32_t *__restrict__ map,
                                                        const uint32_t *__restrict__ pos,
                                                        int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) map[pixel_of(pos[i], W)] = kEmpty;
}

__global__ void __launch_bounds__(kBlock) k_splat_min(uint32_t *__restrict__ map,
                                                      const uint32_t *__restrict__ pos,
                                                      int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) atomicMin(&map[pixel_of(pos[i], W)], (uint32_t)i);
}

__global__ void __launch_bounds__(kBlock) k_splat_xy(uint32_t *__restrict__ map,
                                                     const uint32_t *__restrict__ pos,
                                                     int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) {
        uint32_t p = pos[i];
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

__global__ void __launch_bounds__(kBlock) k_move(uint32_t *__restrict__ pos, int32_t S,
                                                 int32_t W, int32_t H, uint64_t move_seed,
                                                 uint64_t t, int32_t lo, uint32_t span)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    uint64_t n = ((t - 1) * (uint64_t)S + (uint64_t)i) * 2u;
    uint32_t p = pos[i];
    int32_t x = (int32_t)(p & 0xFFFFu) + draw(move_seed, n + 0, lo, span);
    int32_t y = (int32_t)(p >> 16) + draw(move_seed, n + 1, lo, span);
    x = min(max(x, 0), W - 1);
    y = min(max(y, 0), H - 1);
    pos[i] = ((uint32_t)y << 16) | (uint32_t)x;
}

__global__ void __launch_bounds__(kBlock) k_index_min(uint32_t *__restrict__ idx,
                                                      const uint32_t *__restrict__ pos,
                                                      int32_t S, int32_t W)
{
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) atomicMin(&idx[pixel_of(pos[i], W)], (uint32_t)i);
}

__global__ void __launch_bounds__(kBlock) k_relabel(uint32_t *__restrict__ map,
                                                    const uint32_t *__restrict__ idx,
                                                    const uint32_t *__restrict__ pos_new,
                                                    int32_t S, int32_t W, int32_t H)
{
    int64_t n = (int64_t)W * H;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        uint32_t l = map[p];
        if (l == kEmpty) continue;
        uint32_t lx = l & 0xFFFFu, ly = l >> 16;
        uint32_t i = (lx < (uint32_t)W && ly < (uint32_t)H) ? idx[(int64_t)ly * W + lx] : kEmpty;
        map[p] = i < (uint32_t)S ? pos_new[i] : kEmpty;
    }
}

// First version of the pass: one thread per pixel, loads through the caches.
template <int LABEL, int METRIC>
__global__ void __launch_bounds__(kBlock) k_flood_simple(const uint32_t *__restrict__ src,
                                                         uint32_t *__restrict__ dst,
                                                         const uint32_t *__restrict__ pos,
                                                         int32_t W, int32_t H, int32_t k,
                                                         int32_t vn)
{
    int32_t x = blockIdx.x * 64 + (threadIdx.x & 63);
    int32_t y = blockIdx.y * (kBlock / 64) + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    uint64_t best = ~0ull;
    for (int32_t oy = -1; oy <= 1; ++oy) {
        int32_t cy = y + oy * k;
        if (cy < 0 || cy >= H) continue;
        for (int32_t ox = -1; ox <= 1; ++ox) {
            if (vn && ox != 0 && oy != 0) continue;
            int32_t cx = x + ox * k;
            if (cx < 0 || cx >= W) continue;
            uint32_t l = src[(int64_t)cy * W + cx];
            if (l == kEmpty) continue;
            uint32_t p = LABEL == kLabelId ? pos[l] : l;
            int32_t dx = x - (int32_t)(p & 0xFFFFu);
            int32_t dy = y - (int32_t)(p >> 16);
            uint32_t d = METRIC == kEuclid ? (uint32_t)(dx * dx + dy * dy)
                                           : (uint32_t)(abs(dx) + abs(dy));
            uint64_t key = ((uint64_t)d << 32) | l;
            best = key < best ? key : best;
        }
    }
    dst[(int64_t)y * W + x] = (uint32_t)best;
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

hipError_t launch_splat_reset(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_reset, grid1d(S), dim3(kBlock), 0, s, map, pos, S, W);
    return hipGetLastError();
}

hipError_t launch_splat_min(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_min, grid1d(S), dim3(kBlock), 0, s, map, pos, S, W);
    return hipGetLastError();
}

hipError_t launch_splat_xy(uint32_t *map, const uint32_t *pos, int32_t S, int32_t W,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_xy, grid1d(S), dim3(kBlock), 0, s, map, pos, S, W);
    return hipGetLastError();
}

hipError_t launch_move(uint32_t *pos, int32_t S, int32_t W, int32_t H, uint64_t move_seed,
                       int64_t t, int32_t lo, int32_t hi, hipStream_t s)
{
    hipLaunchKernelGGL(k_move, grid1d(S), dim3(kBlock), 0, s, pos, S, W, H, move_seed,
                       (uint64_t)t, lo, (uint32_t)(hi - lo + 1));
    return hipGetLastError();
}

hipError_t launch_index_old(uint32_t *idx, const uint32_t *pos_old, int32_t S, int32_t W,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_splat_reset, grid1d(S), dim3(kBlock), 0, s, idx, pos_old, S, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_index_min, grid1d(S), dim3(kBlock), 0, s, idx, pos_old, S, W);
    return hipGetLastError();
}

hipError_t launch_relabel(uint32_t *map, const uint32_t *idx, const uint32_t *pos_new,
                          int32_t S, int32_t W, int32_t H, hipStream_t s)
{
    hipLaunchKernelGGL(k_relabel, grid1d((int64_t)W * H, 8192), dim3(kBlock), 0, s, map, idx,
                       pos_new, S, W, H);
    return hipGetLastError();
}

hipError_t launch_flood(const uint32_t *src, uint32_t *dst, const uint32_t *pos, int32_t W,
                        int32_t H, int32_t k, int32_t vn, int32_t label, int32_t metric,
                        hipStream_t s)
{
    dim3 grid((unsigned)((W + 63) / 64), (unsigned)((H + kBlock / 64 - 1) / (kBlock / 64)));
    if (label == kLabelId && metric == kEuclid)
        hipLaunchKernelGGL((k_flood_simple<kLabelId, kEuclid>), grid, dim3(kBlock), 0, s, src,
                           dst, pos, W, H, k, vn);
    else if (label == kLabelId)
        hipLaunchKernelGGL((k_flood_simple<kLabelId, kManhattan>), grid, dim3(kBlock), 0, s,
                           src, dst, pos, W, H, k, vn);
    else if (metric == kEuclid)
        hipLaunchKernelGGL((k_flood_simple<kLabelXy, kEuclid>), grid, dim3(kBlock), 0, s, src,
                           dst, pos, W, H, k, vn);
    else
        hipLaunchKernelGGL((k_flood_simple<kLabelXy, kManhattan>), grid, dim3(kBlock), 0, s,
                           src, dst, pos, W, H, k, vn);
    return hipGetLastError();
}

}  // namespace vd
