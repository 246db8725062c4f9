// The first flood pass of an XY-label dJFA step with the relabel folded in
// (Sec. V, Alg. 1: the previous diagram, whose labels are the old seed
// positions, seen with the moved positions).  The pass is the four-column
// shared-row tile of vd_quad.h; each label it loads is translated through
// the old-position index (RelabelLookup) before the candidates are
// compared, so the map needs no separate relabel pass over it.
#include <type_traits>

#include "vd_quad.h"

namespace vd {

namespace {

template <int METRIC, int VN, int NS, int ST, bool WIDE, int DL>
__global__ void __launch_bounds__(kBlock) k_flood_quad_relabel(const uint32_t *__restrict__ src,
                                                               uint32_t *__restrict__ dst,
                                                               const uint32_t *__restrict__ idx,
                                                               int32_t W, int32_t H, int32_t k,
                                                               FloodGrid g)
{
    using Q = typename std::conditional<WIDE, QuadRowWide, QuadRow>::type;
    __shared__ Q lds[2];
    const RelabelLookup lk{
        __builtin_amdgcn_make_buffer_rsrc((void *)idx, 0, 4 * W * H, kRsrcWord3), W};
    // Tiles are taken segment-major: the index lines of the old positions in
    // one band of rows -- each cell's rows lie on different chains -- are
    // fetched into one L2 and reused there.
    flood_quad_id_tile<METRIC, VN, 0, NS, ST, Q, RelabelLookup, DL>(
        src, dst, lk, W, H, k, g, seg_major(xcd_logical(blockIdx.x, g.nblocks), g), lds);
}

}  // namespace

bool relabel_fold_ok(int32_t W, int32_t k)
{
    return W % kQuad == 0 && k >= kQuad && k <= kMaxQuadLdsStep && k % kQuad == 0;
}

hipError_t launch_flood_relabel(const uint32_t *src, uint32_t *dst, const uint32_t *idx,
                                int32_t W, int32_t H, int32_t k, int32_t vn, int32_t metric,
                                int32_t variant, int32_t seg_rows, hipStream_t s)
{
    if (!relabel_fold_ok(W, k) || variant < 0 || variant >= kFloodVariants)
        return hipErrorInvalidValue;
    const FloodGrid g = flood_grid_quad(W, H, k, seg_rows);
    if (g.nblocks == 0) return hipErrorInvalidValue;
    const dim3 grid(g.nblocks), block(kBlock);
    // rows in flight: 3 (labels one row ahead of their gathers, gathers one
    // row ahead of use), 4 with the gathers one row ahead (base variants 2)
    // or two rows ahead (5, for their latency)
    const int base = variant % (kFloodVariants / 2);
    const int rows = base == 2 ? 1 : (base == 5 ? 2 : 0);
    const bool nt = variant >= kFloodVariants / 2;    // non-temporal stores
    const bool wide = k > kMaxLdsStep;
#define VD_RL(MT, V, NS, ST, DL)                                                             \
    do {                                                                                     \
        if (wide)                                                                            \
            hipLaunchKernelGGL((k_flood_quad_relabel<MT, V, NS, ST, true, DL>), grid, block, 0, \
                               s, src, dst, idx, W, H, k, g);                                \
        else                                                                                 \
            hipLaunchKernelGGL((k_flood_quad_relabel<MT, V, NS, ST, false, DL>), grid, block, \
                               0, s, src, dst, idx, W, H, k, g);                             \
    } while (0)
#define VD_RL_ST(MT, V, NS, DL)                                                              \
    do {                                                                                     \
        if (nt) VD_RL(MT, V, NS, kStoreNT, DL); else VD_RL(MT, V, NS, 0, DL);                \
    } while (0)
#define VD_RL_NS(MT, V)                                                                      \
    do {                                                                                     \
        if (rows == 1) VD_RL_ST(MT, V, 4, 2);                                                \
        else if (rows == 2) VD_RL_ST(MT, V, 4, 1);                                           \
        else VD_RL_ST(MT, V, 3, 1);                                                          \
    } while (0)
    if (metric == kEuclid) {
        if (vn) VD_RL_NS(kEuclid, 1); else VD_RL_NS(kEuclid, 0);
    } else {
        if (vn) VD_RL_NS(kManhattan, 1); else VD_RL_NS(kManhattan, 0);
    }
#undef VD_RL_NS
#undef VD_RL_ST
#undef VD_RL
    return hipGetLastError();
}

}  // namespace vd
