// Batched time steps over many simulations of different sizes.
//
// One batch step advances every member simulation by one time step (move,
// then a JFA or a dJFA step, Sec. III / Sec. V) with a fixed number of
// launches, whatever the number of simulations:
//   begin (clear work counters), move, then the step's start as a lone
//   simulation makes it -- JFA: fill (ID labels: all ones) and splat; dJFA:
//   the compare-and-swap splat into the previous diagram, or for XY labels
//   the old-position index, the relabel and the splat -- then one
//   persistent flood launch per pass level, then end (advance t, flip the
//   current-map index where the pass count is odd; XY labels: the diagram
//   now refers to the current positions).  The per-seed arithmetic is the
//   single-simulation kernels' (vd_device.h), the relabel theirs too.
// Level i runs pass i of every simulation that has one; the tiles of all of
// them form one work list.  A fixed grid of workgroups (as many as fit on
// the GPU at once) takes tiles from it until it is empty: each XCD first
// drains its own eighth of the list (tiles of a simulation are contiguous,
// so neighbouring tiles meet in that XCD's L2), then helps the others.
//
// The current-map index and the time step of each simulation live in device
// memory and are read by the kernels, so a step captured once in a hipGraph
// replays correctly for every later step (no node holds a step-dependent
// argument).  The host mirrors both values in each vd_sim, which keeps
// vd_read_map, vd_read_seeds and vd_get_info valid between batch steps.
#include <string.h>

#include <algorithm>
#include <functional>
#include <limits>
#include <map>
#include <new>
#include <vector>

#include "vd_multi.h"
#include "vd_sim.h"

namespace vd {

namespace {

struct BatchSim {        // device copy of one member simulation
    uint32_t *map[2];
    uint32_t *table;
    uint32_t *pos_map;   // XY labels: the positions the diagram refers to
    uint32_t *idx;       // XY labels: the old-position index
    int32_t W, H, S;
    int32_t lo;          // move range [lo, lo + span)
    uint32_t span;
    int32_t label;
    uint64_t move_seed;
};

struct DevState {        // per-simulation state the kernels read and update
    int32_t cur;         // map[cur] holds the current diagram
    int32_t pad;
    uint64_t t;          // time step
};

struct LevelSim {        // one simulation's pass at one level
    int32_t k;           // 0: no pass at this level
    int32_t vn;
    FloodGrid g;
    uint32_t first;      // index of its first item in the level's work list
    uint32_t per;        // tiles per item
    int32_t quad;        // four-column tiles (item_grid)
    int32_t pad;
};

struct LevelInfo {
    uint32_t total;      // tiles at this level
    uint32_t chunk[9];   // XCD c drains tiles [chunk[c], chunk[c + 1]) first
};

constexpr int kMaxLevels = 24;   // > ceil(log2 16368) + 2 extra passes
// Solo members' passes run on kSoloLanes streams, by size (lane_of).
constexpr int kSoloLanes = 4;
constexpr int64_t kLaneBigPixels = 4096 * 4096;

// A wave-uniform 32-bit value or pointer, stated as such to the compiler.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
}
template <class T>
__device__ __forceinline__ T *uni_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(v >> 32));
    return (T *)(lo | (hi << 32));
}

__global__ void __launch_bounds__(kBlock) k_batch_begin(uint32_t *__restrict__ ctr, int32_t n)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0u;
}

// Per-member kernels: blockIdx.y is the member, blockIdx.x strides over
// its seeds (or its relabel blocks).
__global__ void __launch_bounds__(kBlock) k_batch_move(const BatchSim *__restrict__ sims,
                                                       const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    const uint64_t t = st[blockIdx.y].t + 1;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sm.S;
         i += gridDim.x * blockDim.x)
        move_one(sm.table, i, sm.S, sm.W, sm.H, sm.move_seed, t, sm.lo, sm.span);
}

// A JFA step's map: unclaimed everywhere (ID labels: all ones, which the
// atomic minimum of the splat needs no reset for).
__global__ void __launch_bounds__(kBlock) k_batch_fill(const BatchSim *__restrict__ sims,
                                                       const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    uint32_t *map = sm.map[st[blockIdx.y].cur];
    const uint32_t v = sm.label == kLabelId ? 0xFFFFFFFFu : kEmpty;
    const int64_t n = (int64_t)sm.W * sm.H;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        map[i] = v;
}

// Seed pixels of a JFA step (on the filled map).
__global__ void __launch_bounds__(kBlock) k_batch_splat_jfa(const BatchSim *__restrict__ sims,
                                                            const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    uint32_t *map = sm.map[st[blockIdx.y].cur];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sm.S;
         i += gridDim.x * blockDim.x) {
        if (sm.label == kLabelId)
            splat_min_seed(map, sm.table, i, sm.W);
        else
            splat_xy_seed(map, sm.table, i, sm.W, 0u);
    }
}

// A dJFA step's splat: ID labels into the previous diagram; XY labels the
// first half of the old-position index (every seed claims its old pixel).
__global__ void __launch_bounds__(kBlock) k_batch_splat_djfa(const BatchSim *__restrict__ sims,
                                                             const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    uint32_t *map = sm.map[st[blockIdx.y].cur];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sm.S;
         i += gridDim.x * blockDim.x) {
        if (sm.label == kLabelId)
            splat_swap_seed(map, sm.table, sm.S, sm.W, i, nullptr, 0u);
        else
            splat_swap_seed(sm.idx, sm.pos_map, sm.S, sm.W, i, nullptr, 0u);
    }
}

// XY labels, dJFA: the index resolved to the moved positions ...
__global__ void __launch_bounds__(kBlock) k_batch_index(const BatchSim *__restrict__ sims)
{
    const BatchSim sm = sims[blockIdx.y];
    if (sm.label != kLabelXy) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sm.S;
         i += gridDim.x * blockDim.x)
        index_resolve_seed(sm.idx, sm.pos_map, sm.table, i, sm.W);
}

// ... every label relabelled through it (widths divisible by 4 with the
// pipelined blocks, others one pixel per lane) ...
__global__ void __launch_bounds__(kBlock) k_batch_relabel(const BatchSim *__restrict__ sims,
                                                          const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    if (sm.label != kLabelXy) return;
    uint32_t *map = sm.map[st[blockIdx.y].cur];
    if (sm.W % kQuad == 0) {
        const int64_t nb = relabel_blocks(sm.W, sm.H);
        for (int64_t b = blockIdx.x; b < nb; b += gridDim.x)
            relabel_block(map, sm.idx, sm.W, sm.H, kRelabelBlockRows, (uint32_t)b);
    } else {
        const int64_t n = (int64_t)sm.W * sm.H;
        for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
             p += (int64_t)gridDim.x * blockDim.x)
            map[p] = relabel_one(map[p], sm.idx, sm.W, sm.H);
    }
}

// ... and the seed pixels claimed.
__global__ void __launch_bounds__(kBlock) k_batch_splat_xy(const BatchSim *__restrict__ sims,
                                                           const DevState *__restrict__ st)
{
    const BatchSim sm = sims[blockIdx.y];
    if (sm.label != kLabelXy) return;
    uint32_t *map = sm.map[st[blockIdx.y].cur];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < sm.S;
         i += gridDim.x * blockDim.x)
        splat_xy_seed(map, sm.table, i, sm.W, 0u);
}

__global__ void __launch_bounds__(kBlock) k_batch_end(DevState *__restrict__ st,
                                                      const int32_t *__restrict__ npasses,
                                                      int32_t n, int32_t moved)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        st[i].cur ^= npasses[i] & 1;
        st[i].t += (uint64_t)moved;
    }
}

// XY labels: the diagram now refers to the current positions.
__global__ void __launch_bounds__(kBlock) k_batch_posmap(const BatchSim *__restrict__ sims)
{
    const BatchSim sm = sims[blockIdx.y];
    if (sm.label != kLabelXy) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= sm.S;
         i += gridDim.x * blockDim.x)
        sm.pos_map[i] = sm.table[i];
}

// Persistent flood pass of one level over every member simulation.  Each
// iteration takes one work item -- one or more adjacent tiles of one chain
// segment of one simulation -- and runs it with the tile functions a lone
// simulation's kernels use (member_tiles).
template <int METRIC>
__global__ void __launch_bounds__(kBlock) k_batch_flood(const BatchSim *__restrict__ sims,
                                                        const DevState *__restrict__ st,
                                                        const LevelSim *__restrict__ ls,
                                                        const LevelInfo *__restrict__ info,
                                                        int32_t n, int32_t level,
                                                        uint32_t *__restrict__ ctr)
{
    __shared__ __align__(16) uint8_t lds[kMultiLds];
    __shared__ uint32_t s_item;
    uint32_t probe = 0;   // chunks already found empty
    for (;;) {
        const uint32_t item = claim_item(info->chunk, ctr, probe, &s_item);
        if (item == 0xFFFFFFFFu) return;
        // the last simulation whose first tile is <= item owns it (a
        // simulation without tiles shares its first with the next one).
        // Every value read from the tables below is the same for the whole
        // workgroup; readfirstlane states it, so addresses and descriptors
        // stay in scalar registers.
        int32_t a = 0, b = n;
        while (b - a > 1) {
            const int32_t m = (a + b) >> 1;
            if (uni(ls[m].first) <= item) a = m; else b = m;
        }
        const LevelSim &lv = ls[a];
        const BatchSim &sm = sims[a];
        MemberPass mp;
        mp.k = uni(lv.k);
        mp.vn = uni(lv.vn);
        mp.quad = uni(lv.quad);
        mp.g.ncol = uni(lv.g.ncol);
        mp.g.nseg = uni(lv.g.nseg);
        mp.g.L = uni(lv.g.L);
        mp.g.nblocks = uni(lv.g.nblocks);
        mp.W = uni(sm.W);
        mp.H = uni(sm.H);
        mp.S = uni(sm.S);
        mp.label = uni(sm.label);
        const int32_t c = uni(st[a].cur) ^ (level & 1);
        uint32_t *m0 = uni_ptr(sm.map[0]), *m1 = uni_ptr(sm.map[1]);
        mp.src = c ? m1 : m0;
        mp.dst = c ? m0 : m1;
        mp.table = uni_ptr(sm.table);
        const uint32_t per = uni(lv.per);
        const uint32_t t0 = (item - uni(lv.first)) * per;
        const uint32_t t1 = min(t0 + per, mp.g.nblocks);
        member_tiles<METRIC>(mp, t0, t1, lds);
    }
}

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

struct Layout {
    size_t sims, state, info[2], ls[2], npasses[2], ctr, total;
};

Layout layout(int32_t n)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align_up(bytes);
        return at;
    };
    L.sims = take(sizeof(BatchSim) * (size_t)n);
    L.state = take(sizeof(DevState) * (size_t)n);
    for (int m = 0; m < 2; ++m) {
        L.info[m] = take(sizeof(LevelInfo) * kMaxLevels);
        L.ls[m] = take(sizeof(LevelSim) * (size_t)kMaxLevels * (size_t)n);
        L.npasses[m] = take(sizeof(int32_t) * (size_t)n);
    }
    L.ctr = take(sizeof(uint32_t) * 8 * kMaxLevels);
    L.total = off + 256;   // alignment slack of the caller's pointer
    return L;
}

}  // namespace

}  // namespace vd

using vd::fail;

struct vd_batch {
    std::vector<vd_sim *> sims;
    hipStream_t stream = nullptr;
    uint8_t *base = nullptr;      // aligned start of the device workspace
    vd::Layout lay{};
    int32_t metric = 0;
    bool any_xy = false;          // a member has XY labels (their relabel and table copy run)
    int32_t levels[2] = {0, 0};   // pass levels of a JFA / dJFA step
    std::vector<int64_t> level_pixels[2];    // pixel-updates per level (timing)
    int32_t grid[2] = {0, 0};     // persistent flood workgroups per mode
    int32_t fit = 1;              // flood workgroups that fit on one CU
    int32_t cus = 1;
    // Members of at least solo_px[mode] pixels run that step kind's passes
    // with their own launches (their tuned kernels, their maps kept in the
    // Infinity Cache across passes) instead of joining the persistent
    // levels; the batch's move, fill, splat and end kernels cover everyone.
    int64_t solo_px[2] = {std::numeric_limits<int64_t>::max(),
                          std::numeric_limits<int64_t>::max()};
    std::vector<char> solo[2];
    int64_t solo_pixels[2] = {0, 0};   // pixel-updates of the solo passes of a step
    int32_t solo_passes[2] = {0, 0};
    bool use_graph = false;
    // Captured steps, keyed by (mode, moved, current map of each solo
    // member): solo launches name their maps directly, so a step is
    // captured once per parity configuration it meets (at most two in a
    // loop of one step kind).
    std::map<std::vector<char>, hipGraphExec_t> graphs;
    hipStream_t capture = nullptr;   // private stream to capture on (the caller's may be
                                     // the null stream, which cannot be captured)
    // Solo passes are spread over the step's stream and kSoloLanes - 1 more
    // (forked and joined by events; see enqueue_solo).
    hipStream_t lane[vd::kSoloLanes - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[vd::kSoloLanes - 1] = {};
    bool timing = false;
    std::vector<vd::EventPair> pool;
    size_t used = 0;
    vd_timing acc{};
    bool broken = false;
};

namespace {

#define VD_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(VD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

template <class T>
T *at(vd_batch *b, size_t off)
{
    return (T *)(b->base + off);
}

int batch_record(vd_batch *b, int kind, bool begin, size_t *slot)
{
    if (!b->timing) return VD_OK;
    if (begin) {
        if (b->used == b->pool.size()) {
            vd::EventPair p;
            VD_HIP(hipEventCreate(&p.a));
            VD_HIP(hipEventCreate(&p.b));
            b->pool.push_back(p);
        }
        *slot = b->used++;
        b->pool[*slot].kind = kind;
        VD_HIP(hipEventRecord(b->pool[*slot].a, b->stream));
    } else {
        VD_HIP(hipEventRecord(b->pool[*slot].b, b->stream));
    }
    return VD_OK;
}

int batch_harvest(vd_batch *b)
{
    if (b->used == 0) return VD_OK;
    VD_HIP(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->used; ++i) {
        float ms = 0.f;
        VD_HIP(hipEventElapsedTime(&ms, b->pool[i].a, b->pool[i].b));
        int kind = b->pool[i].kind;
        if (kind >= 2 + 2 * vd::kMaxLevels) {   // solo passes of a step: 2 + 2 kMaxLevels + mode
            const int mode = kind - 2 - 2 * vd::kMaxLevels;
            b->acc.flood_launches += b->solo_passes[mode];
            b->acc.flood_ms += ms;
            b->acc.flood_pixels += b->solo_pixels[mode];
        } else if (kind >= 2) {   // flood level: kind = 2 + mode * kMaxLevels + level
            int mode = (kind - 2) / vd::kMaxLevels, level = (kind - 2) % vd::kMaxLevels;
            b->acc.flood_launches += 1;
            b->acc.flood_ms += ms;
            b->acc.flood_pixels += b->level_pixels[mode][level];
        } else {
            b->acc.step_count += 1;
            b->acc.step_ms += ms;
        }
    }
    b->used = 0;
    return VD_OK;
}

// Flood launch of level `lvl` of `mode` using the level parity of
// `parity_level`: equal to lvl in a step; 0 while tuning, so the launch
// reads the current diagrams and writes the idle buffers.
hipError_t launch_level(vd_batch *b, int mode, int32_t lvl, int32_t parity_level, int32_t grid,
                        hipStream_t stream)
{
    const int32_t n = (int32_t)b->sims.size();
    const vd::BatchSim *sims = at<vd::BatchSim>(b, b->lay.sims);
    const vd::DevState *st = at<vd::DevState>(b, b->lay.state);
    const vd::LevelSim *ls = at<vd::LevelSim>(b, b->lay.ls[mode]) + (size_t)lvl * n;
    const vd::LevelInfo *info = at<vd::LevelInfo>(b, b->lay.info[mode]) + lvl;
    uint32_t *ctr = at<uint32_t>(b, b->lay.ctr) + 8 * lvl;
    if (b->metric == VD_EUCLID)
        hipLaunchKernelGGL(vd::k_batch_flood<vd::kEuclid>, dim3((unsigned)grid),
                           dim3(vd::kBlock), 0, stream, sims, st, ls, info, n, parity_level, ctr);
    else
        hipLaunchKernelGGL(vd::k_batch_flood<vd::kManhattan>, dim3((unsigned)grid),
                           dim3(vd::kBlock), 0, stream, sims, st, ls, info, n, parity_level, ctr);
    return hipGetLastError();
}

// The passes of the solo members, each with its own kernels, from the map
// the host mirror names current (the batch keeps the mirror in step with
// the device state).  `tuning`: every pass reads the current map and writes
// the idle one, so nothing changes.
// A solo member's passes, as its own step would run them: its kernel
// variants, and its last passes fused where the member fuses them (each
// launch flips its current map; step_launches counts them).
// Map flips of member i in a step of kind `mode`: one per pass level when
// it runs fused with the others, one per launch of its own when solo.
int32_t flips(const vd_batch *b, int mode, int32_t i)
{
    const vd_sim *s = b->sims[(size_t)i];
    const bool dyn = mode == VD_STEP_DJFA;
    if (b->solo[mode][(size_t)i]) return vd::step_launches(s, dyn);
    return (int32_t)(dyn ? s->djfa_passes : s->jfa_passes).size();
}

// The stream of a solo member by its size: members of kLaneBigPixels and
// up on lane 0, those of a quarter of that and up on lane 1, one of each at
// a time, so that their maps stay in the Infinity Cache beside each other
// (128 + 32 MiB at 4096^2 and 2048^2); smaller ones alternate between
// lanes 2 and 3.
int lane_of(const vd_sim *s, int32_t *nth)
{
    const int64_t px = (int64_t)s->cfg.width * s->cfg.height;
    if (px >= vd::kLaneBigPixels) return 0;
    if (px >= vd::kLaneBigPixels / 4) return 1;
    return 2 + (*nth)++ % 2;
}

// Streams for the solo passes of a `mode` step: `stream` and the batch's
// other lanes (created on first use), which wait for what `stream` has
// queued so far; *used receives the number of streams (1 when a single
// member runs solo).
int fork_lanes(vd_batch *b, int mode, hipStream_t stream, int *used)
{
    int32_t alone = 0;
    for (size_t i = 0; i < b->sims.size(); ++i) alone += b->solo[mode][i] ? 1 : 0;
    const int n = alone > 1 ? vd::kSoloLanes : 1;
    *used = n;
    if (n == 1) return VD_OK;
    if (!b->fork) {
        VD_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        for (int l = 0; l < vd::kSoloLanes - 1; ++l) {
            VD_HIP(hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking));
            VD_HIP(hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming));
        }
    }
    VD_HIP(hipEventRecord(b->fork, stream));
    for (int l = 1; l < n; ++l) VD_HIP(hipStreamWaitEvent(b->lane[l - 1], b->fork, 0));
    return VD_OK;
}

int join_lanes(vd_batch *b, hipStream_t stream, int used)
{
    for (int l = 1; l < used; ++l) {
        VD_HIP(hipEventRecord(b->join[l - 1], b->lane[l - 1]));
        VD_HIP(hipStreamWaitEvent(stream, b->join[l - 1], 0));
    }
    return VD_OK;
}

// The passes of the solo members, each as its own step would run them, on
// lane_of's stream when `lanes` streams are in use (fork_lanes).
int enqueue_solo(vd_batch *b, int mode, bool tuning, hipStream_t stream, int lanes = 1)
{
    int32_t nth = 0;
    for (size_t i = 0; i < b->sims.size(); ++i) {
        if (!b->solo[mode][i]) continue;
        const vd_sim *s = b->sims[i];
        hipStream_t on = stream;
        if (lanes > 1) {
            const int l = lane_of(s, &nth);
            if (l) on = b->lane[l - 1];
        }
        const vd_config &c = s->cfg;
        const std::vector<vd::Pass> &ps = mode == VD_STEP_DJFA ? s->djfa_passes : s->jfa_passes;
        const int32_t th = s->tail_th[mode == VD_STEP_DJFA ? 1 : 0];
        const size_t m = th ? vd::tail_len(ps) : 0;
        int cur = s->cur;
        size_t j0 = 0;
        if (vd::pair_at_start(s, ps, ps.size() - m)) {   // as the simulation's own step
            VD_HIP(vd::launch_flood_pair(s->map[cur], s->map[cur ^ 1], s->pos, c.num_seeds,
                                         c.width, c.height, ps[0].k, c.label, false, c.metric,
                                         ps[1].variant >= vd::kFloodVariants / 2, on));
            if (!tuning) cur ^= 1;
            j0 = 2;
        }
        for (size_t j = j0; j + m < ps.size(); ++j) {
            const vd::Pass &p = ps[j];
            VD_HIP(vd::launch_flood(s->map[cur], s->map[cur ^ 1], s->pos, c.num_seeds, c.width,
                                    c.height, p.k, p.vn, c.label, c.metric, p.variant,
                                    p.seg_rows, on));
            if (!tuning) cur ^= 1;
        }
        if (m) {
            int32_t ks[vd::kTailMaxPasses], vns[vd::kTailMaxPasses];
            for (size_t j = 0; j < m; ++j) {
                ks[j] = ps[ps.size() - m + j].k;
                vns[j] = ps[ps.size() - m + j].vn;
            }
            const bool nt = ps.back().variant >= vd::kFloodVariants / 2;
            VD_HIP(vd::launch_flood_tail(s->map[cur], s->map[cur ^ 1], s->pos, c.num_seeds,
                                         c.width, c.height, ks, vns, (int32_t)m, c.label,
                                         c.metric, nt, th, on));
            if (!tuning) cur ^= 1;
        }
    }
    return VD_OK;
}

// Enqueues one batch step on `stream` (b->stream, or the capture stream
// while a graph is recorded; then timing is off).
int enqueue_step(vd_batch *b, int mode, int moved, hipStream_t stream)
{
    const int32_t n = (int32_t)b->sims.size();
    int32_t maxS = 1;
    for (vd_sim *s : b->sims) maxS = std::max(maxS, s->cfg.num_seeds);
    const vd::BatchSim *sims = at<vd::BatchSim>(b, b->lay.sims);
    vd::DevState *st = at<vd::DevState>(b, b->lay.state);
    uint32_t *ctr = at<uint32_t>(b, b->lay.ctr);
    const dim3 blk(vd::kBlock);
    const dim3 gseeds((unsigned)std::min<int64_t>((maxS + vd::kBlock - 1) / vd::kBlock, 1024),
                      (unsigned)n);
    hipLaunchKernelGGL(vd::k_batch_begin, dim3(1), blk, 0, stream, ctr,
                       8 * vd::kMaxLevels);
    VD_HIP(hipGetLastError());
    if (moved) {
        hipLaunchKernelGGL(vd::k_batch_move, gseeds, blk, 0, stream, sims,
                           (const vd::DevState *)st);
        VD_HIP(hipGetLastError());
    }
    if (mode == VD_STEP_JFA) {
        hipLaunchKernelGGL(vd::k_batch_fill, dim3(256, (unsigned)n), blk, 0, stream, sims,
                           (const vd::DevState *)st);
        VD_HIP(hipGetLastError());
        hipLaunchKernelGGL(vd::k_batch_splat_jfa, gseeds, blk, 0, stream, sims,
                           (const vd::DevState *)st);
        VD_HIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL(vd::k_batch_splat_djfa, gseeds, blk, 0, stream, sims,
                           (const vd::DevState *)st);
        VD_HIP(hipGetLastError());
        if (b->any_xy) {
            hipLaunchKernelGGL(vd::k_batch_index, gseeds, blk, 0, stream, sims);
            VD_HIP(hipGetLastError());
            hipLaunchKernelGGL(vd::k_batch_relabel, dim3(256, (unsigned)n), blk, 0, stream, sims,
                               (const vd::DevState *)st);
            VD_HIP(hipGetLastError());
            hipLaunchKernelGGL(vd::k_batch_splat_xy, gseeds, blk, 0, stream, sims,
                               (const vd::DevState *)st);
            VD_HIP(hipGetLastError());
        }
    }
    if (b->solo_passes[mode] > 0) {
        // per-launch timing keeps one stream, so each timed range covers
        // one kind of work
        size_t slot = 0;
        int r = batch_record(b, 2 + 2 * vd::kMaxLevels + mode, true, &slot);
        if (r) return r;
        int lanes = 1;
        if (!b->timing) r = fork_lanes(b, mode, stream, &lanes);
        if (r) return r;
        r = enqueue_solo(b, mode, false, stream, lanes);
        if (r == VD_OK) r = join_lanes(b, stream, lanes);
        if (r) return r;
        r = batch_record(b, 0, false, &slot);
        if (r) return r;
    }
    for (int32_t lvl = 0; lvl < b->levels[mode]; ++lvl) {
        size_t slot = 0;
        int r = batch_record(b, 2 + mode * vd::kMaxLevels + lvl, true, &slot);
        if (r) return r;
        VD_HIP(launch_level(b, mode, lvl, lvl, b->grid[mode], stream));
        r = batch_record(b, 0, false, &slot);
        if (r) return r;
    }
    hipLaunchKernelGGL(vd::k_batch_end, dim3(1), blk, 0, stream, st,
                       (const int32_t *)at<int32_t>(b, b->lay.npasses[mode]), n, moved);
    VD_HIP(hipGetLastError());
    if (b->any_xy) {
        hipLaunchKernelGGL(vd::k_batch_posmap, gseeds, blk, 0, stream, sims);
        VD_HIP(hipGetLastError());
    }
    return VD_OK;
}

int query_fit(vd_batch *b)
{
    int dev = 0, cus = 0, fit = 0;
    VD_HIP(hipGetDevice(&dev));
    VD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (b->metric == VD_EUCLID)
        VD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &fit, vd::k_batch_flood<vd::kEuclid>, vd::kBlock, 0));
    else
        VD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &fit, vd::k_batch_flood<vd::kManhattan>, vd::kBlock, 0));
    b->cus = std::max(cus, 1);
    b->fit = std::max(fit, 1);
    return VD_OK;
}

int32_t grid_for(const vd_batch *b, int32_t wg_per_cu)
{
    return b->cus * (wg_per_cu > 0 ? std::min(wg_per_cu, b->fit) : b->fit);
}

void drop_graphs(vd_batch *b)
{
    for (auto &kv : b->graphs)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

// Key of the captured step: mode, moved, and the current map of each solo
// member.
std::vector<char> graph_key(const vd_batch *b, int mode, int moved)
{
    std::vector<char> key = {(char)mode, (char)moved};
    for (size_t i = 0; i < b->sims.size(); ++i)
        if (b->solo[mode][i]) key.push_back((char)b->sims[i]->cur);
    return key;
}

// Builds and uploads the device tables from the members' host state: the
// members, their current map and time step, and per step kind the levels of
// the persistent passes over the members that do not run solo.  Waits for
// the batch's stream (no step may be in flight while the tables change).
int build_tables(vd_batch *b)
{
    const int32_t n = (int32_t)b->sims.size();
    VD_HIP(hipStreamSynchronize(b->stream));
    std::vector<vd::BatchSim> hs((size_t)n);
    std::vector<vd::DevState> hst((size_t)n);
    std::vector<vd::LevelInfo> hinfo[2];
    std::vector<vd::LevelSim> hls[2];
    std::vector<int32_t> hnp[2];
    for (int32_t i = 0; i < n; ++i) {
        const vd_sim *s = b->sims[(size_t)i];
        vd::BatchSim &d = hs[(size_t)i];
        memset(&d, 0, sizeof d);
        d.map[0] = s->map[0];
        d.map[1] = s->map[1];
        d.table = s->pos;
        d.pos_map = s->pos_map;
        d.idx = s->idx;
        d.label = s->cfg.label;
        d.W = s->cfg.width;
        d.H = s->cfg.height;
        d.S = s->cfg.num_seeds;
        d.lo = s->cfg.disp_lo;
        d.span = (uint32_t)(s->cfg.disp_hi - s->cfg.disp_lo + 1);
        d.move_seed = s->move_seed;
        hst[(size_t)i] = vd::DevState{s->cur, 0, (uint64_t)s->t};
    }
    for (int m = 0; m < 2; ++m) {
        b->solo[m].assign((size_t)n, 0);
        b->solo_pixels[m] = 0;
        b->solo_passes[m] = 0;
        int32_t levels = 0;
        for (int32_t i = 0; i < n; ++i) {
            const vd_sim *s = b->sims[(size_t)i];
            const int32_t np = (int32_t)(m ? s->djfa_passes : s->jfa_passes).size();
            if (np > vd::kMaxLevels) return fail(VD_EINVAL, "too many passes per step (%d)", np);
            if ((int64_t)s->cfg.width * s->cfg.height >= b->solo_px[m]) {
                b->solo[m][(size_t)i] = 1;
                b->solo_pixels[m] += (int64_t)s->cfg.width * s->cfg.height * np;
                b->solo_passes[m] += np;
            } else {
                levels = std::max(levels, np);
            }
        }
        b->levels[m] = levels;
        hinfo[m].assign(vd::kMaxLevels, vd::LevelInfo{});
        hls[m].assign((size_t)vd::kMaxLevels * n, vd::LevelSim{});
        hnp[m].resize((size_t)n);
        b->level_pixels[m].assign(vd::kMaxLevels, 0);
        for (int32_t lvl = 0; lvl < levels; ++lvl) {
            uint32_t first = 0;
            for (int32_t i = 0; i < n; ++i) {
                const vd_sim *s = b->sims[(size_t)i];
                const std::vector<vd::Pass> &ps = m ? s->djfa_passes : s->jfa_passes;
                vd::LevelSim &e = hls[m][(size_t)lvl * n + i];
                e.first = first;   // a member without items shares its first with the next
                if (!b->solo[m][(size_t)i] && lvl < (int32_t)ps.size()) {
                    e.k = ps[(size_t)lvl].k;
                    e.vn = ps[(size_t)lvl].vn;
                    const vd::ItemGrid ig = vd::item_grid(s->cfg.width, s->cfg.height, e.k);
                    e.g = ig.g;
                    e.per = ig.per;
                    e.quad = ig.quad;
                    if (ig.items == 0 || (uint64_t)first + ig.items > 0xFFFFFFF0ull)
                        return fail(VD_EINVAL, "level %d of the batch is too large", lvl);
                    first += ig.items;
                    b->level_pixels[m][(size_t)lvl] += (int64_t)s->cfg.width * s->cfg.height;
                }
            }
            vd::LevelInfo &li = hinfo[m][(size_t)lvl];
            li.total = first;
            for (int c = 0; c <= 8; ++c) li.chunk[c] = (uint32_t)((uint64_t)first * c / 8);
        }
        // map flips per step: one per level, or per launch of a solo member
        for (int32_t i = 0; i < n; ++i)
            hnp[m][(size_t)i] = flips(b, m, i);
    }
    const vd::Layout &lay = b->lay;
    hipStream_t stream = b->stream;
    hipError_t e = hipMemcpyAsync(b->base + lay.sims, hs.data(), sizeof(vd::BatchSim) * n,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->base + lay.state, hst.data(), sizeof(vd::DevState) * n,
                           hipMemcpyHostToDevice, stream);
    for (int m = 0; m < 2 && e == hipSuccess; ++m) {
        e = hipMemcpyAsync(b->base + lay.info[m], hinfo[m].data(),
                           sizeof(vd::LevelInfo) * vd::kMaxLevels, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->base + lay.ls[m], hls[m].data(),
                               sizeof(vd::LevelSim) * hls[m].size(), hipMemcpyHostToDevice,
                               stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->base + lay.npasses[m], hnp[m].data(), sizeof(int32_t) * n,
                               hipMemcpyHostToDevice, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);   // the host images are locals
    if (e != hipSuccess)
        return fail(VD_EDEVICE, "uploading the batch tables failed: %s", hipGetErrorString(e));
    return VD_OK;
}

}  // namespace

extern "C" {

size_t vd_batch_footprint_bytes(int32_t n)
{
    if (n < 1 || n > (1 << 15)) return 0;
    return vd::layout(n).total;
}

int vd_batch_create(vd_sim *const *sims, int32_t n, void *dev_workspace, size_t ws_bytes,
                    void *hip_stream, vd_batch **out)
{
    if (!out) return fail(VD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!sims || n < 1 || n > (1 << 15))
        return fail(VD_EINVAL, "need 1 <= n <= 32768 simulations, got %d", n);
    if (!dev_workspace) return fail(VD_EINVAL, "dev_workspace is NULL");
    vd::Layout lay = vd::layout(n);
    if (ws_bytes < lay.total)
        return fail(VD_ENOMEM, "workspace holds %zu bytes, the batch needs %zu", ws_bytes,
                    lay.total);
    hipStream_t stream = (hipStream_t)hip_stream;
    for (int32_t i = 0; i < n; ++i) {
        const vd_sim *s = sims[i];
        if (!s) return fail(VD_EINVAL, "simulation %d is NULL", i);
        if (s->batch) return fail(VD_ESTATE, "simulation %d already belongs to a batch", i);
        if (s->broken) return fail(VD_ESTATE, "simulation %d is unusable", i);
        if (s->cfg.metric != sims[0]->cfg.metric)
            return fail(VD_EINVAL, "all simulations of a batch share one metric");
        if (s->measured)
            return fail(VD_EINVAL, "batches take a fixed d_max (simulation %d measures it)", i);
        if (s->masked)
            return fail(VD_EINVAL, "batches take simulations with every seed present and kept "
                        "(simulation %d has inserted or removed seeds)", i);
        if (s->stream != stream)
            return fail(VD_EINVAL, "simulation %d runs on another stream than the batch", i);
        for (int32_t j = 0; j < i; ++j)
            if (sims[j] == s) return fail(VD_EINVAL, "simulation %d appears twice", i);
    }
    vd_batch *b = new (std::nothrow) vd_batch;
    if (!b) return fail(VD_ENOMEM, "host allocation of the batch failed");
    b->sims.assign(sims, sims + n);
    b->stream = stream;
    b->lay = lay;
    b->metric = sims[0]->cfg.metric;
    for (int32_t i = 0; i < n; ++i) b->any_xy = b->any_xy || sims[i]->cfg.label == VD_LABEL_XY16;
    b->base = (uint8_t *)(((uintptr_t)dev_workspace + 255) / 256 * 256);

    int r = build_tables(b);
    if (r == VD_OK) r = query_fit(b);
    if (r) {
        delete b;
        return r;
    }
    b->grid[0] = b->grid[1] = grid_for(b, 0);
    for (vd_sim *s : b->sims) s->batch = b;
    *out = b;
    return VD_OK;
}

int vd_batch_step(vd_batch *b, int32_t mode, int32_t move)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (b->broken) return fail(VD_ESTATE, "batch unusable after an earlier device error");
    if (mode != VD_STEP_JFA && mode != VD_STEP_DJFA)
        return fail(VD_EINVAL, "mode must be VD_STEP_JFA or VD_STEP_DJFA, got %d", mode);
    const int moved = move ? 1 : 0;
    size_t slot = 0;
    int r = batch_record(b, 1, true, &slot);
    if (r) return r;
    if (b->use_graph) {
        const std::vector<char> key = graph_key(b, mode, moved);
        if (!b->graphs.count(key) && b->graphs.size() >= 16) drop_graphs(b);   // bound the cache
        hipGraphExec_t &g = b->graphs[key];
        if (!g) {
            hipGraph_t graph = nullptr;
            const bool was_timing = b->timing;
            b->timing = false;   // no event nodes inside the graph
            hipError_t e = hipSuccess;
            if (!b->capture) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                b->timing = was_timing;
                return fail(VD_EDEVICE, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
            }
            r = enqueue_step(b, mode, moved, b->capture);
            e = hipStreamEndCapture(b->capture, &graph);
            b->timing = was_timing;
            if (r == VD_OK && e != hipSuccess)
                r = fail(VD_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
            if (r == VD_OK) {
                e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
                if (e != hipSuccess)
                    r = fail(VD_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
            }
            if (graph) (void)hipGraphDestroy(graph);
            if (r) {
                g = nullptr;
                b->broken = true;
                return r;
            }
        }
        hipError_t e = hipGraphLaunch(g, b->stream);
        if (e != hipSuccess) {
            b->broken = true;
            return fail(VD_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(e));
        }
    } else {
        r = enqueue_step(b, mode, moved, b->stream);
        if (r) {
            b->broken = true;
            return r;
        }
    }
    r = batch_record(b, 1, false, &slot);
    if (r) return r;
    for (size_t i = 0; i < b->sims.size(); ++i) {   // host mirror of the device-side state
        vd_sim *s = b->sims[i];
        s->cur ^= (int)(flips(b, mode, (int32_t)i) & 1);
        s->t += moved;
        s->reach = 0;   // the diagram refers to the current positions
    }
    if (b->timing && b->used >= 4096) return batch_harvest(b);
    return VD_OK;
}

int vd_batch_set_graph(vd_batch *b, int enable)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    b->use_graph = enable != 0;
    if (!b->use_graph) drop_graphs(b);
    return VD_OK;
}

int vd_batch_set_shape(vd_batch *b, int32_t wg_per_cu)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (wg_per_cu < 0 || wg_per_cu > 64)
        return fail(VD_EINVAL, "wg_per_cu must be in [0, 64], got %d", wg_per_cu);
    b->grid[0] = b->grid[1] = grid_for(b, wg_per_cu);
    drop_graphs(b);   // the grid is baked into captured launches
    return VD_OK;
}

int vd_batch_autotune(vd_batch *b, int32_t reps)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (b->broken) return fail(VD_ESTATE, "batch unusable after an earlier device error");
    if (reps < 1 || reps > 1000) return fail(VD_EINVAL, "reps must be in [1, 1000], got %d", reps);
    uint32_t *ctr = at<uint32_t>(b, b->lay.ctr);
    // The flood work of one step of `mode` in tuning form: every persistent
    // level and every solo pass reads the current maps and writes the idle
    // ones, so the members' state does not change.
    auto flood_work = [&](int mode, int32_t grid) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int32_t lvl = 0; lvl < b->levels[mode] && e == hipSuccess; ++lvl) {
            hipLaunchKernelGGL(vd::k_batch_begin, dim3(1), dim3(vd::kBlock), 0, b->stream, ctr,
                               8 * vd::kMaxLevels);
            e = hipGetLastError();
            if (e == hipSuccess) e = launch_level(b, mode, lvl, 0, grid, b->stream);
        }
        if (e == hipSuccess && b->solo_passes[mode] > 0) {
            int lanes = 1;
            if (fork_lanes(b, mode, b->stream, &lanes) != VD_OK ||
                enqueue_solo(b, mode, true, b->stream, lanes) != VD_OK ||
                join_lanes(b, b->stream, lanes) != VD_OK)
                e = hipErrorUnknown;
        }
        return e;
    };
    // Times `cands.size()` configurations of one mode; set(c) installs
    // candidate c.  Returns the index of the fastest (-1 on failure).
    auto pick = [&](int mode, size_t ncand, const std::function<int(size_t)> &set,
                    const std::function<int32_t()> &grid) -> long {
        std::vector<hipEvent_t> ev(2 * ncand, nullptr);
        int r = VD_OK;
        for (hipEvent_t &e : ev)
            if (hipEventCreate(&e) != hipSuccess) r = fail(VD_EDEVICE, "hipEventCreate failed");
        float best = 1e30f;
        long win = -1;
        for (size_t c = 0; r == VD_OK && c < ncand; ++c) {
            r = set(c);
            if (r) break;
            hipError_t e = flood_work(mode, grid());   // warm-up
            if (e == hipSuccess) e = hipEventRecord(ev[2 * c], b->stream);
            for (int32_t k = 0; k < reps && e == hipSuccess; ++k) e = flood_work(mode, grid());
            if (e == hipSuccess) e = hipEventRecord(ev[2 * c + 1], b->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]);
            if (e != hipSuccess) {
                r = fail(VD_EDEVICE, "batch autotune failed: %s", hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                win = (long)c;
            }
        }
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        return r == VD_OK ? win : -1;
    };
    // 1. persistent grid per mode (all members in the levels)
    std::vector<int32_t> grids;
    for (int32_t w : {1, 2, 4, 8, 0}) {
        int32_t g = grid_for(b, w);
        if (std::find(grids.begin(), grids.end(), g) == grids.end()) grids.push_back(g);
    }
    const int64_t none = std::numeric_limits<int64_t>::max();
    b->solo_px[0] = b->solo_px[1] = none;
    int r = build_tables(b);
    if (r) return r;
    for (int mode = 0; mode < 2; ++mode) {
        if (b->levels[mode] == 0) continue;
        size_t cur = 0;
        long w = pick(mode, grids.size(), [&](size_t c) { cur = c; return VD_OK; },
                      [&]() { return grids[cur]; });
        if (w < 0) return VD_EDEVICE;
        b->grid[mode] = grids[(size_t)w];
    }
    // 2. which members run solo: none, or every member of at least one of
    //    the members' sizes
    std::vector<int64_t> th = {none};
    for (vd_sim *s : b->sims) {
        const int64_t px = (int64_t)s->cfg.width * s->cfg.height;
        if (std::find(th.begin(), th.end(), px) == th.end()) th.push_back(px);
    }
    for (int mode = 0; mode < 2; ++mode) {
        long w = pick(mode, th.size(),
                      [&](size_t c) {
                          b->solo_px[mode] = th[c];
                          return build_tables(b);
                      },
                      [&]() { return b->grid[mode]; });
        if (w < 0) {
            b->solo_px[mode] = none;
            (void)build_tables(b);
            return VD_EDEVICE;
        }
        b->solo_px[mode] = th[(size_t)w];
    }
    r = build_tables(b);
    drop_graphs(b);
    return r;
}

int vd_batch_set_solo(vd_batch *b, int32_t mode, int64_t min_pixels)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (mode != VD_STEP_JFA && mode != VD_STEP_DJFA)
        return fail(VD_EINVAL, "mode must be VD_STEP_JFA or VD_STEP_DJFA, got %d", mode);
    b->solo_px[mode] = min_pixels <= 0 ? std::numeric_limits<int64_t>::max() : min_pixels;
    drop_graphs(b);
    return build_tables(b);
}

int vd_batch_set_timing(vd_batch *b, int enable)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (b->used) {
        VD_HIP(hipStreamSynchronize(b->stream));
        b->used = 0;
    }
    b->timing = enable != 0;
    memset(&b->acc, 0, sizeof b->acc);
    return VD_OK;
}

int vd_batch_get_timing(vd_batch *b, vd_timing *out)
{
    if (!b || !out) return fail(VD_EINVAL, "NULL argument");
    int r = batch_harvest(b);
    if (r) return r;
    *out = b->acc;
    memset(&b->acc, 0, sizeof b->acc);
    return VD_OK;
}

int vd_batch_info(const vd_batch *b, int32_t *levels_jfa, int32_t *levels_djfa, int32_t *grid)
{
    if (!b) return fail(VD_EINVAL, "batch is NULL");
    if (levels_jfa) *levels_jfa = b->levels[VD_STEP_JFA];
    if (levels_djfa) *levels_djfa = b->levels[VD_STEP_DJFA];
    if (grid) *grid = b->grid[VD_STEP_DJFA];
    return VD_OK;
}

void vd_batch_destroy(vd_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (vd::EventPair &p : b->pool) {
        if (p.a) (void)hipEventDestroy(p.a);
        if (p.b) (void)hipEventDestroy(p.b);
    }
    for (vd_sim *s : b->sims) {
        s->batch = nullptr;
        // the batch built 4-byte indices in idx: its own steps' single-launch
        // index starts from a fill
        s->idx_builds = vd::kIndexEpochs;
        if (s->release) vd_destroy(s);   // destroyed by its owner while in the batch
    }
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int l = 0; l < vd::kSoloLanes - 1; ++l) {
        if (b->lane[l]) (void)hipStreamDestroy(b->lane[l]);
        if (b->join[l]) (void)hipEventDestroy(b->join[l]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

}  // extern "C"
