// Serving loop: time-step requests of many resident simulations.
//
// A request asks for one time step of one simulation (move, then a JFA or a
// dJFA step); requests of one simulation run in submission order.  A
// scheduler thread forms "ticks", enqueued on the server's stream with at
// most two in flight.  Two policies decide how a started request runs.
//
// Whole steps (VD_SERVE_STEPS): the next request of every idle simulation
// runs as its move and step with the simulation's own launches (its tuned
// kernel variants and fused tail), simulation after simulation, and the
// tick's event completes them.  Each step keeps its two maps in the
// Infinity Cache across its passes and uses the simulation's fastest
// kernels.
//
// Batched ticks (VD_SERVE_PASSES, the default; continuous batching): the
// requests that start in a tick run their moves and step starts (fill and
// splat, or for XY dJFA the old-position index, the relabel and the splat)
// as one launch of each kind over all of them; then each simulation's
// passes run with its own launches, spread over four streams joined by
// events, so different requests' passes run side by side.  Simulations of
// kLaneBigPixels and up share the first stream, so that only one at a time
// streams its maps through the Infinity Cache; those below
// vd_server_set_solo's size can instead share one persistent launch per
// pass level.  A tick in which only one request starts has nothing to
// share or overlap: that request runs as a whole step.  The next tick is
// enqueued while the current one runs (two in flight), so newcomers wait at
// most for the tick in progress.
//
// Memory: the caller hands the server one device pool.  The server keeps
// its tick tables in it and places each simulation's workspace (two maps
// and the seed table) with a first-fit allocator; a simulation is admitted
// (made resident, with VD_0 computed) only when its footprint fits, and
// waits in arrival order otherwise.  Removing a simulation frees its memory
// and admits waiting ones.  A resident simulation keeps its positions and
// current diagram on the device between requests: the state dJFA reuses.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "vd_multi.h"
#include "vd_sim.h"

namespace vd {

namespace {

constexpr int kRing = 4;       // tick table slots
constexpr int kMaxInflight = 2;   // ticks enqueued ahead of the GPU: enough to keep it busy,
                                  // few enough that a new request joins within a tick
constexpr int kMaxLevels = 24;    // > ceil(log2 16368) + 2 extra passes
// Batched ticks: simulations of at least kSoloPixels pixels run their passes
// with their own launches (their maps stay in the Infinity Cache across the
// passes, and their tuned kernels run); smaller ones share one persistent
// launch per pass level when at least kFuseMin of them start in the tick.
constexpr int64_t kSoloPixels = 0;   // default of vd_server_set_solo: no pass-level fusion
constexpr int kFuseMin = 2;
// Batched ticks run the passes of their simulations on kLanes streams (the
// server's own and kLanes - 1 more, all of the default priority), so the
// passes of different requests run side by side on the device.
constexpr int kLanes = 4;
constexpr int64_t kLaneBigPixels = 4096 * 4096;   // two maps: 128 MiB

struct TickSim {            // one active simulation's pass in a tick
    const uint32_t *src;
    uint32_t *dst;
    const uint32_t *table;
    int32_t W, H, S, k, vn, label;
    FloodGrid g;
    uint32_t first;         // its first item in the tick's work list
    uint32_t per;           // tiles per item
    int32_t quad;           // four-column tiles (item_grid)
};

struct TickPrep {           // one simulation starting (or ending) a request in a tick
    uint32_t *map;          // its current diagram
    uint32_t *table;
    uint32_t *pos_map;      // XY labels: the positions the diagram refers to
    uint32_t *idx;          // XY labels: the old-position index
    int32_t W, H, S, lo;
    uint32_t span;
    int32_t fill;           // JFA: the step starts from an unclaimed map
    int32_t label;
    int32_t pad;
    uint64_t move_seed;
    uint64_t t;             // the time step being entered (>= 1)
};

struct TickHeader {          // one pass level of a tick
    uint32_t total;         // items in the level's flood launch
    uint32_t chunk[9];      // XCD c drains items [chunk[c], chunk[c + 1]) first
    int32_t nactive;        // simulations with a pass at this level
    int32_t begin;          // their first TickSim in the tick's table
};

// Claim counters of a tick (zero when uploaded).  They live in their own
// 256-byte block: atomics on a line that every workgroup also reads the
// chunk bounds from slowed the flood launch down almost threefold.
struct TickCounters {
    uint32_t ctr[8];
    uint32_t pad[56];
};

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

// Kernels over the simulations starting a request in a tick: blockIdx.y is
// the simulation, blockIdx.x strides over its seeds or pixels.  Each does
// what a lone simulation's move and step start do (vd_device.h): the move;
// for a JFA step the fill (ID labels: all ones) and splat; for a dJFA step
// the compare-and-swap splat into the previous diagram, or for XY labels
// the old-position index, the relabel and the splat.
__global__ void __launch_bounds__(kBlock) k_tick_fill(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    if (!p.fill) return;
    const uint32_t v = p.label == kLabelId ? 0xFFFFFFFFu : kEmpty;
    const int64_t n = (int64_t)p.W * p.H;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p.map[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_tick_move(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.S;
         i += gridDim.x * blockDim.x)
        move_one(p.table, i, p.S, p.W, p.H, p.move_seed, p.t, p.lo, p.span);
}

__global__ void __launch_bounds__(kBlock) k_tick_splat(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.S;
         i += gridDim.x * blockDim.x) {
        if (p.fill) {
            if (p.label == kLabelId)
                splat_min_seed(p.map, p.table, i, p.W);
            else
                splat_xy_seed(p.map, p.table, i, p.W, 0u);
        } else if (p.label == kLabelId) {
            splat_swap_seed(p.map, p.table, p.S, p.W, i, nullptr, 0u);
        } else {   // the first half of the old-position index
            splat_swap_seed(p.idx, p.pos_map, p.S, p.W, i, nullptr, 0u);
        }
    }
}

// XY labels, dJFA: the index resolved, every label relabelled through it,
// the seed pixels claimed.
__global__ void __launch_bounds__(kBlock) k_tick_index(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    if (p.fill || p.label != kLabelXy) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.S;
         i += gridDim.x * blockDim.x)
        index_resolve_seed(p.idx, p.pos_map, p.table, i, p.W);
}

__global__ void __launch_bounds__(kBlock) k_tick_relabel(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    if (p.fill || p.label != kLabelXy) return;
    if (p.W % kQuad == 0) {
        const int64_t nb = relabel_blocks(p.W, p.H);
        for (int64_t b = blockIdx.x; b < nb; b += gridDim.x)
            relabel_block(p.map, p.idx, p.W, p.H, kRelabelBlockRows, (uint32_t)b);
    } else {
        const int64_t n = (int64_t)p.W * p.H;
        for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
             q += (int64_t)gridDim.x * blockDim.x)
            p.map[q] = relabel_one(p.map[q], p.idx, p.W, p.H);
    }
}

__global__ void __launch_bounds__(kBlock) k_tick_splat_xy(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    if (p.fill || p.label != kLabelXy) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < p.S;
         i += gridDim.x * blockDim.x)
        splat_xy_seed(p.map, p.table, i, p.W, 0u);
}

// After the passes of a tick (XY labels): the diagram now refers to the
// current positions.
__global__ void __launch_bounds__(kBlock) k_tick_posmap(const TickPrep *__restrict__ prep)
{
    const TickPrep p = prep[blockIdx.y];
    if (p.label != kLabelXy) return;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= p.S;
         i += gridDim.x * blockDim.x)
        p.pos_map[i] = p.table[i];
}

// The flood pass of every active simulation, each at its own pass: work
// items claimed as in a batch level, run by the tiles a lone simulation's
// kernels use (member_tiles).
template <int METRIC>
__global__ void __launch_bounds__(kBlock) k_tick_flood(const TickHeader *__restrict__ hd,
                                                       const TickSim *__restrict__ sims,
                                                       uint32_t *__restrict__ ctr)
{
    __shared__ __align__(16) uint8_t lds[kMultiLds];
    __shared__ uint32_t s_item;
    const int32_t n = uni(hd->nactive);
    uint32_t probe = 0;
    for (;;) {
        const uint32_t item = claim_item(hd->chunk, ctr, probe, &s_item);
        if (item == 0xFFFFFFFFu) return;
        int32_t a = 0, b = n;
        while (b - a > 1) {
            const int32_t m = (a + b) >> 1;
            if (uni(sims[m].first) <= item) a = m; else b = m;
        }
        const TickSim &ts = sims[a];
        MemberPass mp;
        mp.k = uni(ts.k);
        mp.vn = uni(ts.vn);
        mp.label = uni(ts.label);
        mp.quad = uni(ts.quad);
        mp.g.ncol = uni(ts.g.ncol);
        mp.g.nseg = uni(ts.g.nseg);
        mp.g.L = uni(ts.g.L);
        mp.g.nblocks = uni(ts.g.nblocks);
        mp.W = uni(ts.W);
        mp.H = uni(ts.H);
        mp.S = uni(ts.S);
        mp.src = uni_ptr(ts.src);
        mp.dst = uni_ptr(ts.dst);
        mp.table = uni_ptr(ts.table);
        const uint32_t per = uni(ts.per);
        const uint32_t t0 = (item - uni(ts.first)) * per;
        const uint32_t t1 = min(t0 + per, mp.g.nblocks);
        member_tiles<METRIC>(mp, t0, t1, lds);
    }
}

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

}  // namespace vd

using vd::fail;

namespace {

struct Request {
    int64_t ticket;
    int32_t mode;
    vd::Clock::time_point submitted;
};

struct Served {
    int32_t id = -1;
    vd_config cfg{};
    std::vector<int32_t> xy;      // initial positions, kept until admission
    size_t bytes = 0, off = 0;
    vd_sim *sim = nullptr;        // resident once admitted
    bool removing = false;
    std::deque<Request> fifo;     // waiting requests
    Request req{};                // the request being enqueued
    int32_t inflight = 0;         // enqueued ticks touching it, not yet finished
    int32_t running = 0;          // requests started and not yet completed
};

struct Tick {
    hipEvent_t done = nullptr;
    int slot = 0;
    std::vector<std::pair<int32_t, Request>> completes;   // (sim id, request)
    std::vector<int32_t> members;                         // simulations it touches
    int64_t pixel_updates = 0;
};

struct Pool {                     // first-fit allocator over [0, size)
    size_t size = 0;
    std::map<size_t, size_t> free;   // offset -> length
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free.begin(); it != free.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                size_t rest = it->second - bytes, at = it->first + bytes;
                free.erase(it);
                if (rest) free[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

}  // namespace

struct vd_server {
    int32_t max_sims = 0, metric = 0;
    int32_t policy = VD_SERVE_PASSES;  // how requests started from now on run
    int64_t solo_px = vd::kSoloPixels;  // batched ticks: simulations this large run alone
    hipStream_t stream = nullptr;
    hipStream_t lane[vd::kLanes - 1] = {};     // the other pass lanes of batched ticks
    hipEvent_t prep_done[vd::kRing] = {};      // per ring slot: the tick's step starts are in
    hipEvent_t lane_done[vd::kRing][vd::kLanes - 1] = {};   // and each lane's passes are done
    uint8_t *base = nullptr;      // aligned device pool
    size_t ring_bytes = 0;        // tick tables at the start of the pool
    size_t slot_bytes = 0;
    Pool pool;
    uint8_t *host_ring = nullptr; // pinned staging, kRing slots
    int grid = 0;
    std::mutex mu;
    std::condition_variable cv;   // new work or state change
    std::condition_variable done_cv;
    std::map<int32_t, Served> sims;
    std::deque<int32_t> admit_queue;   // waiting for memory, in arrival order
    std::vector<int32_t> order;   // resident ids in admission order (tick order)
    int32_t next_id = 0;
    int64_t next_ticket = 1;
    std::map<int64_t, double> finished;    // ticket -> latency (ms), until collected
    std::vector<double> latencies;         // since the last stats reset
    int64_t submitted = 0, completed = 0, pixel_updates = 0, ticks = 0;
    vd::Clock::time_point stats_t0 = vd::Clock::now();
    std::deque<Tick> inflight;
    bool stop = false;
    int error = VD_OK;
    char error_msg[256] = "";
    std::thread worker;
};

namespace {

// A tick slot: level headers | level counters | joiner table | the levels'
// simulation tables, packed level after level.
size_t off_counters() { return vd::align_up(sizeof(vd::TickHeader) * vd::kMaxLevels); }
size_t off_prep() { return off_counters() + vd::align_up(sizeof(vd::TickCounters) * vd::kMaxLevels); }
size_t off_sims(int32_t max_sims)
{
    return off_prep() + vd::align_up(sizeof(vd::TickPrep) * (size_t)max_sims);
}
size_t slot_size(int32_t max_sims)
{
    return off_sims(max_sims) +
           vd::align_up(sizeof(vd::TickSim) * (size_t)vd::kMaxLevels * (size_t)max_sims);
}

// Called with mu held.  Admits waiting simulations in arrival order while
// their footprints fit; VD_0 is computed by a full JFA on the stream.
void admit(vd_server *sv)
{
    while (!sv->admit_queue.empty()) {
        Served &s = sv->sims[sv->admit_queue.front()];
        if (s.removing) {
            sv->sims.erase(s.id);
            sv->admit_queue.pop_front();
            continue;
        }
        size_t off = 0;
        if (!sv->pool.alloc(s.bytes, &off)) return;
        vd_sim *sim = nullptr;
        int r = vd_init_sim(&s.cfg, s.xy.data(), sv->base + off, s.bytes, sv->stream, &sim);
        if (r != VD_OK) {
            sv->pool.release(off, s.bytes);
            sv->error = r;
            snprintf(sv->error_msg, sizeof sv->error_msg, "admitting simulation %d: %s", s.id,
                     vd_last_error());
            return;
        }
        s.off = off;
        s.sim = sim;
        s.xy.clear();
        s.xy.shrink_to_fit();
        sv->order.push_back(s.id);
        sv->admit_queue.pop_front();
    }
}

// Completes every finished tick at the front of the queue (mu held).  Only
// the scheduler thread calls it, so only it destroys tick events.
void reap(vd_server *sv, bool wait_one)
{
    while (!sv->inflight.empty()) {
        Tick &t = sv->inflight.front();
        hipError_t q = wait_one ? hipEventSynchronize(t.done) : hipEventQuery(t.done);
        wait_one = false;
        if (q == hipErrorNotReady) return;
        if (q != hipSuccess) {
            sv->error = VD_EDEVICE;
            snprintf(sv->error_msg, sizeof sv->error_msg, "tick failed: %s", hipGetErrorString(q));
            return;
        }
        const vd::Clock::time_point now = vd::Clock::now();
        for (auto &c : t.completes) {
            sv->sims[c.first].running -= 1;
            double ms = vd::ms_between(c.second.submitted, now);
            sv->finished[c.second.ticket] = ms;
            sv->latencies.push_back(ms);
            sv->completed += 1;
        }
        sv->pixel_updates += t.pixel_updates;
        for (int32_t id : t.members) sv->sims[id].inflight -= 1;
        (void)hipEventDestroy(t.done);
        sv->inflight.pop_front();
        sv->done_cv.notify_all();
    }
}

// Whole-step requests (VD_SERVE_STEPS): the next request of each idle
// simulation runs as its move and step with the simulation's own launches
// (tuned kernel variants, fused tail), one simulation after another on the
// stream; the tick's event completes them.  Returns false on a launch
// failure (the error is recorded).
bool enqueue_steps(vd_server *sv, Tick &t, const std::vector<int32_t> &ids)
{
    for (int32_t id : ids) {
        Served &s = sv->sims[id];
        vd_sim *m = s.sim;
        const bool dyn = s.req.mode == VD_STEP_DJFA;
        int r = vd_move_seeds(m);
        if (r == VD_OK) r = dyn ? vd_djfa_step(m) : vd_jfa_step(m);
        if (r != VD_OK) {
            sv->error = VD_EDEVICE;
            snprintf(sv->error_msg, sizeof sv->error_msg, "simulation %d: %s", id,
                     vd_last_error());
            return false;
        }
        t.members.push_back(id);
        s.inflight += 1;
        t.pixel_updates += (int64_t)m->cfg.width * m->cfg.height *
                           (int64_t)(dyn ? m->djfa_passes : m->jfa_passes).size();
        t.completes.emplace_back(id, s.req);
    }
    return true;
}

// Batched requests (VD_SERVE_PASSES): every joining simulation's move and
// step start run in shared launches over all of them (one of each kind);
// then the simulations of at least solo_px pixels run their passes with
// their own launches, spread over the pass lanes so that different
// requests' passes run side by side, and the smaller ones -- when at least
// kFuseMin start in this tick -- share one persistent launch per pass
// level, each at its own step size (otherwise they too run alone).  Every
// request completes with the tick.  Returns false on a failure (recorded).
bool enqueue_batched(vd_server *sv, Tick &t, const std::vector<int32_t> &ids)
{
    const int slot = (int)(sv->ticks % vd::kRing);
    uint8_t *h = sv->host_ring + (size_t)slot * sv->slot_bytes;
    uint8_t *d = sv->base + (size_t)slot * sv->slot_bytes;
    vd::TickHeader *hh = (vd::TickHeader *)h;
    vd::TickPrep *hp = (vd::TickPrep *)(h + off_prep());
    vd::TickSim *hs = (vd::TickSim *)(h + off_sims(sv->max_sims));
    memset(h, 0, off_prep());   // headers and claim counters
    std::vector<vd_sim *> sims;
    int32_t maxS = 1, small = 0;
    bool any_fill = false, any_relabel = false, any_xy = false;
    for (size_t j = 0; j < ids.size(); ++j) {
        Served &s = sv->sims[ids[j]];
        vd_sim *m = s.sim;
        sims.push_back(m);
        m->t += 1;
        m->reach = 0;   // after the tick the diagram refers to the moved positions
        vd::TickPrep &p = hp[j];
        memset(&p, 0, sizeof p);
        p.map = m->map[m->cur];
        p.table = m->pos;
        p.pos_map = m->pos_map;
        p.idx = m->idx;
        // the tick builds a 4-byte index in idx: the simulation's own next
        // single-launch index build starts from a fill
        m->idx_builds = vd::kIndexEpochs;
        p.label = m->cfg.label;
        p.W = m->cfg.width;
        p.H = m->cfg.height;
        p.S = m->cfg.num_seeds;
        p.lo = m->cfg.disp_lo;
        p.span = (uint32_t)(m->cfg.disp_hi - m->cfg.disp_lo + 1);
        p.fill = s.req.mode == VD_STEP_JFA;
        p.move_seed = m->move_seed;
        p.t = (uint64_t)m->t;
        maxS = std::max(maxS, p.S);
        any_fill |= p.fill != 0;
        any_relabel |= p.fill == 0 && p.label == VD_LABEL_XY16;
        any_xy |= p.label == VD_LABEL_XY16;
        if ((int64_t)p.W * p.H < sv->solo_px) ++small;
    }
    const bool fuse = small >= vd::kFuseMin;
    std::vector<char> fused(ids.size(), 0);
    std::vector<const std::vector<vd::Pass> *> plist(ids.size());
    int32_t levels = 0;
    for (size_t j = 0; j < ids.size(); ++j) {
        const vd_sim *m = sims[j];
        plist[j] = sv->sims[ids[j]].req.mode == VD_STEP_DJFA ? &m->djfa_passes : &m->jfa_passes;
        fused[j] = fuse && (int64_t)m->cfg.width * m->cfg.height < sv->solo_px;
        if (fused[j]) levels = std::max(levels, (int32_t)plist[j]->size());
    }
    if (levels > vd::kMaxLevels) {
        sv->error = VD_EINVAL;
        snprintf(sv->error_msg, sizeof sv->error_msg, "a step has %d passes (at most %d)", levels,
                 vd::kMaxLevels);
        return false;
    }
    // The fused simulations' pass levels; the host mirror of each current
    // map flips once per level it takes part in.
    int32_t nsims = 0;
    for (int32_t l = 0; l < levels; ++l) {
        vd::TickHeader &lh = hh[l];
        lh.begin = nsims;
        uint32_t first = 0;
        for (size_t j = 0; j < ids.size(); ++j) {
            if (!fused[j] || l >= (int32_t)plist[j]->size()) continue;
            vd_sim *m = sims[j];
            const vd::Pass &ps = (*plist[j])[(size_t)l];
            vd::TickSim &e = hs[nsims++];
            memset(&e, 0, sizeof e);
            e.src = m->map[m->cur];
            e.dst = m->map[m->cur ^ 1];
            e.table = m->pos;
            e.W = m->cfg.width;
            e.H = m->cfg.height;
            e.S = m->cfg.num_seeds;
            e.k = ps.k;
            e.vn = ps.vn;
            e.label = m->cfg.label;
            const vd::ItemGrid ig = vd::item_grid(e.W, e.H, e.k);
            e.g = ig.g;
            e.per = ig.per;
            e.quad = ig.quad;
            e.first = first;
            first += ig.items;
            m->cur ^= 1;
        }
        lh.total = first;
        lh.nactive = nsims - lh.begin;
        for (int c = 0; c <= 8; ++c) lh.chunk[c] = (uint32_t)((uint64_t)first * c / 8);
    }
    const size_t used = off_sims(sv->max_sims) + sizeof(vd::TickSim) * (size_t)nsims;
    hipError_t e = hipMemcpyAsync(d, h, used, hipMemcpyHostToDevice, sv->stream);
    const vd::TickPrep *dp = (const vd::TickPrep *)(d + off_prep());
    const dim3 blk(vd::kBlock);
    const unsigned nj = (unsigned)ids.size();
    const unsigned gs = (unsigned)std::min<int64_t>((maxS + vd::kBlock - 1) / vd::kBlock, 1024);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(vd::k_tick_move, dim3(gs, nj), blk, 0, sv->stream, dp);
        if (any_fill) hipLaunchKernelGGL(vd::k_tick_fill, dim3(256, nj), blk, 0, sv->stream, dp);
        hipLaunchKernelGGL(vd::k_tick_splat, dim3(gs, nj), blk, 0, sv->stream, dp);
        if (any_relabel) {
            hipLaunchKernelGGL(vd::k_tick_index, dim3(gs, nj), blk, 0, sv->stream, dp);
            hipLaunchKernelGGL(vd::k_tick_relabel, dim3(256, nj), blk, 0, sv->stream, dp);
            hipLaunchKernelGGL(vd::k_tick_splat_xy, dim3(gs, nj), blk, 0, sv->stream, dp);
        }
        e = hipGetLastError();
    }
    // The simulations that run alone go over the lanes: those whose two maps
    // fill a large share of the Infinity Cache (kLaneBigPixels and up) one
    // after another on the first lane, so that each keeps its maps cached
    // across its passes, the others round the remaining lanes beside them.
    // The other lanes start after the step starts and the server's stream
    // waits for them.
    int32_t alone = 0, big = 0;
    for (size_t j = 0; j < ids.size(); ++j) {
        if (fused[j]) continue;
        ++alone;
        big += (int64_t)sims[j]->cfg.width * sims[j]->cfg.height >= vd::kLaneBigPixels ? 1 : 0;
    }
    const int lanes = (int)std::min<int32_t>(vd::kLanes, std::max<int32_t>(alone - std::max(big - 1, 0), 1));
    if (e == hipSuccess && lanes > 1) {
        e = hipEventRecord(sv->prep_done[slot], sv->stream);
        for (int l = 1; l < lanes && e == hipSuccess; ++l)
            e = hipStreamWaitEvent(sv->lane[l - 1], sv->prep_done[slot], 0);
    }
    int32_t nth = 0;
    for (size_t j = 0; j < ids.size() && e == hipSuccess; ++j) {
        if (fused[j]) continue;
        const bool large = (int64_t)sims[j]->cfg.width * sims[j]->cfg.height >= vd::kLaneBigPixels;
        const int l = large || lanes == 1 ? 0 : (big ? 1 + nth++ % (lanes - 1) : nth++ % lanes);
        if (vd::launch_step_passes(sims[j], sv->sims[ids[j]].req.mode == VD_STEP_DJFA,
                                   l ? sv->lane[l - 1] : sv->stream) != VD_OK)
            e = hipErrorLaunchFailure;
    }
    for (int l = 1; l < lanes && e == hipSuccess; ++l) {
        e = hipEventRecord(sv->lane_done[slot][l - 1], sv->lane[l - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(sv->stream, sv->lane_done[slot][l - 1], 0);
    }
    const vd::TickSim *ds = (const vd::TickSim *)(d + off_sims(sv->max_sims));
    uint32_t *dc = (uint32_t *)(d + off_counters());
    for (int32_t l = 0; l < levels && e == hipSuccess; ++l) {
        const vd::TickHeader *dh = (const vd::TickHeader *)d + l;
        const unsigned grid = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((int64_t)hh[l].total, (int64_t)sv->grid));
        uint32_t *ctr = dc + (size_t)l * (sizeof(vd::TickCounters) / sizeof(uint32_t));
        if (sv->metric == VD_EUCLID)
            hipLaunchKernelGGL(vd::k_tick_flood<vd::kEuclid>, dim3(grid), dim3(vd::kBlock), 0,
                               sv->stream, dh, ds + hh[l].begin, ctr);
        else
            hipLaunchKernelGGL(vd::k_tick_flood<vd::kManhattan>, dim3(grid), dim3(vd::kBlock), 0,
                               sv->stream, dh, ds + hh[l].begin, ctr);
        e = hipGetLastError();
    }
    if (e == hipSuccess && any_xy) {
        hipLaunchKernelGGL(vd::k_tick_posmap, dim3(gs, nj), blk, 0, sv->stream, dp);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        sv->error = VD_EDEVICE;
        snprintf(sv->error_msg, sizeof sv->error_msg, "enqueueing a batched tick failed: %s",
                 hipGetErrorString(e));
        return false;
    }
    for (size_t j = 0; j < ids.size(); ++j) {
        Served &s = sv->sims[ids[j]];
        t.members.push_back(ids[j]);
        s.inflight += 1;
        t.pixel_updates += (int64_t)sims[j]->cfg.width * sims[j]->cfg.height *
                           (int64_t)plist[j]->size();
        t.completes.emplace_back(ids[j], s.req);
    }
    return true;
}

// Builds and enqueues one tick (mu held): the next request of every
// resident simulation that has one, run whole or batched by the policy.
// Requests of one simulation stay in order: every tick runs on the
// server's stream.  Returns false if there is no work.
bool tick(vd_server *sv)
{
    std::vector<int32_t> whole, batched;
    for (int32_t id : sv->order) {
        Served &s = sv->sims[id];
        if (!s.fifo.empty() && !s.removing) {
            s.req = s.fifo.front();
            s.fifo.pop_front();
            s.running += 1;
            (sv->policy == VD_SERVE_STEPS ? whole : batched).push_back(id);
        }
    }
    if (whole.empty() && batched.empty()) return false;
    if (batched.size() == 1) {   // nothing to share or overlap: the same result as a whole step
        whole.push_back(batched.front());
        batched.clear();
    }
    while ((int)sv->inflight.size() >= vd::kMaxInflight && !sv->error) reap(sv, true);
    if (sv->error) return false;
    Tick t;
    t.slot = -1;
    if (!enqueue_steps(sv, t, whole)) return false;
    if (!batched.empty()) {
        t.slot = (int)(sv->ticks % vd::kRing);
        if (!enqueue_batched(sv, t, batched)) return false;
    }
    hipError_t e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(t.done, sv->stream);
    if (e != hipSuccess) {
        sv->error = VD_EDEVICE;
        snprintf(sv->error_msg, sizeof sv->error_msg, "enqueueing a tick failed: %s",
                 hipGetErrorString(e));
        return false;
    }
    sv->ticks += 1;
    sv->inflight.push_back(std::move(t));
    return true;
}

void worker_main(vd_server *sv)
{
    std::unique_lock<std::mutex> lock(sv->mu);
    while (!sv->stop) {
        if (sv->error) {
            sv->done_cv.notify_all();
            sv->cv.wait(lock, [&] { return sv->stop; });
            break;
        }
        admit(sv);
        reap(sv, false);
        if (tick(sv)) continue;
        if (!sv->inflight.empty()) {
            // nothing new to start: let the GPU finish the oldest tick (the
            // event stays valid: only this thread destroys tick events)
            lock.unlock();
            hipEvent_t ev = sv->inflight.front().done;
            (void)hipEventSynchronize(ev);
            lock.lock();
            continue;
        }
        sv->cv.wait_for(lock, std::chrono::milliseconds(5));
    }
}

void release_lanes(vd_server *sv)
{
    for (hipStream_t &l : sv->lane)
        if (l) (void)hipStreamDestroy(l), l = nullptr;
    for (int r = 0; r < vd::kRing; ++r) {
        if (sv->prep_done[r]) (void)hipEventDestroy(sv->prep_done[r]);
        for (hipEvent_t &ev : sv->lane_done[r])
            if (ev) (void)hipEventDestroy(ev), ev = nullptr;
        sv->prep_done[r] = nullptr;
    }
}

int server_error(vd_server *sv)
{
    return fail(sv->error, "%s", sv->error_msg);
}

}  // namespace

extern "C" {

size_t vd_server_footprint_bytes(int32_t max_sims)
{
    if (max_sims < 1 || max_sims > (1 << 15)) return 0;
    return (size_t)vd::kRing * slot_size(max_sims) + 256;
}

int vd_server_create(int32_t max_sims, int32_t metric, void *dev_pool, size_t pool_bytes,
                     void *hip_stream, vd_server **out)
{
    if (!out) return fail(VD_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_sims < 1 || max_sims > (1 << 15))
        return fail(VD_EINVAL, "max_sims must be in [1, 32768], got %d", max_sims);
    if (metric != VD_EUCLID && metric != VD_MANHATTAN)
        return fail(VD_EINVAL, "unknown metric %d", metric);
    if (!dev_pool) return fail(VD_EINVAL, "dev_pool is NULL");
    size_t ring = (size_t)vd::kRing * slot_size(max_sims);
    if (pool_bytes < ring + 256)
        return fail(VD_ENOMEM, "pool holds %zu bytes, the server tables need %zu", pool_bytes,
                    ring + 256);
    vd_server *sv = new (std::nothrow) vd_server;
    if (!sv) return fail(VD_ENOMEM, "host allocation of the server failed");
    sv->max_sims = max_sims;
    sv->metric = metric;
    sv->stream = (hipStream_t)hip_stream;
    sv->base = (uint8_t *)(((uintptr_t)dev_pool + 255) / 256 * 256);
    sv->slot_bytes = slot_size(max_sims);
    sv->ring_bytes = ring;
    size_t usable = pool_bytes - 256 - ring;
    sv->pool.size = usable;
    sv->pool.free[ring] = usable;   // offsets are relative to base
    int dev = 0, cus = 0, fit = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = metric == VD_EUCLID
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, vd::k_tick_flood<vd::kEuclid>,
                                                               vd::kBlock, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                      &fit, vd::k_tick_flood<vd::kManhattan>, vd::kBlock, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->host_ring, ring, hipHostMallocDefault);
    for (int l = 0; l + 1 < vd::kLanes && e == hipSuccess; ++l)
        e = hipStreamCreateWithFlags(&sv->lane[l], hipStreamNonBlocking);
    for (int r = 0; r < vd::kRing && e == hipSuccess; ++r) {
        e = hipEventCreateWithFlags(&sv->prep_done[r], hipEventDisableTiming);
        for (int l = 0; l + 1 < vd::kLanes && e == hipSuccess; ++l)
            e = hipEventCreateWithFlags(&sv->lane_done[r][l], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release_lanes(sv);
        if (sv->host_ring) (void)hipHostFree(sv->host_ring);
        delete sv;
        return fail(VD_EDEVICE, "server set-up failed: %s", hipGetErrorString(e));
    }
    sv->grid = std::max(cus, 1) * std::max(fit, 1);
    try {
        sv->worker = std::thread(worker_main, sv);
    } catch (...) {
        release_lanes(sv);
        (void)hipHostFree(sv->host_ring);
        delete sv;
        return fail(VD_ENOMEM, "could not start the scheduler thread");
    }
    *out = sv;
    return VD_OK;
}

int vd_server_add_sim(vd_server *sv, const vd_config *cfg, const int32_t *host_xy,
                      int32_t *sim_id)
{
    if (!sv || !cfg || !sim_id) return fail(VD_EINVAL, "NULL argument");
    if (cfg->metric != sv->metric)
        return fail(VD_EINVAL, "simulation metric %d differs from the server's %d", cfg->metric,
                    sv->metric);
    if (cfg->dmax_override == VD_DMAX_MEASURED)
        return fail(VD_EINVAL, "served simulations take a fixed d_max (the schedule of each "
                               "request is planned ahead)");
    size_t bytes = vd_footprint_bytes(cfg);
    if (bytes == 0) return VD_EINVAL;   // message set by the validation
    std::vector<int32_t> placed;        // positions drawn from sim_seed when none are given
    if (!host_xy) {
        try {
            placed.resize(2 * (size_t)cfg->num_seeds);
        } catch (...) {
            return fail(VD_ENOMEM, "host allocation failed");
        }
        const int r = vd_place_seeds(cfg->width, cfg->height, cfg->num_seeds, cfg->sim_seed,
                                     placed.data());
        if (r) return r;
        host_xy = placed.data();
    }
    for (int64_t i = 0; i < 2 * (int64_t)cfg->num_seeds; i += 2)
        if (host_xy[i] < 0 || host_xy[i] >= cfg->width || host_xy[i + 1] < 0 ||
            host_xy[i + 1] >= cfg->height)
            return fail(VD_EINVAL, "seed %lld is outside the grid", (long long)(i / 2));
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->error) return server_error(sv);
    if ((int32_t)sv->sims.size() >= sv->max_sims)
        return fail(VD_ENOMEM, "the server holds its maximum of %d simulations", sv->max_sims);
    if (bytes > sv->pool.size)
        return fail(VD_ENOMEM, "simulation needs %zu bytes, the whole pool has %zu", bytes,
                    sv->pool.size);
    Served s;
    s.id = sv->next_id++;
    s.cfg = *cfg;
    s.bytes = vd::align_up(bytes);
    try {
        s.xy.assign(host_xy, host_xy + 2 * (size_t)cfg->num_seeds);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation failed");
    }
    sv->sims[s.id] = std::move(s);
    sv->admit_queue.push_back(sv->next_id - 1);
    *sim_id = sv->next_id - 1;
    sv->cv.notify_all();
    return VD_OK;
}

int vd_server_set_solo(vd_server *sv, int64_t min_pixels)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->solo_px = min_pixels <= 0 ? 0 : min_pixels;
    return VD_OK;
}

int vd_server_set_policy(vd_server *sv, int32_t policy)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    if (policy != VD_SERVE_STEPS && policy != VD_SERVE_PASSES)
        return fail(VD_EINVAL, "policy must be VD_SERVE_STEPS or VD_SERVE_PASSES, got %d", policy);
    std::lock_guard<std::mutex> lock(sv->mu);
    sv->policy = policy;
    return VD_OK;
}

int vd_server_submit(vd_server *sv, int32_t sim_id, int32_t mode, int64_t *ticket)
{
    if (!sv || !ticket) return fail(VD_EINVAL, "NULL argument");
    if (mode != VD_STEP_JFA && mode != VD_STEP_DJFA)
        return fail(VD_EINVAL, "mode must be VD_STEP_JFA or VD_STEP_DJFA, got %d", mode);
    std::lock_guard<std::mutex> lock(sv->mu);
    if (sv->error) return server_error(sv);
    auto it = sv->sims.find(sim_id);
    if (it == sv->sims.end() || it->second.removing)
        return fail(VD_EINVAL, "no simulation %d", sim_id);
    Request r{sv->next_ticket++, mode, vd::Clock::now()};
    it->second.fifo.push_back(r);
    sv->submitted += 1;
    *ticket = r.ticket;
    sv->cv.notify_all();
    return VD_OK;
}

int vd_server_wait(vd_server *sv, int64_t ticket, double timeout_ms, double *latency_ms)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lock(sv->mu);
    if (ticket < 1 || ticket >= sv->next_ticket) return fail(VD_EINVAL, "unknown ticket %lld",
                                                             (long long)ticket);
    auto ready = [&] { return sv->error || sv->finished.count(ticket); };
    bool ok = timeout_ms < 0 ? (sv->done_cv.wait(lock, ready), true)
                             : sv->done_cv.wait_for(
                                   lock, std::chrono::duration<double, std::milli>(timeout_ms),
                                   ready);
    if (sv->error) return server_error(sv);
    if (!ok) return fail(VD_EBUSY, "ticket %lld not finished", (long long)ticket);
    if (latency_ms) *latency_ms = sv->finished[ticket];
    sv->finished.erase(ticket);
    return VD_OK;
}

int vd_server_drain(vd_server *sv, double timeout_ms)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lock(sv->mu);
    auto idle = [&] {
        if (sv->error) return true;
        if (!sv->inflight.empty()) return false;
        for (auto &kv : sv->sims)
            if (!kv.second.fifo.empty()) return false;
        return true;
    };
    sv->cv.notify_all();
    bool ok = timeout_ms < 0 ? (sv->done_cv.wait(lock, idle), true)
                             : sv->done_cv.wait_for(
                                   lock, std::chrono::duration<double, std::milli>(timeout_ms),
                                   idle);
    if (sv->error) return server_error(sv);
    return ok ? VD_OK : fail(VD_EBUSY, "requests still pending");
}

int vd_server_remove_sim(vd_server *sv, int32_t sim_id)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lock(sv->mu);
    auto it = sv->sims.find(sim_id);
    if (it == sv->sims.end() || it->second.removing)
        return fail(VD_EINVAL, "no simulation %d", sim_id);
    Served &s = it->second;
    s.removing = true;
    s.fifo.clear();
    if (!s.sim) {   // still waiting for admission: the worker drops it
        sv->cv.notify_all();
        return VD_OK;
    }
    sv->cv.notify_all();
    sv->done_cv.wait(lock, [&] { return sv->error || s.inflight == 0; });
    if (sv->error) return server_error(sv);
    vd_sim *sim = s.sim;
    sv->order.erase(std::find(sv->order.begin(), sv->order.end(), sim_id));
    sv->pool.release(s.off, s.bytes);
    sv->sims.erase(it);
    vd_destroy(sim);
    sv->cv.notify_all();   // memory freed: waiting simulations may be admitted
    return VD_OK;
}

int vd_server_read_map(vd_server *sv, int32_t sim_id, int32_t *host_dst, size_t count)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(sv->mu);
    auto it = sv->sims.find(sim_id);
    if (it == sv->sims.end()) return fail(VD_EINVAL, "no simulation %d", sim_id);
    Served &s = it->second;
    if (!s.sim) return fail(VD_ESTATE, "simulation %d is not resident yet", sim_id);
    if (sv->error) return server_error(sv);   // its steps may never complete
    if (s.running || !s.fifo.empty())
        return fail(VD_ESTATE, "simulation %d has requests in progress", sim_id);
    return vd_read_map(s.sim, host_dst, count);
}

int vd_server_sim_state(vd_server *sv, int32_t sim_id, int32_t *resident, int64_t *t,
                        int32_t *pending)
{
    if (!sv) return fail(VD_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(sv->mu);
    auto it = sv->sims.find(sim_id);
    if (it == sv->sims.end()) return fail(VD_EINVAL, "no simulation %d", sim_id);
    const Served &s = it->second;
    if (resident) *resident = s.sim != nullptr;
    if (t) *t = s.sim ? s.sim->t : 0;
    if (pending) *pending = (int32_t)s.fifo.size() + s.running;
    return VD_OK;
}

int vd_server_stats(vd_server *sv, vd_server_stats_t *out, int reset)
{
    if (!sv || !out) return fail(VD_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(sv->mu);
    memset(out, 0, sizeof *out);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->pixel_updates = sv->pixel_updates;
    out->ticks = sv->ticks;
    out->elapsed_s = vd::ms_between(sv->stats_t0, vd::Clock::now()) / 1e3;
    int32_t res = 0;
    for (auto &kv : sv->sims) res += kv.second.sim != nullptr;
    out->resident = res;
    out->waiting_admission = (int32_t)sv->admit_queue.size();
    std::vector<double> l = sv->latencies;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto q = [&](double p) {
            size_t i = (size_t)std::min<double>((double)l.size() - 1, p * (l.size() - 1) + 0.5);
            return l[i];
        };
        double sum = 0;
        for (double v : l) sum += v;
        out->mean_ms = sum / l.size();
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        out->max_ms = l.back();
    }
    if (reset) {
        sv->latencies.clear();
        sv->submitted = sv->completed = sv->pixel_updates = sv->ticks = 0;
        sv->stats_t0 = vd::Clock::now();
    }
    return sv->error ? server_error(sv) : VD_OK;
}

void vd_server_destroy(vd_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lock(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipStreamSynchronize(sv->stream);
    for (Tick &t : sv->inflight)
        if (t.done) (void)hipEventDestroy(t.done);
    for (auto &kv : sv->sims)
        if (kv.second.sim) vd_destroy(kv.second.sim);
    for (hipStream_t l : sv->lane)
        if (l) (void)hipStreamSynchronize(l);
    release_lanes(sv);
    if (sv->host_ring) (void)hipHostFree(sv->host_ring);
    delete sv;
}

}  // extern "C"
