// Internal state of a simulation, shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "vd_kernels.h"
#include "../../include/vdflood.h"

namespace vd {

struct Pass {
    int32_t k;
    int32_t vn;
    int32_t variant;    // flood kernel variant (same result, different speed)
    int32_t seg_rows;   // rows per chain segment, 0: chosen from the map size
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;     // 0: flood passes, 1: whole step
    int count = 1;    // kind 0: passes between the two events
};

// Sets this thread's vd_last_error() message; returns status.
int fail(int status, const char *fmt, ...);

// Eq. (2): the first JFA step k1 (0 for a 1-pixel grid).
int32_t first_k(int32_t W, int32_t H);
// Eq. (5): the first dJFA step delta_1, capped at k1.
int32_t first_delta(int32_t W, int32_t H, int32_t S, int32_t dmax);
// Kernel variant of a pass and tile height of fused last passes before any
// tuning (both change speed only).
int32_t default_variant(const vd_config &c, bool dynamic, int32_t k);
int32_t default_tail_th(const vd_config &c, bool dynamic);
// Checks a configuration; sets the error message and returns VD_EINVAL.
int validate(const vd_config *c);

// Number of trailing passes that can run as one fused launch: the longest
// suffix of steps 1, 2 or 4 summing to at most kTailHalo, at most
// kTailMaxPasses long; 0 if shorter than two.
inline size_t tail_len(const std::vector<Pass> &passes)
{
    size_t m = 0;
    int32_t sum = 0;
    while (m < passes.size() && m < (size_t)kTailMaxPasses) {
        const int32_t k = passes[passes.size() - 1 - m].k;
        if ((k != 1 && k != 2 && k != 4) || sum + k > kTailHalo) break;
        sum += k;
        ++m;
    }
    return m >= 2 ? m : 0;
}

}  // namespace vd

struct vd_batch;

struct vd_sim {
    vd_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint32_t *map[2] = {nullptr, nullptr};
    int cur = 0;                 // map[cur] holds the current diagram
    uint32_t *pos = nullptr;     // seed table: sentinel, then current positions
    uint32_t *pos_map = nullptr; // XY mode: the table the diagram's labels refer to
    uint32_t *idx = nullptr;     // XY mode: the old-position index of dJFA steps (a map)
    int32_t idx_builds = 0;      // single-launch index builds since idx was filled with
                                 // all ones (kIndexEpochs: fill before the next)
    int32_t reach = 0;           // bound on how far (per axis) any seed has moved since the
                                 // diagram was made
    bool diagram = false;        // map[cur] holds a diagram (no marked labels): an XY JFA
                                 // step may start from it instead of a filled map
    int64_t t = 0;
    int32_t dmax = 0;
    uint32_t *disp = nullptr;    // [0]: displacement bound since the last step, [1]: scratch
                                 // of a move, [2]: unclaimed-pixel count of a step
    // The seed set (insertion and removal): one byte per seed, kPresent |
    // kKept, on the device and mirrored here.
    uint8_t *state = nullptr;
    std::vector<uint8_t> host_state;
    uint32_t *parked = nullptr;  // ID labels: positions of absent seeds (their table
                                 // entries hold the sentinel)
    int32_t present = 0;         // seeds in the set now
    bool changed = false;        // a seed inserted or removed since the diagram was made
    bool removed = false;        // a seed removed since then
    bool reinserted = false;     // a slot removed since then was inserted again
    bool masked = false;         // changed, or some seed absent: kernels read `state`
    int64_t fallbacks = 0;       // dJFA steps replaced by a JFA step (unrefilled pixels)
    bool measured = false;       // d_max of each dJFA step from disp[0]
    int32_t forced_variant = -1; // vd_set_flood_variant's choice, -1: defaults and tuning
    int32_t tail_th[2] = {0, 0}; // JFA, dJFA: last passes in one launch with tiles of this
                                 // height (16, 24, 32), 0: not fused
    int32_t forced_fuse = -1;    // vd_set_tail_fusion's tile height (0: off), -1: defaults
                                 // and tuning
    int32_t k1 = 0, delta1 = 0;
    uint64_t move_seed = 0;
    std::vector<vd::Pass> jfa_passes, djfa_passes;
    bool timing = false;
    std::vector<vd::EventPair> pool;   // recorded pairs
    size_t used = 0;
    vd_timing acc{};
    bool broken = false;
    vd_batch *batch = nullptr;   // set while a batch drives this simulation
    bool release = false;        // vd_destroy was called while in a batch: the batch's
                                 // destruction releases the handle
};

namespace vd {
// The flood passes of a step of kind `dynamic` on `stream`, as the
// simulation's own step runs them (its kernel variants and fused tail;
// an XY dJFA step's relabel must have run first), flipping s->cur per
// launch.  For drivers of many simulations (the server's batched ticks).
int launch_step_passes(vd_sim *s, bool dynamic, hipStream_t stream);

// Whether the first two of the n passes that run with launches of their
// own (ps minus a fused tail) run as one launch (launch_flood_pair): k and
// k / 2, both Moore, on a map of sides at most 2 k (a JFA step's start).
inline bool pair_at_start(const vd_sim *s, const std::vector<Pass> &ps, size_t n)
{
    return n >= 2 && ps[0].vn == 0 && ps[1].vn == 0 && ps[1].k * 2 == ps[0].k &&
           flood_pair_ok(s->cfg.width, s->cfg.height, ps[0].k);
}

// Launches of a step of kind `dynamic` run by the simulation's own pass
// driver (the fused tail and the fused first two passes count once); each
// flips the current map.
inline int32_t step_launches(const vd_sim *s, bool dynamic)
{
    const std::vector<Pass> &ps = dynamic ? s->djfa_passes : s->jfa_passes;
    const size_t m = s->tail_th[dynamic ? 1 : 0] ? tail_len(ps) : 0;
    const bool pair = pair_at_start(s, ps, ps.size() - m);
    return (int32_t)(ps.size() - (m ? m - 1 : 0) - (pair ? 1 : 0));
}
}  // namespace vd
