// vdflood runtime: simulation state, workspace carving, pass schedules,
// stream ordering, timing, and the C ABI of include/vdflood.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vd_sim.h"

namespace vd {

thread_local char g_err[512] = "";

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

}  // namespace vd

using vd::fail;
using vd::Pass;
using vd::EventPair;

namespace {

#define VD_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(VD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

namespace vd {

// Eq. (2): k1 = 2^(ceil(log2 N) - 1), N = max(W, H); 0 for a 1-pixel grid.
int32_t first_k(int32_t W, int32_t H)
{
    int64_t N = W > H ? W : H;
    if (N <= 1) return 0;
    int64_t p = 1;
    while (p < N) p <<= 1;
    return (int32_t)(p >> 1);
}

// Eq. (5) with L_avg = sqrt(W*H/S) (Eq. (4)): the smallest power of two P
// with P >= d_max and P >= 2 L_avg, i.e. P*P*S >= 4*W*H; capped at k1.
int32_t first_delta(int32_t W, int32_t H, int32_t S, int32_t dmax)
{
    int32_t k1 = first_k(W, H);
    if (k1 == 0) return 0;
    int64_t P = 1;
    while (P < dmax || P * P * (int64_t)S < 4 * (int64_t)W * (int64_t)H) P <<= 1;
    return P < k1 ? (int32_t)P : k1;
}

// Kernel variant of a pass before any tuning, from measurements on MI355X
// (4096^2 and 8192^2 maps, the autotuner's choices): ID labels take the
// four-column kernel in JFA steps (many distinct labels: fewer, wider
// loads win) and LDS-shared rows in dJFA steps (few distinct labels); XY
// labels take the four-column kernel for JFA's long jumps and the chain
// walk otherwise.  When the two maps exceed what the 256 MB Infinity Cache
// can keep (here: 192 MiB), the output maps are stored non-temporally.
int32_t default_variant(const vd_config &c, bool dynamic, int32_t k)
{
    int32_t v;
    if (c.label == VD_LABEL_ID32)
        v = dynamic ? 3 : 4;
    else
        v = !dynamic && k >= 512 ? 4 : 1;
    if (8 * (int64_t)c.width * c.height > (int64_t)192 << 20) v += vd::kFloodVariants / 2;
    return v;
}

// Tile height of a step kind's fused last passes before any tuning (0: not
// fused).  Measured on MI355X (square maps, one seed per 256 pixels, both
// step kinds): the fused launch saves two launches and two map round trips
// but recomputes the tile halo and leaves up to a quarter of its lanes
// idle, about 1.6x the arithmetic of the separate passes.  It wins while
// the passes are short (up to 2048^2 with ID labels, 1536^2 with XY labels:
// 10-20% per step) and loses on larger maps, whose separate passes are
// bound by arithmetic and table lookups rather than by launches or bytes.
int32_t default_tail_th(const vd_config &c, bool)
{
    const int64_t px = (int64_t)c.width * c.height;
    const int64_t limit = c.label == VD_LABEL_ID32 ? 2048 * 2048 : 1536 * 1536;
    if (px > limit) return 0;
    return px <= ((int64_t)1 << 19) ? 16 : 24;
}

int validate(const vd_config *c)
{
    if (!c) return fail(VD_EINVAL, "config is NULL");
    if (c->width < 1 || c->width > VD_MAX_SIDE || c->height < 1 || c->height > VD_MAX_SIDE)
        return fail(VD_EINVAL, "width and height must be in [1, %d], got %d x %d", VD_MAX_SIDE,
                    c->width, c->height);
    if (c->num_seeds < 1 || (int64_t)c->num_seeds > (int64_t)c->width * c->height)
        return fail(VD_EINVAL, "num_seeds must be in [1, width*height], got %d", c->num_seeds);
    if (c->disp_lo > c->disp_hi || c->disp_lo < -VD_MAX_SIDE || c->disp_hi > VD_MAX_SIDE)
        return fail(VD_EINVAL, "need -%d <= disp_lo <= disp_hi <= %d, got [%d, %d]", VD_MAX_SIDE,
                    VD_MAX_SIDE, c->disp_lo, c->disp_hi);
    if (c->label != VD_LABEL_ID32 && c->label != VD_LABEL_XY16)
        return fail(VD_EINVAL, "unknown label mode %d", c->label);
    if (c->metric != VD_EUCLID && c->metric != VD_MANHATTAN)
        return fail(VD_EINVAL, "unknown metric %d", c->metric);
    if (c->vn_passes < 0 || c->vn_passes > 64)
        return fail(VD_EINVAL, "vn_passes must be in [0, 64], got %d", c->vn_passes);
    if (c->extra_passes < 0 || c->extra_passes > VD_MAX_EXTRA_PASSES)
        return fail(VD_EINVAL, "extra_passes must be 0, 1 or 2, got %d", c->extra_passes);
    if (c->dmax_override > 2 * VD_MAX_SIDE || c->dmax_override < VD_DMAX_MEASURED)
        return fail(VD_EINVAL, "dmax_override must be in [%d, %d], got %d", VD_DMAX_MEASURED,
                    2 * VD_MAX_SIDE, c->dmax_override);
    return VD_OK;
}

}  // namespace vd

using vd::first_k;
using vd::first_delta;
using vd::default_variant;
using vd::default_tail_th;
using vd::validate;

namespace {

constexpr int32_t kTailHeights[] = {16, 24, 32};

void set_default_variants(vd_sim *s)
{
    for (Pass &p : s->jfa_passes) p.variant = default_variant(s->cfg, false, p.k);
    for (Pass &p : s->djfa_passes) p.variant = default_variant(s->cfg, true, p.k);
    for (int dyn = 0; dyn < 2; ++dyn)
        s->tail_th[dyn] = s->forced_fuse >= 0 ? s->forced_fuse : default_tail_th(s->cfg, dyn != 0);
}


// Pass list of one step: k = first, first/2, ..., 1; the first vn of them
// Von Neumann (clamped so the last main pass is Moore); extra passes k = 1
// (one extra) or k = 2, 1 (two extras), Moore.
std::vector<Pass> schedule(int32_t first, int32_t vn_passes, int32_t extra, int32_t variant)
{
    std::vector<Pass> out;
    int32_t n = 0;
    for (int32_t k = first; k >= 1; k >>= 1) ++n;
    int32_t vn = vn_passes < n - 1 ? vn_passes : n - 1;
    if (vn < 0) vn = 0;
    int32_t i = 0;
    for (int32_t k = first; k >= 1; k >>= 1, ++i)
        out.push_back({k, i < vn ? 1 : 0, variant, 0});
    for (int32_t e = extra; e >= 1; --e) out.push_back({e, 0, variant, 0});
    return out;
}

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

size_t footprint(const vd_config *c)
{
    size_t npix = (size_t)c->width * (size_t)c->height;
    size_t seeds = (size_t)c->num_seeds * 4;
    size_t b = 2 * align_up(npix * 4) + align_up(seeds + 4);   // + the sentinel entry
    if (c->label == VD_LABEL_XY16) b += align_up(seeds + 4) + align_up(npix * 4);
    b += align_up(12);                     // step counters
    b += align_up((size_t)c->num_seeds);   // seed-set state bytes
    if (c->label == VD_LABEL_ID32) b += align_up(seeds);   // parked positions
    return b + kAlign;
}

}  // namespace

namespace {

int record(vd_sim *s, int kind, bool begin, size_t *slot, int count = 1)
{
    if (!s->timing) return VD_OK;
    if (begin) {
        if (s->used == s->pool.size()) {
            EventPair p;
            VD_HIP(hipEventCreate(&p.a));
            VD_HIP(hipEventCreate(&p.b));
            s->pool.push_back(p);
        }
        *slot = s->used++;
        s->pool[*slot].kind = kind;
        s->pool[*slot].count = count;
        VD_HIP(hipEventRecord(s->pool[*slot].a, s->stream));
    } else {
        VD_HIP(hipEventRecord(s->pool[*slot].b, s->stream));
    }
    return VD_OK;
}

int harvest(vd_sim *s)
{
    if (s->used == 0) return VD_OK;
    VD_HIP(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < s->used; ++i) {
        float ms = 0.f;
        VD_HIP(hipEventElapsedTime(&ms, s->pool[i].a, s->pool[i].b));
        if (s->pool[i].kind == 0) {
            s->acc.flood_launches += s->pool[i].count;
            s->acc.flood_ms += ms;
            s->acc.flood_pixels += (int64_t)s->pool[i].count * s->cfg.width * s->cfg.height;
        } else {
            s->acc.step_count += 1;
            s->acc.step_ms += ms;
        }
    }
    s->used = 0;
    return VD_OK;
}

// The passes of one step run back to back between one pair of timing
// events (events around every launch would add their own latency to each
// short pass).
// With th (a tile height) non-zero, the step's last passes (tail_len) run
// as one launch with the store policy of the last pass.
// With relabel (an XY dJFA step's old-position index) non-null, the first
// pass reads the previous diagram through it (launch_flood_relabel); with
// seeds, an XY JFA step's first pass reads the previous diagram with the
// seed pixels marked (launch_flood_seeds).  Where the first two passes are
// k and k / 2 on a map of sides at most 2 k (a JFA step's start), they run
// as one launch (launch_flood_pair).
int launch_passes(vd_sim *s, const std::vector<Pass> &passes, int32_t th,
                  const uint32_t *relabel = nullptr, hipStream_t stream = nullptr,
                  bool seeds = false)
{
    if (!stream) stream = s->stream;
    const size_t m = th ? vd::tail_len(passes) : 0;
    const size_t n = passes.size() - m;
    for (size_t i = 0; i < n; ++i) {
        const Pass &p = passes[i];
        if (i == 0 && !relabel && vd::pair_at_start(s, passes, n)) {
            // the first two passes in one launch (the store policy of the second)
            VD_HIP(vd::launch_flood_pair(s->map[s->cur], s->map[s->cur ^ 1], s->pos,
                                         s->cfg.num_seeds, s->cfg.width, s->cfg.height, p.k,
                                         s->cfg.label, seeds, s->cfg.metric,
                                         passes[1].variant >= vd::kFloodVariants / 2, stream));
            s->cur ^= 1;
            ++i;
            continue;
        }
        if (i == 0 && relabel)
            VD_HIP(vd::launch_flood_relabel(s->map[s->cur], s->map[s->cur ^ 1], relabel,
                                            s->cfg.width, s->cfg.height, p.k, p.vn,
                                            s->cfg.metric, p.variant, p.seg_rows, stream));
        else if (i == 0 && seeds)
            VD_HIP(vd::launch_flood_seeds(s->map[s->cur], s->map[s->cur ^ 1], s->cfg.width,
                                          s->cfg.height, p.k, p.vn, s->cfg.metric, p.variant,
                                          stream));
        else
            VD_HIP(vd::launch_flood(s->map[s->cur], s->map[s->cur ^ 1], s->pos,
                                    s->cfg.num_seeds, s->cfg.width, s->cfg.height, p.k, p.vn,
                                    s->cfg.label, s->cfg.metric, p.variant, p.seg_rows,
                                    stream));
        s->cur ^= 1;
    }
    if (m) {
        int32_t ks[vd::kTailMaxPasses], vns[vd::kTailMaxPasses];
        for (size_t i = 0; i < m; ++i) {
            ks[i] = passes[n + i].k;
            vns[i] = passes[n + i].vn;
        }
        const bool nt = passes.back().variant >= vd::kFloodVariants / 2;
        VD_HIP(vd::launch_flood_tail(s->map[s->cur], s->map[s->cur ^ 1], s->pos,
                                     s->cfg.num_seeds, s->cfg.width, s->cfg.height, ks, vns,
                                     (int32_t)m, s->cfg.label, s->cfg.metric, nt, th,
                                     stream));
        s->cur ^= 1;
    }
    return VD_OK;
}

int run_passes(vd_sim *s, const std::vector<Pass> &passes, int32_t th,
               const uint32_t *relabel = nullptr, bool seeds = false)
{
    if (passes.empty()) return VD_OK;
    size_t slot = 0;
    int r = record(s, 0, true, &slot, (int)passes.size());
    if (r) return r;
    r = launch_passes(s, passes, th, relabel, nullptr, seeds);
    if (r) return r;
    r = record(s, 0, false, &slot);
    if (r) return r;
    if (s->timing && s->used >= 4096) {
        r = harvest(s);
        if (r) return r;
    }
    return VD_OK;
}

}  // namespace

namespace vd {

int launch_step_passes(vd_sim *s, bool dynamic, hipStream_t stream)
{
    return launch_passes(s, dynamic ? s->djfa_passes : s->jfa_passes, s->tail_th[dynamic ? 1 : 0],
                         nullptr, stream);
}

}  // namespace vd

namespace {

// The seed-set bytes the kernels read: null while every seed is present
// and kept (the common case costs nothing).
const uint8_t *seed_state(const vd_sim *s) { return s->masked ? s->state : nullptr; }

// Whether an XY JFA step skips the fill: its first pass then reads the
// previous diagram, where only the seed pixels (splatted with the top bit)
// count as claimed.  Needs a diagram in map[cur] and the block tile for the
// first pass, run with its own launch.
bool seeds_for(const vd_sim *s, const std::vector<Pass> &passes, int32_t th)
{
    if (s->cfg.label != VD_LABEL_XY16 || !s->diagram || passes.empty()) return false;
    const size_t m = th ? vd::tail_len(passes) : 0;
    if (m >= passes.size()) return false;
    return vd::flood_seeds_ok(s->cfg.width, s->cfg.height, passes[0].k);
}

// The map a JFA step floods: unclaimed everywhere but the seed pixels.  ID
// maps are filled with all ones rather than label 0 (both read as the
// sentinel position in the passes, and every pixel is claimed by the end
// of the step), so the atomic minimum of the seed labels needs no reset.
// With seeds (seeds_for), an XY step leaves the previous diagram in place
// and marks the seed pixels instead.
int jfa_prologue(vd_sim *s, bool seeds)
{
    const vd_config &c = s->cfg;
    int64_t npix = (int64_t)c.width * c.height;
    if (c.label == VD_LABEL_XY16 && seeds) {
        VD_HIP(vd::launch_splat_xy_marked(s->map[s->cur], s->pos, c.num_seeds, c.width,
                                          seed_state(s), s->stream));
    } else if (c.label == VD_LABEL_XY16) {
        VD_HIP(vd::launch_fill(s->map[s->cur], npix, vd::kEmpty, s->stream));
        VD_HIP(vd::launch_splat_xy(s->map[s->cur], s->pos, c.num_seeds, c.width, seed_state(s),
                                   s->stream));
    } else {
        VD_HIP(vd::launch_fill(s->map[s->cur], npix, 0xFFFFFFFFu, s->stream));
        VD_HIP(vd::launch_splat_id_over_ones(s->map[s->cur], s->pos, c.num_seeds, c.width,
                                             seed_state(s), s->stream));
    }
    return VD_OK;
}

// The map a dJFA step floods: the previous diagram (XY: relabelled to the
// moved positions) with every seed pixel claimed by its seed.  After
// insertions or removals, labels of seeds not kept since the diagram was
// made leave it first.  XY: the relabel finds no kept seed for them.  ID: a
// removed seed's table entry holds the sentinel position, so the passes
// treat its labels like unclaimed pixels without touching the map; only a
// slot removed and inserted again (whose entry is a live position) needs
// its old labels purged.
// Whether an XY dJFA step translates the previous diagram's labels inside
// its first flood pass (which then reads the map through the index) rather
// than in a relabel pass of its own: where the four-column shared-row tile
// runs that pass and it is not part of a fused tail, and the index's move
// codes hold every seed's move since the diagram was made.
bool fold_for(const vd_sim *s, const std::vector<Pass> &passes, int32_t th)
{
    if (s->cfg.label != VD_LABEL_XY16 || !s->idx || passes.empty() ||
        (uint32_t)s->cfg.num_seeds + 1u >= vd::kIndexNoLabel || s->reach > vd::kIndexMaxReach)
        return false;
    const size_t m = th ? vd::tail_len(passes) : 0;
    if (m >= passes.size()) return false;
    return vd::relabel_fold_ok(s->cfg.width, passes[0].k);
}

bool fold_relabel(const vd_sim *s) { return fold_for(s, s->djfa_passes, s->tail_th[1]); }

int djfa_prologue(vd_sim *s, bool fold)
{
    const vd_config &c = s->cfg;
    uint32_t *cur = s->map[s->cur];
    if (c.label == VD_LABEL_XY16 && fold) {
        // The index of old positions goes to its own map; the first pass
        // reads the diagram through it.  This step's seed pixels are marked
        // so that the first pass takes them as they are.
        if (s->idx_builds >= vd::kIndexEpochs) {
            VD_HIP(vd::launch_fill(s->idx, (int64_t)c.width * c.height, 0xFFFFFFFFu,
                                   s->stream));
            s->idx_builds = 0;
        }
        const uint32_t epoch = (uint32_t)(vd::kIndexEpochs - 1 - s->idx_builds++);
        VD_HIP(vd::launch_index_marked(s->idx, cur, s->pos_map, s->pos, c.num_seeds, c.width,
                                       seed_state(s), epoch, s->stream));
    } else if (c.label == VD_LABEL_XY16) {
        // The idle ping-pong buffer serves as the old-position index; the
        // first flood pass overwrites it.
        uint32_t *idx = s->map[s->cur ^ 1];
        VD_HIP(vd::launch_index_old(idx, s->pos_map, s->pos, c.num_seeds, c.width, seed_state(s),
                                    s->stream));
        VD_HIP(vd::launch_relabel(cur, idx, c.width, c.height, s->stream));
        VD_HIP(vd::launch_splat_xy(cur, s->pos, c.num_seeds, c.width, seed_state(s), s->stream));
    } else {
        if (s->reinserted)
            VD_HIP(vd::launch_purge(cur, s->state, c.num_seeds, (int64_t)c.width * c.height,
                                    s->stream));
        VD_HIP(vd::launch_splat_id(cur, s->pos, c.num_seeds, c.width, seed_state(s), s->stream));
    }
    return VD_OK;
}

// XY mode: the diagram now refers to the current positions.
int step_epilogue(vd_sim *s)
{
    const vd_config &c = s->cfg;
    if (c.label == VD_LABEL_XY16)
        VD_HIP(hipMemcpyAsync(s->pos_map, s->pos, ((size_t)c.num_seeds + 1) * 4,
                              hipMemcpyDeviceToDevice, s->stream));
    return VD_OK;
}

int do_jfa(vd_sim *s)
{
    const bool seeds = seeds_for(s, s->jfa_passes, s->tail_th[0]);
    int r = jfa_prologue(s, seeds);
    if (r == VD_OK) r = run_passes(s, s->jfa_passes, s->tail_th[0], nullptr, seeds);
    if (r == VD_OK) r = step_epilogue(s);
    return r;
}

int do_djfa(vd_sim *s)
{
    const bool fold = fold_relabel(s);
    int r = djfa_prologue(s, fold);
    if (r == VD_OK) r = run_passes(s, s->djfa_passes, s->tail_th[1], fold ? s->idx : nullptr);
    if (r == VD_OK) r = step_epilogue(s);
    return r;
}

// After a dJFA step that followed removals: a removed seed's cell must
// have been refilled by its neighbours within the passes.  If a pixel is
// still unclaimed (label 0, or in ID mode an absent seed's label), the step
// is redone as a full JFA step.  Reads the count back, so the step waits
// for its stream here.
int refill_check(vd_sim *s)
{
    const vd_config &c = s->cfg;
    uint32_t n = 0;
    VD_HIP(vd::launch_count_unclaimed(s->map[s->cur], (int64_t)c.width * c.height,
                                      c.label == VD_LABEL_ID32 ? s->state : nullptr,
                                      c.num_seeds, &s->disp[2], s->stream));
    VD_HIP(hipMemcpyAsync(&n, &s->disp[2], 4, hipMemcpyDeviceToHost, s->stream));
    VD_HIP(hipStreamSynchronize(s->stream));
    if (n == 0) return VD_OK;
    s->fallbacks += 1;
    return do_jfa(s);
}

// After a step: the diagram holds exactly the present seeds.
int settle(vd_sim *s)
{
    if (!s->masked) return VD_OK;
    VD_HIP(vd::launch_settle(s->state, s->cfg.num_seeds, s->stream));
    for (uint8_t &b : s->host_state)
        b = (b & vd::kPresent) ? (uint8_t)(vd::kPresent | vd::kKept) : (uint8_t)0;
    s->changed = s->removed = s->reinserted = false;
    s->masked = s->present < s->cfg.num_seeds;
    return VD_OK;
}

void apply_tuning(vd_sim *s);

// The dJFA schedule for the current d_max and number of present seeds
// (Eq. (5)); passes are rebuilt only when delta_1 changes.
void replan_djfa(vd_sim *s)
{
    const vd_config &c = s->cfg;
    const int32_t delta1 = first_delta(c.width, c.height, s->present, s->dmax);
    if (delta1 == s->delta1 && !s->djfa_passes.empty()) return;
    s->delta1 = delta1;
    s->djfa_passes = schedule(delta1, c.vn_passes, c.extra_passes, 0);
    for (Pass &p : s->djfa_passes)
        p.variant = s->forced_variant >= 0 ? s->forced_variant : default_variant(c, true, p.k);
    if (s->forced_variant < 0) apply_tuning(s);
}

// Measured d_max (dmax_override = VD_DMAX_MEASURED): the dJFA schedule of
// this step from the displacement the moves since the last step recorded
// on the device.  Reads it back, so the step waits for the stream here.
int measured_schedule(vd_sim *s)
{
    uint32_t d = 0;
    VD_HIP(hipMemcpyAsync(&d, s->disp, 4, hipMemcpyDeviceToHost, s->stream));
    VD_HIP(hipStreamSynchronize(s->stream));
    s->dmax = (int32_t)std::min<uint32_t>(d, 2u * VD_MAX_SIDE);
    replan_djfa(s);
    return VD_OK;
}

int step(vd_sim *s, bool dynamic)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    int r = VD_OK;
    if (dynamic && s->measured) r = measured_schedule(s);
    if (r) {
        s->broken = true;
        return r;
    }
    size_t slot = 0;
    r = record(s, 1, true, &slot);
    if (r) return r;
    const bool removed = s->removed;
    r = dynamic ? do_djfa(s) : do_jfa(s);
    if (r == VD_OK) {
        s->reach = 0;   // the diagram refers to the current positions
        s->diagram = true;
    }
    if (r == VD_OK && dynamic && removed) r = refill_check(s);
    if (r == VD_OK) r = settle(s);
    // the diagram now refers to the current positions
    if (r == VD_OK && s->measured) {
        hipError_t e = vd::launch_fill(s->disp, 1, 0u, s->stream);
        if (e != hipSuccess) r = fail(VD_EDEVICE, "counter reset failed: %s", hipGetErrorString(e));
    }
    if (r == VD_OK) r = record(s, 1, false, &slot);
    if (r == VD_EDEVICE) s->broken = true;
    return r;
}

// ---------------------------------------------------------------------------
// Autotuning.  A pass's kernel variant and segment length change its speed,
// never its output, so they can be chosen by timing.  Choices live in a
// process-wide table keyed by (GPU architecture, grid, seed count, label,
// metric, k, neighbourhood); simulations created later with the same key
// start from them.  The table can be exported and imported as text.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, std::pair<int32_t, int32_t>> g_tune;   // key -> (variant, seg_rows)
std::map<std::string, float> g_tune_us;   // key -> best measured pass time (this process)

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// A pass of a JFA step and one of a dJFA step with the same k read very
// different maps (partly flooded vs nearly converged), so the step kind is
// part of the key.
std::string tune_key(const std::string &arch, const vd_config &c, const Pass &p, bool dynamic)
{
    char buf[192];
    snprintf(buf, sizeof buf, "%s %dx%d S%d %s %s k%d %s %s", arch.c_str(), c.width, c.height,
             c.num_seeds, c.label == VD_LABEL_XY16 ? "xy" : "id",
             c.metric == VD_MANHATTAN ? "manhattan" : "euclid", p.k, p.vn ? "vn" : "moore",
             dynamic ? "djfa" : "jfa");
    return buf;
}

// Key of a step kind's tail-fusion choice (value: 0 not fused, i > 0 fused
// with tiles of height kTailHeights[i - 1]).
std::string fuse_key(const std::string &arch, const vd_config &c, bool dynamic)
{
    char buf[192];
    snprintf(buf, sizeof buf, "%s %dx%d S%d %s %s tail %s", arch.c_str(), c.width, c.height,
             c.num_seeds, c.label == VD_LABEL_XY16 ? "xy" : "id",
             c.metric == VD_MANHATTAN ? "manhattan" : "euclid", dynamic ? "djfa" : "jfa");
    return buf;
}

void apply_tuning(vd_sim *s)
{
    const std::string arch = arch_name();
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (int dyn = 0; dyn < 2; ++dyn) {
        for (Pass &p : dyn ? s->djfa_passes : s->jfa_passes) {
            auto it = g_tune.find(tune_key(arch, s->cfg, p, dyn != 0));
            if (it != g_tune.end()) {
                p.variant = it->second.first;
                p.seg_rows = it->second.second;
            }
        }
        if (s->forced_fuse < 0) {
            auto it = g_tune.find(fuse_key(arch, s->cfg, dyn != 0));
            if (it != g_tune.end()) {
                const int32_t v = it->second.first;
                s->tail_th[dyn] = v >= 1 && v <= 3 ? kTailHeights[v - 1] : 0;
            }
        }
    }
}

}  // namespace

extern "C" {

int vd_autotune(vd_sim *s, int32_t reps)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    if (reps < 1 || reps > 1000) return fail(VD_EINVAL, "reps must be in [1, 1000], got %d", reps);
    const vd_config &c = s->cfg;
    static const int32_t kSegRows[] = {0, 8, 16, 64};
    struct Cand {
        int32_t variant, seg_rows;
    };
    // Kernel and segment length are chosen per pass among the variants with
    // ordinary stores; whether the output maps are stored non-temporally is
    // then chosen per step kind from whole replayed steps, because it
    // changes the speed of the next pass (which finds, or does not find,
    // its input in the Infinity Cache), not of the pass that stores.
    constexpr int32_t kBase = vd::kFloodVariants / 2;
    std::vector<Cand> cands;
    for (int32_t v = 0; v < kBase; ++v)
        for (int32_t L : kSegRows) cands.push_back({v, L});
    const std::string arch = arch_name();
    const size_t npix = (size_t)c.width * c.height;
    const size_t tab_bytes = ((size_t)c.num_seeds + 1) * 4;
    const int cur0 = s->cur;

    // The replayed steps overwrite both maps (and, in XY mode, nothing
    // else); the diagram and the XY position table are saved and put back.
    uint32_t *save = nullptr, *save_pm = nullptr;
    if (hipMalloc((void **)&save, npix * 4) != hipSuccess ||
        (s->pos_map && hipMalloc((void **)&save_pm, tab_bytes) != hipSuccess)) {
        if (save) (void)hipFree(save);
        return fail(VD_ENOMEM, "autotune needs %zu bytes of device scratch", npix * 4 + tab_bytes);
    }
    std::vector<std::string> keys;     // distinct passes, in replay order
    std::vector<int> key_dyn;          // their step kind (1: dJFA)
    std::vector<hipEvent_t> ev;        // two per (pass, candidate)
    int r = VD_OK;
    auto hip = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && r == VD_OK)
            r = fail(VD_EDEVICE, "autotune: %s failed: %s", what, hipGetErrorString(e));
        return r == VD_OK;
    };
    hip(hipMemcpyAsync(save, s->map[s->cur], npix * 4, hipMemcpyDeviceToDevice, s->stream),
        "save");
    if (save_pm)
        hip(hipMemcpyAsync(save_pm, s->pos_map, tab_bytes, hipMemcpyDeviceToDevice, s->stream),
            "save");
    // Replay one JFA step (from scratch) and one dJFA step (from the saved
    // diagram).  Before each pass, every candidate runs on the pass's real
    // input (reading it, writing the idle buffer); the pass itself then
    // advances the replay.
    // The replays run every pass with its own launch; an XY dJFA step's first
    // pass then reads through the old-position index where it can.
    const bool fold = fold_for(s, s->djfa_passes, 0);
    const bool seeds = seeds_for(s, s->jfa_passes, 0);
    for (int dyn = 0; dyn < 2 && r == VD_OK; ++dyn) {
        if (dyn) {
            hip(hipMemcpyAsync(s->map[s->cur], save, npix * 4, hipMemcpyDeviceToDevice,
                               s->stream), "restore");
            if (save_pm)
                hip(hipMemcpyAsync(s->pos_map, save_pm, tab_bytes, hipMemcpyDeviceToDevice,
                                   s->stream), "restore");
        }
        if (r == VD_OK) {
            int pr = dyn ? djfa_prologue(s, fold) : jfa_prologue(s, seeds);
            if (pr) r = pr;
        }
        size_t pass_i = 0;
        for (const Pass &p : dyn ? s->djfa_passes : s->jfa_passes) {
            if (r != VD_OK) break;
            std::string key = tune_key(arch, c, p, dyn != 0);
            bool fresh = std::find(keys.begin(), keys.end(), key) == keys.end();
            const bool first_pass = pass_i++ == 0;
            const bool relabel = dyn && fold && first_pass;
            const bool from_seeds = !dyn && seeds && first_pass;
            auto launch = [&](int32_t variant, int32_t seg_rows) {
                if (relabel)
                    return vd::launch_flood_relabel(s->map[s->cur], s->map[s->cur ^ 1], s->idx,
                                                    c.width, c.height, p.k, p.vn, c.metric,
                                                    variant, seg_rows, s->stream);
                if (from_seeds)
                    return vd::launch_flood_seeds(s->map[s->cur], s->map[s->cur ^ 1], c.width,
                                                  c.height, p.k, p.vn, c.metric, variant,
                                                  s->stream);
                return vd::launch_flood(s->map[s->cur], s->map[s->cur ^ 1], s->pos, c.num_seeds,
                                        c.width, c.height, p.k, p.vn, c.label, c.metric,
                                        variant, seg_rows, s->stream);
            };
            if (fresh) {
                keys.push_back(key);
                key_dyn.push_back(dyn);
                for (const Cand &cd : cands) {
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (!hip(hipEventCreate(&e0), "hipEventCreate")) break;
                    ev.push_back(e0);
                    if (!hip(hipEventCreate(&e1), "hipEventCreate")) break;
                    ev.push_back(e1);
                    if (!hip(launch(cd.variant, cd.seg_rows), "launch")) break;   // warm-up
                    if (!hip(hipEventRecord(e0, s->stream), "hipEventRecord")) break;
                    for (int32_t i = 0; i < reps && r == VD_OK; ++i)
                        hip(launch(cd.variant, cd.seg_rows), "launch");
                    if (!hip(hipEventRecord(e1, s->stream), "hipEventRecord")) break;
                }
            }
            if (hip(launch(p.variant, p.seg_rows), "launch")) s->cur ^= 1;
        }
    }
    hip(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    std::map<std::string, Cand> picks;
    std::map<std::string, float> pick_us;
    if (r == VD_OK && ev.size() == 2 * keys.size() * cands.size()) {
        for (size_t i = 0; i < keys.size(); ++i) {
            float best = 1e30f;
            Cand pick = cands[0];
            for (size_t j = 0; j < cands.size(); ++j) {
                float ms = 0.f;
                size_t at = 2 * (i * cands.size() + j);
                if (hipEventElapsedTime(&ms, ev[at], ev[at + 1]) == hipSuccess && ms < best) {
                    best = ms;
                    pick = cands[j];
                }
            }
            picks[keys[i]] = pick;
            pick_us[keys[i]] = 1e3f * best / reps;
        }
    }
    // Store policy per step kind: replay the step's passes with the picks,
    // with ordinary and with non-temporal stores, twice each; keep the faster.
    bool nt[2] = {false, false};
    for (int dyn = 0; dyn < 2 && r == VD_OK; ++dyn) {
        const std::vector<Pass> &passes = dyn ? s->djfa_passes : s->jfa_passes;
        float best[2] = {1e30f, 1e30f};
        for (int trial = 0; trial < 4 && r == VD_OK; ++trial) {
            const int policy = trial & 1;
            hip(hipMemcpyAsync(s->map[s->cur], save, npix * 4, hipMemcpyDeviceToDevice,
                               s->stream), "restore");
            if (save_pm)
                hip(hipMemcpyAsync(s->pos_map, save_pm, tab_bytes, hipMemcpyDeviceToDevice,
                                   s->stream), "restore");
            if (r == VD_OK) {
                int pr = dyn ? djfa_prologue(s, fold) : jfa_prologue(s, seeds);
                if (pr) r = pr;
            }
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (!hip(hipEventCreate(&e0), "hipEventCreate")) break;
            ev.push_back(e0);
            if (!hip(hipEventCreate(&e1), "hipEventCreate")) break;
            ev.push_back(e1);
            hip(hipEventRecord(e0, s->stream), "hipEventRecord");
            bool first = true;
            for (const Pass &p : passes) {
                if (r != VD_OK) break;
                const Cand &c0 = picks[tune_key(arch, c, p, dyn != 0)];
                const int32_t v = c0.variant + (policy ? kBase : 0);
                const hipError_t le =
                    dyn && fold && first
                        ? vd::launch_flood_relabel(s->map[s->cur], s->map[s->cur ^ 1], s->idx,
                                                   c.width, c.height, p.k, p.vn, c.metric, v,
                                                   c0.seg_rows, s->stream)
                    : !dyn && seeds && first
                        ? vd::launch_flood_seeds(s->map[s->cur], s->map[s->cur ^ 1], c.width,
                                                 c.height, p.k, p.vn, c.metric, v, s->stream)
                        : vd::launch_flood(s->map[s->cur], s->map[s->cur ^ 1], s->pos,
                                           c.num_seeds, c.width, c.height, p.k, p.vn, c.label,
                                           c.metric, v, c0.seg_rows, s->stream);
                first = false;
                if (hip(le, "launch")) s->cur ^= 1;
            }
            hip(hipEventRecord(e1, s->stream), "hipEventRecord");
            float ms = 0.f;
            if (hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
                hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime") && ms < best[policy])
                best[policy] = ms;
        }
        nt[dyn] = best[1] < best[0];
    }
    // Tail fusion per step kind, the same way: whole replayed steps with the
    // picks and the store policy, the last passes separate or fused with
    // each tile height (option 0: separate, i: kTailHeights[i - 1]).
    int32_t fz[2] = {0, 0};
    for (int dyn = 0; dyn < 2 && r == VD_OK; ++dyn) {
        std::vector<Pass> passes = dyn ? s->djfa_passes : s->jfa_passes;
        if (vd::tail_len(passes) == 0) continue;
        for (Pass &p : passes) {
            const Cand &c0 = picks[tune_key(arch, c, p, dyn != 0)];
            p.variant = c0.variant + (nt[dyn] ? kBase : 0);
            p.seg_rows = c0.seg_rows;
        }
        constexpr int kOpts = 1 + (int)(sizeof kTailHeights / sizeof kTailHeights[0]);
        float best[kOpts];
        for (float &b : best) b = 1e30f;
        for (int trial = 0; trial < 2 * kOpts && r == VD_OK; ++trial) {
            const int policy = trial % kOpts;
            hip(hipMemcpyAsync(s->map[s->cur], save, npix * 4, hipMemcpyDeviceToDevice,
                               s->stream), "restore");
            if (save_pm)
                hip(hipMemcpyAsync(s->pos_map, save_pm, tab_bytes, hipMemcpyDeviceToDevice,
                                   s->stream), "restore");
            const int32_t th = policy ? kTailHeights[policy - 1] : 0;
            const bool fold_t = dyn && fold_for(s, passes, th);
            const bool seeds_t = !dyn && seeds_for(s, passes, th);
            if (r == VD_OK) {
                int pr = dyn ? djfa_prologue(s, fold_t) : jfa_prologue(s, seeds_t);
                if (pr) r = pr;
            }
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (!hip(hipEventCreate(&e0), "hipEventCreate")) break;
            ev.push_back(e0);
            if (!hip(hipEventCreate(&e1), "hipEventCreate")) break;
            ev.push_back(e1);
            hip(hipEventRecord(e0, s->stream), "hipEventRecord");
            if (r == VD_OK) {
                int lr = launch_passes(s, passes, th, fold_t ? s->idx : nullptr, nullptr, seeds_t);
                if (lr) r = lr;
            }
            hip(hipEventRecord(e1, s->stream), "hipEventRecord");
            float ms = 0.f;
            if (hip(hipEventSynchronize(e1), "hipEventSynchronize") &&
                hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime") && ms < best[policy])
                best[policy] = ms;
        }
        for (int o = 1; o < kOpts; ++o)
            if (best[o] < best[fz[dyn]]) fz[dyn] = o;
    }
    if (r == VD_OK && !picks.empty()) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (size_t i = 0; i < keys.size(); ++i) {
            const Cand &pk = picks[keys[i]];
            g_tune[keys[i]] = {pk.variant + (nt[key_dyn[i]] ? kBase : 0), pk.seg_rows};
            g_tune_us[keys[i]] = pick_us[keys[i]];
        }
        for (int dyn = 0; dyn < 2; ++dyn)
            if (vd::tail_len(dyn ? s->djfa_passes : s->jfa_passes))
                g_tune[fuse_key(arch, c, dyn != 0)] = {fz[dyn], 0};
    }
    // put the diagram back where the simulation expects it
    s->cur = cur0;
    hipError_t e1 = hipMemcpyAsync(s->map[s->cur], save, npix * 4, hipMemcpyDeviceToDevice,
                                   s->stream);
    hipError_t e2 = save_pm ? hipMemcpyAsync(s->pos_map, save_pm, tab_bytes,
                                             hipMemcpyDeviceToDevice, s->stream)
                            : hipSuccess;
    hipError_t e3 = hipStreamSynchronize(s->stream);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    (void)hipFree(save);
    if (save_pm) (void)hipFree(save_pm);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        s->broken = true;
        if (r == VD_OK) r = fail(VD_EDEVICE, "autotune: restoring the diagram failed");
    }
    if (r == VD_EDEVICE) s->broken = true;
    if (r == VD_OK) apply_tuning(s);
    return r;
}

int vd_get_tuning_us(const vd_sim *s, float *us, int32_t cap)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (!us) return fail(VD_EINVAL, "us is NULL");
    int32_t n = (int32_t)(s->jfa_passes.size() + s->djfa_passes.size());
    if (cap < n) return fail(VD_EINVAL, "need room for %d passes, got %d", n, cap);
    const std::string arch = arch_name();
    std::lock_guard<std::mutex> lock(g_tune_mu);
    int32_t i = 0;
    for (int dyn = 0; dyn < 2; ++dyn)
        for (const Pass &p : dyn ? s->djfa_passes : s->jfa_passes) {
            auto it = g_tune_us.find(tune_key(arch, s->cfg, p, dyn != 0));
            us[i++] = it == g_tune_us.end() ? 0.f : it->second;
        }
    return VD_OK;
}

int vd_tuning_export(char *buf, size_t cap, size_t *needed)
{
    std::string text;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const auto &kv : g_tune) {
            char line[256];
            snprintf(line, sizeof line, "%s|%d|%d\n", kv.first.c_str(), kv.second.first,
                     kv.second.second);
            text += line;
        }
    }
    if (needed) *needed = text.size() + 1;
    if (!buf) return VD_OK;
    if (cap < text.size() + 1)
        return fail(VD_ENOMEM, "buffer of %zu bytes, the table needs %zu", cap, text.size() + 1);
    memcpy(buf, text.c_str(), text.size() + 1);
    return VD_OK;
}

int vd_tuning_import(const char *text)
{
    if (!text) return fail(VD_EINVAL, "text is NULL");
    std::map<std::string, std::pair<int32_t, int32_t>> add;
    const char *p = text;
    while (*p) {
        const char *end = strchr(p, '\n');
        std::string line = end ? std::string(p, end) : std::string(p);
        p = end ? end + 1 : p + line.size();
        if (line.empty()) continue;
        size_t a = line.find('|'), b = line.rfind('|');
        if (a == std::string::npos || a == b)
            return fail(VD_EINVAL, "malformed tuning line: %s", line.c_str());
        int32_t variant = atoi(line.substr(a + 1, b - a - 1).c_str());
        int32_t seg = atoi(line.substr(b + 1).c_str());
        if (variant < 0 || variant >= vd::kFloodVariants || seg < 0 || seg > vd::kMaxTunedSegRows)
            return fail(VD_EINVAL, "tuning values out of range: %s", line.c_str());
        add[line.substr(0, a)] = {variant, seg};
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto &kv : add) g_tune[kv.first] = kv.second;
    return VD_OK;
}

int vd_tuning_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    g_tune_us.clear();
    return VD_OK;
}

int vd_get_tuning(const vd_sim *s, int32_t *variants, int32_t *seg_rows, int32_t cap)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    int32_t n = (int32_t)(s->jfa_passes.size() + s->djfa_passes.size());
    if (cap < n) return fail(VD_EINVAL, "need room for %d passes, got %d", n, cap);
    int32_t i = 0;
    for (const std::vector<Pass> *ps : {&s->jfa_passes, &s->djfa_passes})
        for (const Pass &p : *ps) {
            if (variants) variants[i] = p.variant;
            if (seg_rows) seg_rows[i] = p.seg_rows;
            ++i;
        }
    return VD_OK;
}

void vd_config_default(vd_config *cfg)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof *cfg);
    cfg->disp_lo = -1;
    cfg->disp_hi = 1;
    cfg->label = VD_LABEL_ID32;
    cfg->metric = VD_EUCLID;
    cfg->vn_passes = 2;
    cfg->extra_passes = 0;
    cfg->dmax_override = 0;
    cfg->sim_seed = 1;
}

size_t vd_footprint_bytes(const vd_config *cfg)
{
    if (validate(cfg) != VD_OK) return 0;
    return footprint(cfg);
}

int vd_place_seeds(int32_t width, int32_t height, int32_t num_seeds, uint64_t seed,
                   int32_t *host_xy)
{
    if (!host_xy) return fail(VD_EINVAL, "host_xy is NULL");
    if (width < 1 || width > VD_MAX_SIDE || height < 1 || height > VD_MAX_SIDE)
        return fail(VD_EINVAL, "width and height must be in [1, %d], got %d x %d", VD_MAX_SIDE,
                    width, height);
    if (num_seeds < 1 || (int64_t)num_seeds > (int64_t)width * height)
        return fail(VD_EINVAL, "num_seeds must be in [1, width*height], got %d", num_seeds);
    std::vector<uint8_t> taken;
    try {
        taken.assign((size_t)width * (size_t)height, 0);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation of the %d x %d placement mask failed", width,
                    height);
    }
    // splitmix64: output n of the stream of `seed` is mix64(seed + (n + 1) * gamma);
    // pair j = (output 2j, output 2j + 1), each mapped onto [0, m) by
    // ((r >> 32) * m) >> 32; a pair whose pixel is taken is skipped.
    constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
    uint64_t n = 0;
    for (int32_t got = 0; got < num_seeds;) {
        const uint64_t rx = mix64(seed + (n + 1) * kGamma);
        const uint64_t ry = mix64(seed + (n + 2) * kGamma);
        n += 2;
        const int32_t x = (int32_t)(((rx >> 32) * (uint64_t)width) >> 32);
        const int32_t y = (int32_t)(((ry >> 32) * (uint64_t)height) >> 32);
        uint8_t &seen = taken[(size_t)y * (size_t)width + (size_t)x];
        if (seen) continue;
        seen = 1;
        host_xy[2 * (size_t)got] = x;
        host_xy[2 * (size_t)got + 1] = y;
        ++got;
    }
    return VD_OK;
}

int vd_init_sim(const vd_config *cfg, const int32_t *host_xy, void *dev_workspace,
                size_t ws_bytes, void *hip_stream, vd_sim **out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(VD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_workspace) return fail(VD_EINVAL, "dev_workspace is NULL");
    size_t need = footprint(cfg);
    if (ws_bytes < need)
        return fail(VD_ENOMEM, "workspace holds %zu bytes, the simulation needs %zu", ws_bytes,
                    need);
    const int32_t S = cfg->num_seeds;
    std::vector<int32_t> placed;   // positions drawn from sim_seed when the caller gives none
    if (!host_xy) {
        try {
            placed.resize(2 * (size_t)S);
        } catch (...) {
            return fail(VD_ENOMEM, "host allocation of %d seeds failed", S);
        }
        r = vd_place_seeds(cfg->width, cfg->height, S, cfg->sim_seed, placed.data());
        if (r) return r;
        host_xy = placed.data();
    }
    std::vector<uint32_t> packed;
    try {
        packed.resize((size_t)S + 1);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation of %d seeds failed", S);
    }
    for (int32_t i = 0; i < S; ++i) {
        int32_t x = host_xy[2 * i], y = host_xy[2 * i + 1];
        if (x < 0 || x >= cfg->width || y < 0 || y >= cfg->height)
            return fail(VD_EINVAL, "seed %d at (%d, %d) is outside the %d x %d grid", i, x, y,
                        cfg->width, cfg->height);
        packed[(size_t)i + 1] = vd::pack_pos(x, y);
    }
    packed[0] = 0;   // sentinel: the position (-kOff, -kOff), beyond every seed
    vd_sim *s = new (std::nothrow) vd_sim;
    if (!s) return fail(VD_ENOMEM, "host allocation of the handle failed");
    s->cfg = *cfg;
    s->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(VD_EDEVICE, "hipGetDevice failed");
    }
    size_t npix = (size_t)cfg->width * (size_t)cfg->height;
    uintptr_t base = ((uintptr_t)dev_workspace + kAlign - 1) / kAlign * kAlign;
    s->map[0] = (uint32_t *)base;
    base += align_up(npix * 4);
    s->map[1] = (uint32_t *)base;
    base += align_up(npix * 4);
    if (cfg->label == VD_LABEL_XY16) {
        s->idx = (uint32_t *)base;
        base += align_up(npix * 4);
    }
    s->pos = (uint32_t *)base;
    base += align_up((size_t)S * 4 + 4);
    if (cfg->label == VD_LABEL_XY16) {
        s->pos_map = (uint32_t *)base;
        base += align_up((size_t)S * 4 + 4);
    }
    s->disp = (uint32_t *)base;
    base += align_up(12);
    s->state = (uint8_t *)base;
    base += align_up((size_t)S);
    if (cfg->label == VD_LABEL_ID32) s->parked = (uint32_t *)base;
    try {
        s->host_state.assign((size_t)S, (uint8_t)(vd::kPresent | vd::kKept));
    } catch (...) {
        delete s;
        return fail(VD_ENOMEM, "host allocation of %d seeds failed", S);
    }
    s->present = S;
    s->measured = cfg->dmax_override == VD_DMAX_MEASURED;
    s->dmax = cfg->dmax_override > 0 ? cfg->dmax_override
                                     : (abs(cfg->disp_lo) > abs(cfg->disp_hi) ? abs(cfg->disp_lo)
                                                                              : abs(cfg->disp_hi));
    s->k1 = first_k(cfg->width, cfg->height);
    s->delta1 = first_delta(cfg->width, cfg->height, S, s->dmax);
    s->jfa_passes = schedule(s->k1, 0, cfg->extra_passes, 0);
    s->djfa_passes = schedule(s->delta1, cfg->vn_passes, cfg->extra_passes, 0);
    set_default_variants(s);
    s->move_seed = mix64(cfg->sim_seed ^ 0x6D6F7665ull);
    apply_tuning(s);
    hipError_t e = hipMemcpyAsync(s->pos, packed.data(), ((size_t)S + 1) * 4,
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->state, s->host_state.data(), (size_t)S, hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // packed is a local buffer
    if (e == hipSuccess) e = vd::launch_fill(s->disp, 3, 0u, s->stream);
    // the old-position index starts empty (see launch_index_marked)
    if (e == hipSuccess && s->idx)
        e = vd::launch_fill(s->idx, (int64_t)npix, 0xFFFFFFFFu, s->stream);
    if (e != hipSuccess) {
        delete s;
        return fail(VD_EDEVICE, "copying seed positions failed: %s", hipGetErrorString(e));
    }
    r = step(s, false);
    if (r) {
        vd_destroy(s);
        return r;
    }
    *out = s;
    return VD_OK;
}

int vd_move_seeds(vd_sim *s)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    s->t += 1;
    s->reach = std::min(s->reach + std::max(abs(s->cfg.disp_lo), abs(s->cfg.disp_hi)), 1 << 20);
    hipError_t e = vd::launch_move(s->pos, s->cfg.num_seeds, s->cfg.width, s->cfg.height,
                                   s->move_seed, s->t, s->cfg.disp_lo, s->cfg.disp_hi,
                                   seed_state(s), s->measured ? s->disp : nullptr, s->stream);
    if (e != hipSuccess) {
        s->broken = true;
        return fail(VD_EDEVICE, "move launch failed: %s", hipGetErrorString(e));
    }
    return VD_OK;
}

int vd_set_seeds(vd_sim *s, const int32_t *host_xy, size_t count)
{
    if (!s || !host_xy) return fail(VD_EINVAL, "NULL argument");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    const int32_t S = s->cfg.num_seeds;
    if (count != 2 * (size_t)S)
        return fail(VD_EINVAL, "count %zu != 2 * num_seeds %zu", count, 2 * (size_t)S);
    std::vector<uint32_t> packed;
    try {
        packed.resize((size_t)S);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation of %d seeds failed", S);
    }
    for (int32_t i = 0; i < S; ++i) {
        const int32_t x = host_xy[2 * i], y = host_xy[2 * i + 1];
        if (x < 0 || x >= s->cfg.width || y < 0 || y >= s->cfg.height)
            return fail(VD_EINVAL, "seed %d at (%d, %d) is outside the %d x %d grid", i, x, y,
                        s->cfg.width, s->cfg.height);
        packed[(size_t)i] = vd::pack_pos(x, y);
    }
    // staged in the idle ping-pong map (W*H >= S entries; no step is running)
    uint32_t *staged = s->map[s->cur ^ 1];
    hipError_t e = hipMemcpyAsync(staged, packed.data(), (size_t)S * 4, hipMemcpyHostToDevice,
                                  s->stream);
    if (e == hipSuccess)
        e = vd::launch_set_seeds(s->pos, staged, S, seed_state(s), s->parked,
                                 s->measured ? s->disp : nullptr, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // packed is a local buffer
    if (e != hipSuccess) {
        s->broken = true;
        return fail(VD_EDEVICE, "setting seed positions failed: %s", hipGetErrorString(e));
    }
    s->t += 1;
    s->reach = 1 << 20;   // any distance
    return VD_OK;
}

int vd_remove_seeds(vd_sim *s, const int32_t *host_ids, size_t n)
{
    if (!s || (!host_ids && n)) return fail(VD_EINVAL, "NULL argument");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    if (n == 0) return VD_OK;
    const int32_t S = s->cfg.num_seeds;
    if (n >= (size_t)s->present)
        return fail(VD_EINVAL, "removing %zu of %d present seeds leaves none", n, s->present);
    std::vector<uint8_t> next = s->host_state;
    for (size_t j = 0; j < n; ++j) {
        const int32_t i = host_ids[j];
        if (i < 0 || i >= S) return fail(VD_EINVAL, "seed index %d outside [0, %d)", i, S);
        if (!(next[(size_t)i] & vd::kPresent))
            return fail(VD_EINVAL, "seed %d is not present (or named twice)", i);
        next[(size_t)i] = (uint8_t)vd::kGone;
    }
    hipError_t e = hipSuccess;
    if (s->parked) {
        // the indices, staged in the idle ping-pong map (n < S <= width*height)
        uint32_t *staged = s->map[s->cur ^ 1];
        e = hipMemcpyAsync(staged, host_ids, n * 4, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = vd::launch_park(s->pos, s->parked, staged, (int32_t)n, s->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->state, next.data(), (size_t)S, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // next is a local buffer
    if (e != hipSuccess) {
        s->broken = true;
        return fail(VD_EDEVICE, "updating the seed set failed: %s", hipGetErrorString(e));
    }
    s->host_state.swap(next);
    s->present -= (int32_t)n;
    s->changed = s->removed = s->masked = true;
    replan_djfa(s);
    return VD_OK;
}

int vd_insert_seeds(vd_sim *s, const int32_t *host_xy, size_t n, int32_t *host_ids)
{
    if (!s || ((!host_xy || !host_ids) && n)) return fail(VD_EINVAL, "NULL argument");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    if (n == 0) return VD_OK;
    const vd_config &c = s->cfg;
    const int32_t S = c.num_seeds;
    if (n > (size_t)(S - s->present))
        return fail(VD_ESTATE, "%zu seeds to insert, %d free slots", n, S - s->present);
    for (size_t j = 0; j < n; ++j) {
        const int32_t x = host_xy[2 * j], y = host_xy[2 * j + 1];
        if (x < 0 || x >= c.width || y < 0 || y >= c.height)
            return fail(VD_EINVAL, "inserted seed %zu at (%d, %d) is outside the %d x %d grid", j,
                        x, y, c.width, c.height);
    }
    std::vector<uint8_t> next = s->host_state;
    std::vector<uint32_t> pairs;
    try {
        pairs.resize(2 * n);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation of %zu seeds failed", n);
    }
    // Free slots in ascending order, first those free since before the
    // diagram was made (no label of theirs is left in it), then those
    // removed since (their old labels must be purged at the next dJFA step).
    size_t j = 0;
    bool again = false;
    for (int pass = 0; pass < 2 && j < n; ++pass) {
        for (int32_t i = 0; i < S && j < n; ++i) {
            const uint8_t b = next[(size_t)i];
            if ((b & vd::kPresent) || ((b & vd::kGone) != 0) != (pass == 1)) continue;
            again = again || pass == 1;
            next[(size_t)i] = (uint8_t)vd::kPresent;   // not kept: no label of its own yet
            pairs[2 * j] = (uint32_t)i;
            pairs[2 * j + 1] = vd::pack_pos(host_xy[2 * j], host_xy[2 * j + 1]);
            ++j;
        }
    }
    // staged in the idle ping-pong map, at most width*height words at a time
    uint32_t *staged = s->map[s->cur ^ 1];
    const size_t chunk = std::max<size_t>(1, (size_t)c.width * c.height / 2);
    hipError_t e = hipSuccess;
    for (size_t at = 0; at < n && e == hipSuccess; at += chunk) {
        const size_t m = std::min(chunk, n - at);
        e = hipMemcpyAsync(staged, &pairs[2 * at], m * 8, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = vd::launch_place(s->pos, staged, (int32_t)m, s->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->state, next.data(), (size_t)S, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // local buffers
    if (e != hipSuccess) {
        s->broken = true;
        return fail(VD_EDEVICE, "inserting seeds failed: %s", hipGetErrorString(e));
    }
    for (size_t k = 0; k < n; ++k) host_ids[k] = (int32_t)pairs[2 * k];
    s->host_state.swap(next);
    s->present += (int32_t)n;
    s->changed = s->masked = true;
    s->reinserted = s->reinserted || again;
    replan_djfa(s);
    return VD_OK;
}

int vd_get_seed_set(const vd_sim *s, uint8_t *host_present, size_t count, int32_t *num_present,
                    int64_t *fallbacks)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (host_present) {
        if (count != (size_t)s->cfg.num_seeds)
            return fail(VD_EINVAL, "count %zu != num_seeds %d", count, s->cfg.num_seeds);
        for (size_t i = 0; i < count; ++i)
            host_present[i] = (s->host_state[i] & vd::kPresent) ? 1 : 0;
    }
    if (num_present) *num_present = s->present;
    if (fallbacks) *fallbacks = s->fallbacks;
    return VD_OK;
}

int vd_jfa_step(vd_sim *s) { return step(s, false); }

int vd_djfa_step(vd_sim *s) { return step(s, true); }

int vd_read_map(vd_sim *s, int32_t *host_dst, size_t count)
{
    if (!s || !host_dst) return fail(VD_EINVAL, "NULL argument");
    size_t npix = (size_t)s->cfg.width * s->cfg.height;
    if (count != npix) return fail(VD_EINVAL, "count %zu != width*height %zu", count, npix);
    // convert into the idle ping-pong buffer, then copy that
    VD_HIP(vd::launch_export(s->map[s->cur], s->map[s->cur ^ 1], (int64_t)npix, s->cfg.label,
                             s->stream));
    VD_HIP(hipMemcpyAsync(host_dst, s->map[s->cur ^ 1], npix * 4, hipMemcpyDeviceToHost,
                          s->stream));
    VD_HIP(hipStreamSynchronize(s->stream));
    return VD_OK;
}

int vd_read_seeds(vd_sim *s, int32_t *host_xy, size_t count)
{
    if (!s || !host_xy) return fail(VD_EINVAL, "NULL argument");
    size_t S = (size_t)s->cfg.num_seeds;
    if (count != 2 * S) return fail(VD_EINVAL, "count %zu != 2*S %zu", count, 2 * S);
    std::vector<uint32_t> packed;
    try {
        packed.resize(S);
    } catch (...) {
        return fail(VD_ENOMEM, "host allocation failed");
    }
    VD_HIP(hipMemcpyAsync(packed.data(), s->pos + 1, S * 4, hipMemcpyDeviceToHost, s->stream));
    if (s->parked && s->present < (int32_t)S) {
        // absent seeds (ID labels): their positions are parked
        std::vector<uint32_t> parked;
        try {
            parked.resize(S);
        } catch (...) {
            return fail(VD_ENOMEM, "host allocation failed");
        }
        VD_HIP(hipMemcpyAsync(parked.data(), s->parked, S * 4, hipMemcpyDeviceToHost, s->stream));
        VD_HIP(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < S; ++i)
            if (!(s->host_state[i] & vd::kPresent)) packed[i] = parked[i];
    }
    VD_HIP(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < S; ++i) {
        host_xy[2 * i] = (int32_t)(packed[i] & 0xFFFFu) - (int32_t)vd::kOff;
        host_xy[2 * i + 1] = (int32_t)(packed[i] >> 16) - (int32_t)vd::kOff;
    }
    return VD_OK;
}

int vd_map_device(vd_sim *s, const void **dev_map)
{
    if (!s || !dev_map) return fail(VD_EINVAL, "NULL argument");
    *dev_map = s->map[s->cur];
    return VD_OK;
}

int vd_get_info(const vd_sim *s, vd_sim_info *o)
{
    if (!s || !o) return fail(VD_EINVAL, "NULL argument");
    o->width = s->cfg.width;
    o->height = s->cfg.height;
    o->num_seeds = s->cfg.num_seeds;
    o->label = s->cfg.label;
    o->metric = s->cfg.metric;
    o->k1 = s->k1;
    o->delta1 = s->delta1;
    o->passes_jfa = (int32_t)s->jfa_passes.size();
    o->passes_djfa = (int32_t)s->djfa_passes.size();
    o->t = s->t;
    return VD_OK;
}

int vd_set_timing(vd_sim *s, int enable)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->used) {
        VD_HIP(hipStreamSynchronize(s->stream));
        s->used = 0;
    }
    s->timing = enable != 0;
    memset(&s->acc, 0, sizeof s->acc);
    return VD_OK;
}

int vd_get_timing(vd_sim *s, vd_timing *out)
{
    if (!s || !out) return fail(VD_EINVAL, "NULL argument");
    int r = harvest(s);
    if (r) return r;
    *out = s->acc;
    memset(&s->acc, 0, sizeof s->acc);
    return VD_OK;
}

void vd_destroy(vd_sim *s)
{
    if (!s) return;
    if (s->batch) {   // a batch member is released by vd_batch_destroy
        s->release = true;
        return;
    }
    (void)hipStreamSynchronize(s->stream);
    for (EventPair &p : s->pool) {
        if (p.a) (void)hipEventDestroy(p.a);
        if (p.b) (void)hipEventDestroy(p.b);
    }
    delete s;
}

int vd_set_flood_variant(vd_sim *s, int variant)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (variant < -1 || variant >= vd::kFloodVariants)
        return fail(VD_EINVAL, "variant must be -1 or in [0, %d), got %d", vd::kFloodVariants,
                    variant);
    s->forced_variant = variant < 0 ? -1 : variant;
    if (variant < 0) {
        set_default_variants(s);
        return VD_OK;
    }
    for (Pass &p : s->jfa_passes) p.variant = variant;
    for (Pass &p : s->djfa_passes) p.variant = variant;
    return VD_OK;
}

int vd_set_tail_fusion(vd_sim *s, int mode)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->batch) return fail(VD_ESTATE, "simulation is driven by a batch (vd_batch_step)");
    if (mode != -1 && mode != 0 && mode != 1 && mode != 16 && mode != 24 && mode != 32)
        return fail(VD_EINVAL, "mode must be -1, 0, 1, 16, 24 or 32, got %d", mode);
    s->forced_fuse = mode == 1 ? 16 : mode;
    for (int dyn = 0; dyn < 2; ++dyn)
        s->tail_th[dyn] = s->forced_fuse >= 0 ? s->forced_fuse : default_tail_th(s->cfg, dyn != 0);
    if (mode < 0) apply_tuning(s);
    return VD_OK;
}

int vd_get_tail_fusion(const vd_sim *s, int32_t *jfa, int32_t *djfa)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (jfa) *jfa = s->tail_th[0] ? (int32_t)vd::tail_len(s->jfa_passes) : 0;
    if (djfa) *djfa = s->tail_th[1] ? (int32_t)vd::tail_len(s->djfa_passes) : 0;
    return VD_OK;
}

const char *vd_last_error(void) { return vd::g_err; }

}  // extern "C"
