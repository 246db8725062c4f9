// vdflood runtime: simulation state, workspace carving, pass schedules,
// stream ordering, timing, and the C ABI of include/vdflood.h.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "vd_kernels.h"
#include "../../include/vdflood.h"

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

#define VD_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(VD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

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

struct Pass {
    int32_t k;
    int32_t vn;
    int32_t variant;   // flood kernel variant (same result, different speed)
};

// Measured on MI355X: ID labels run fastest with rows shared through LDS
// (fewer seed-table lookups), XY labels with the plain chain walk that
// requests rows two ahead.
int32_t default_variant(int32_t label) { return label == VD_LABEL_ID32 ? 3 : 1; }

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
        out.push_back({k, i < vn ? 1 : 0, variant});
    for (int32_t e = extra; e >= 1; --e) out.push_back({e, 0, variant});
    return out;
}

uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
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
    if (c->dmax_override > 2 * VD_MAX_SIDE)
        return fail(VD_EINVAL, "dmax_override too large: %d", c->dmax_override);
    return VD_OK;
}

size_t footprint(const vd_config *c)
{
    size_t npix = (size_t)c->width * (size_t)c->height;
    size_t seeds = (size_t)c->num_seeds * 4;
    size_t b = 2 * align_up(npix * 4) + align_up(seeds + 4);   // + the sentinel entry
    if (c->label == VD_LABEL_XY16) b += align_up(seeds + 4);
    return b + kAlign;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;   // 0: flood pass, 1: whole step
};

}  // namespace

struct vd_sim {
    vd_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint32_t *map[2] = {nullptr, nullptr};
    int cur = 0;                 // map[cur] holds the current diagram
    uint32_t *pos = nullptr;     // seed table: sentinel, then current positions
    uint32_t *pos_map = nullptr; // XY mode: the table the diagram's labels refer to
    int64_t t = 0;
    int32_t dmax = 0;
    int32_t k1 = 0, delta1 = 0;
    uint64_t move_seed = 0;
    std::vector<Pass> jfa_passes, djfa_passes;
    bool timing = false;
    std::vector<EventPair> pool;   // recorded pairs
    size_t used = 0;
    vd_timing acc{};
    bool broken = false;
};

namespace {

int record(vd_sim *s, int kind, bool begin, size_t *slot)
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
            s->acc.flood_launches += 1;
            s->acc.flood_ms += ms;
            s->acc.flood_pixels += (int64_t)s->cfg.width * s->cfg.height;
        } else {
            s->acc.step_count += 1;
            s->acc.step_ms += ms;
        }
    }
    s->used = 0;
    return VD_OK;
}

int run_passes(vd_sim *s, const std::vector<Pass> &passes)
{
    for (const Pass &p : passes) {
        size_t slot = 0;
        int r = record(s, 0, true, &slot);
        if (r) return r;
        VD_HIP(vd::launch_flood(s->map[s->cur], s->map[s->cur ^ 1], s->pos, s->cfg.num_seeds,
                                s->cfg.width, s->cfg.height, p.k, p.vn, s->cfg.label,
                                s->cfg.metric, p.variant, s->stream));
        r = record(s, 0, false, &slot);
        if (r) return r;
        s->cur ^= 1;
        if (s->timing && s->used >= 4096) {
            r = harvest(s);
            if (r) return r;
        }
    }
    return VD_OK;
}

int do_jfa(vd_sim *s)
{
    const vd_config &c = s->cfg;
    int64_t npix = (int64_t)c.width * c.height;
    VD_HIP(vd::launch_fill(s->map[s->cur], npix, vd::kEmpty, s->stream));
    if (c.label == VD_LABEL_XY16)
        VD_HIP(vd::launch_splat_xy(s->map[s->cur], s->pos, c.num_seeds, c.width, s->stream));
    else
        VD_HIP(vd::launch_splat_id(s->map[s->cur], s->pos, c.num_seeds, c.width, s->stream));
    int r = run_passes(s, s->jfa_passes);
    if (r) return r;
    if (c.label == VD_LABEL_XY16)
        VD_HIP(hipMemcpyAsync(s->pos_map, s->pos, ((size_t)c.num_seeds + 1) * 4,
                              hipMemcpyDeviceToDevice, s->stream));
    return VD_OK;
}

int do_djfa(vd_sim *s)
{
    const vd_config &c = s->cfg;
    uint32_t *cur = s->map[s->cur];
    if (c.label == VD_LABEL_XY16) {
        // The idle ping-pong buffer serves as the old-position index; the
        // first flood pass overwrites it.
        uint32_t *idx = s->map[s->cur ^ 1];
        VD_HIP(vd::launch_index_old(idx, s->pos_map, c.num_seeds, c.width, s->stream));
        VD_HIP(vd::launch_relabel(cur, idx, s->pos, c.num_seeds, c.width, c.height, s->stream));
        VD_HIP(vd::launch_splat_xy(cur, s->pos, c.num_seeds, c.width, s->stream));
    } else {
        VD_HIP(vd::launch_splat_id(cur, s->pos, c.num_seeds, c.width, s->stream));
    }
    int r = run_passes(s, s->djfa_passes);
    if (r) return r;
    if (c.label == VD_LABEL_XY16)
        VD_HIP(hipMemcpyAsync(s->pos_map, s->pos, ((size_t)c.num_seeds + 1) * 4,
                              hipMemcpyDeviceToDevice, s->stream));
    return VD_OK;
}

int step(vd_sim *s, bool dynamic)
{
    if (!s) return fail(VD_EINVAL, "sim is NULL");
    if (s->broken) return fail(VD_ESTATE, "simulation unusable after an earlier device error");
    size_t slot = 0;
    int r = record(s, 1, true, &slot);
    if (r) return r;
    r = dynamic ? do_djfa(s) : do_jfa(s);
    if (r == VD_OK) r = record(s, 1, false, &slot);
    if (r == VD_EDEVICE) s->broken = true;
    return r;
}

}  // namespace

extern "C" {

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

int vd_init_sim(const vd_config *cfg, const int32_t *host_xy, void *dev_workspace,
                size_t ws_bytes, void *hip_stream, vd_sim **out)
{
    int r = validate(cfg);
    if (r) return r;
    if (!out) return fail(VD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!host_xy) return fail(VD_EINVAL, "host_xy is NULL");
    if (!dev_workspace) return fail(VD_EINVAL, "dev_workspace is NULL");
    size_t need = footprint(cfg);
    if (ws_bytes < need)
        return fail(VD_ENOMEM, "workspace holds %zu bytes, the simulation needs %zu", ws_bytes,
                    need);
    const int32_t S = cfg->num_seeds;
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
    s->pos = (uint32_t *)base;
    base += align_up((size_t)S * 4 + 4);
    if (cfg->label == VD_LABEL_XY16) s->pos_map = (uint32_t *)base;
    s->dmax = cfg->dmax_override > 0 ? cfg->dmax_override
                                     : (abs(cfg->disp_lo) > abs(cfg->disp_hi) ? abs(cfg->disp_lo)
                                                                              : abs(cfg->disp_hi));
    s->k1 = first_k(cfg->width, cfg->height);
    s->delta1 = first_delta(cfg->width, cfg->height, S, s->dmax);
    s->jfa_passes = schedule(s->k1, 0, cfg->extra_passes, default_variant(cfg->label));
    s->djfa_passes = schedule(s->delta1, cfg->vn_passes, cfg->extra_passes,
                              default_variant(cfg->label));
    s->move_seed = mix64(cfg->sim_seed ^ 0x6D6F7665ull);
    hipError_t e = hipMemcpyAsync(s->pos, packed.data(), ((size_t)S + 1) * 4,
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);   // packed is a local buffer
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
    s->t += 1;
    hipError_t e = vd::launch_move(s->pos, s->cfg.num_seeds, s->cfg.width, s->cfg.height,
                                   s->move_seed, s->t, s->cfg.disp_lo, s->cfg.disp_hi, s->stream);
    if (e != hipSuccess) {
        s->broken = true;
        return fail(VD_EDEVICE, "move launch failed: %s", hipGetErrorString(e));
    }
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
    int32_t v = variant < 0 ? default_variant(s->cfg.label) : variant;
    for (Pass &p : s->jfa_passes) p.variant = v;
    for (Pass &p : s->djfa_passes) p.variant = v;
    return VD_OK;
}

const char *vd_last_error(void) { return g_err; }

}  // extern "C"
