// Allocation-free JFA diagram: vd_jfa_noalloc of include/vdflood.h.  The
// same computation as a simulation's VD_0 (a JFA step from scratch: fill,
// splat, passes k = k1 .. 1 plus the extra passes), with the scratch that a
// simulation keeps in its workspace -- the seed table, the seed state bytes
// and the second ping-pong map -- in a fixed device array.  Nothing here
// allocates, on the device or the host.
#include <mutex>

#include "vd_sim.h"

using vd::fail;

namespace {

constexpr size_t kScratchBytes = VD_NOALLOC_SCRATCH_BYTES;

// One array per GPU, alive from the code object's load until the process
// ends.  Host code never names it as an address: the device address comes
// from hipGetSymbolAddress, once per device.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
uint8_t *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The scratch array's address on the current device (dev), resolved on the
// first call there.
int scratch_on(int dev, uint8_t **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VD_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                        hipGetErrorString(e));
        g_scratch[dev] = (uint8_t *)p;
    }
    *out = g_scratch[dev];
    return VD_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

extern "C" int vd_jfa_noalloc(const vd_config *cfg, const int32_t *dev_xy, int32_t *dev_map,
                              void *hip_stream)
{
    int r = vd::validate(cfg);
    if (r) return r;
    if (!dev_xy || !dev_map) return fail(VD_EINVAL, "dev_xy and dev_map must not be NULL");
    const int32_t W = cfg->width, H = cfg->height, S = cfg->num_seeds;
    const size_t npix = (size_t)W * (size_t)H;
    const size_t tab_bytes = align256(((size_t)S + 1) * 4), state_bytes = align256((size_t)S);
    const size_t need = tab_bytes + state_bytes + align256(npix * 4);
    if (need > kScratchBytes)
        return fail(VD_EINVAL,
                    "a %d x %d map with %d seeds needs %zu bytes of scratch; the fixed array "
                    "holds %zu (VD_NOALLOC_SCRATCH_BYTES)",
                    W, H, S, need, kScratchBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(VD_EDEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(VD_EDEVICE, "device %d is beyond the %d this library tracks", dev, kMaxDevices);
    uint8_t *base = nullptr;
    r = scratch_on(dev, &base);
    if (r) return r;
    uint32_t *table = (uint32_t *)base;
    uint8_t *state = base + tab_bytes;
    uint32_t *partner = (uint32_t *)(base + tab_bytes + state_bytes);
    hipStream_t st = (hipStream_t)hip_stream;

    // The pass list of a JFA step (Eq. (2), Moore throughout; extra passes
    // k = 1, or k = 2 then 1) and its fused tail, as a simulation builds them.
    int32_t ks[32];
    int32_t n = 0;
    for (int32_t k = vd::first_k(W, H); k >= 1; k >>= 1) ks[n++] = k;
    for (int32_t e = cfg->extra_passes; e >= 1; --e) ks[n++] = e;
    int32_t m = 0;
    const int32_t th = vd::default_tail_th(*cfg, false);
    if (th) {
        int32_t sum = 0;
        while (m < n && m < vd::kTailMaxPasses) {
            const int32_t k = ks[n - 1 - m];
            if ((k != 1 && k != 2 && k != 4) || sum + k > vd::kTailHalo) break;
            sum += k;
            ++m;
        }
        if (m < 2) m = 0;
    }
    const int32_t launches = (n - m) + (m ? 1 : 0);
    // The passes alternate between the caller's map and the partner; start
    // where the last one lands in the partner, which is then converted into
    // the caller's map.
    uint32_t *maps[2] = {partner, (uint32_t *)dev_map};
    int cur = launches % 2 == 0 ? 0 : 1;

#define VD_NA_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(VD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

    VD_NA_HIP(vd::launch_pack_positions(table, state, dev_xy, S, W, H, st));
    if (cfg->label == VD_LABEL_XY16) {
        VD_NA_HIP(vd::launch_fill(maps[cur], (int64_t)npix, vd::kEmpty, st));
        VD_NA_HIP(vd::launch_splat_xy(maps[cur], table, S, W, state, st));
    } else {
        VD_NA_HIP(vd::launch_fill(maps[cur], (int64_t)npix, 0xFFFFFFFFu, st));
        VD_NA_HIP(vd::launch_splat_id_over_ones(maps[cur], table, S, W, state, st));
    }
    for (int32_t i = 0; i < n - m; ++i) {
        VD_NA_HIP(vd::launch_flood(maps[cur], maps[cur ^ 1], table, S, W, H, ks[i], 0,
                                   cfg->label, cfg->metric,
                                   vd::default_variant(*cfg, false, ks[i]), 0, st));
        cur ^= 1;
    }
    if (m) {
        int32_t vns[vd::kTailMaxPasses] = {0, 0, 0, 0};
        const bool nt = vd::default_variant(*cfg, false, ks[n - 1]) >= vd::kFloodVariants / 2;
        VD_NA_HIP(vd::launch_flood_tail(maps[cur], maps[cur ^ 1], table, S, W, H, &ks[n - m], vns,
                                        m, cfg->label, cfg->metric, nt, th, st));
        cur ^= 1;
    }
    // cur == 0 here: the diagram is in the partner
    VD_NA_HIP(vd::launch_export(maps[cur], (uint32_t *)dev_map, (int64_t)npix, cfg->label, st));
#undef VD_NA_HIP
    return VD_OK;
}
