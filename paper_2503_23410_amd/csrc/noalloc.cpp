// Allocation-free variant of the binocular reprojection entry point: its
// workspace (left hit points, right texel keys, hole list and count) lives
// in a static device array instead of caller memory, for callers that cannot
// allocate device memory (HIP graph capture, tight serving loops).
#include <mutex>

#include "vafr_internal.h"

namespace {

// Workspace of vafr_shade_lp_rep for layouts of up to
// (kScratchBytes - 16) / 28 = 1,198,372 texels (the paper's acuity layout has
// 1,063,314).  Every GPU the library runs on holds one copy until the
// process ends.  Host code never uses this name as an address: the per-device
// address comes from hipGetSymbolAddress.
constexpr int64_t kScratchBytes = (int64_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
int scratch_on_current_device(void** out) {
    int dev = -1;
    VAFR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return vafr::fail(VAFR_E_UNSUPPORTED, "device %d: too many devices", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return vafr::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return vafr::fail(VAFR_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return VAFR_OK;
}

}  // namespace

using namespace vafr;

extern "C" int vafr_shade_lp_rep_noalloc(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right,
                                         vafr_gaze gaze, const vafr_shading* sh, vafr_layout L, float* lp_left,
                                         float* lp_right, int32_t* hit_left, int32_t* hit_right, hipStream_t stream) {
    int64_t need;
    if (int rc = vafr_rep_workspace_bytes(L, &need)) return rc;
    if (need > kScratchBytes)
        return fail(VAFR_E_BUDGET, "layout of %lld texels needs a %lld-byte workspace; the static one holds %lld",
                    (long long)L->n_texels, (long long)need, (long long)kScratchBytes);
    bool resident = false;
    if (int rc = layout_resident(L, &resident)) return rc;
    if (!resident)
        return fail(VAFR_E_UNSUPPORTED,
                    "layout tables are not on this device yet (any per-frame call with the layout uploads them)");
    void* ws = nullptr;
    if (int rc = scratch_on_current_device(&ws)) return rc;
    return shade_lp_rep_ws(scene, cam_left, cam_right, gaze, sh, L, lp_left, lp_right, hit_left, hit_right, ws,
                           kScratchBytes, stream, nullptr);
}
