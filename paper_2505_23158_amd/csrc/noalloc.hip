// lodge_render_static: lodge_render with the caller's workspace replaced by a
// scratch array the library holds in device memory, for callers that cannot
// allocate (code under HIP graph capture, serving loops that must not
// allocate, harnesses that forbid hipMalloc).  The kernels are lodge_render's;
// only where their scratch lives differs.
//
// `scratch` is a file-scope device array of LODGE_STATIC_SCRATCH_BYTES.  Each
// GPU holds its own copy, at its own address, from the moment this code
// object is loaded on it until the process ends.  In host code the array's
// name is only a host-side stand-in, so the device address of each GPU's copy
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and kept; every kernel argument derived from the scratch comes
// from that address.
//
// The workspace laid out in the scratch is sized per call from the image size
// and the selection's capacity (the instance capacity takes what remains), so
// successive calls may use different layouts: every region a frame reads is
// written or cleared by that frame's own kernels (counters by the setup
// kernel, tile totals by the chunk scan, the rest before use), and the
// overflow flags are cleared at the start of each call.  Calls that overlap on
// one GPU (different streams, or host threads) share the array and race.
#include <mutex>
#include <vector>

#include "lodge_internal.hpp"

namespace lodge {

namespace {

static __device__ __align__(256) unsigned char scratch[LODGE_STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // per device: the device address of its copy (null until looked up)

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device.
lodge_status scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "lodge_render_static: hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "lodge_render_static: hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0)
            return fail(LODGE_ERR_HIP, "lodge_render_static: the scratch array has no 256-byte aligned address");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return LODGE_OK;
}

// Overflow report of the call: bit 0 the selection's count exceeded its
// capacity, bit 1 the instances exceeded the scratch's instance capacity.
__global__ void k_report_overflow(const FrameInfo* info, const uint32_t* count, uint32_t cap, uint32_t* out)
{
    if (threadIdx.x == 0) *out = (info->overflow & kOvfInstances) | (*count > cap ? kOvfSelect : 0u);
}

}  // namespace

}  // namespace lodge

using namespace lodge;

extern "C" lodge_status lodge_render_static(const lodge_scene* scene, const lodge_selection* sel,
                                            const lodge_camera* cam, const lodge_render_opts* opts, float* image,
                                            float* final_T, uint32_t* n_contrib, uint32_t* overflow, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    if (!cam) return fail(LODGE_ERR_INVALID_ARG, "lodge_render_static needs a camera");
    lodge_status s;
    if ((s = check_cam(cam, nullptr)) != LODGE_OK) return s;
    if (cam->width <= 0 || cam->height <= 0 || cam->width > 16384 || cam->height > 16384)
        return fail(LODGE_ERR_INVALID_ARG, "image size out of range");
    if (tiles_of(cam->width, cam->height) > (uint64_t)kMaxTiles)
        return fail(LODGE_ERR_UNSUPPORTED, "image has more than 32768 16x16 tiles");
    if (!sel || !sel->ids || !sel->w || !sel->count) return fail(LODGE_ERR_INVALID_ARG, "selection buffers are NULL");
    if (sel->cap >= (1u << 31)) return fail(LODGE_ERR_INVALID_ARG, "selection cap must be < 2^31");
    if (!image || !final_T || !n_contrib) return fail(LODGE_ERR_INVALID_ARG, "output buffers are NULL");
    lodge_render_opts o;
    if ((s = check_render_opts(opts, &o)) != LODGE_OK) return s;

    // the largest instance capacity whose layout fits the scratch (the layout grows with it)
    const size_t kBytes = LODGE_STATIC_SCRATCH_BYTES;
    const size_t base_need = make_layout(0, cam->width, cam->height, sel->cap, 1).total;
    if (base_need > kBytes) {
        char buf[224];
        snprintf(buf, sizeof buf,
                 "lodge_render_static: a %dx%d frame with selection capacity %u needs %zu bytes of scratch before any "
                 "instance; the static scratch holds %zu",
                 cam->width, cam->height, sel->cap, base_need, kBytes);
        return fail(LODGE_ERR_INVALID_ARG, buf);
    }
    uint64_t lo = 1, hi = (1ull << 32) - 1;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (make_layout(0, cam->width, cam->height, sel->cap, mid).total <= kBytes) lo = mid;
        else hi = mid - 1;
    }
    void* base = nullptr;
    if ((s = scratch_address(&base)) != LODGE_OK) return s;
    lodge_workspace ws{base, kBytes, cam->width, cam->height, sel->cap, lo};
    const Views v = views_of(&ws, 0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((s = render_stages(scene, *sel, cam, o, v, false, image, final_T, n_contrib, st)) != LODGE_OK) return s;
    if (overflow) {
        k_report_overflow<<<1, 64, 0, st>>>(v.info, sel->count, sel->cap, overflow);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "lodge_render_static: overflow report");
    }
    return LODGE_OK;
}
