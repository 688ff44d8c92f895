// Host side of the C ABI declared in include/lodge.h: argument validation,
// the workspace layout, and the per-frame launch sequences.  No call here
// allocates device memory or synchronises the host except lodge_check and
// lodge_frame_info_read, which say so.
#include <string.h>

#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "lodge_internal.hpp"

namespace lodge {

namespace {
thread_local std::string g_last_error;
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

lodge_status fail(lodge_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

lodge_status hip_fail(hipError_t e, const char* where)
{
    return fail(LODGE_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

uint64_t tiles_of(int32_t w, int32_t h) { return (uint64_t)((w + kTile - 1) / kTile) * (uint64_t)((h + kTile - 1) / kTile); }

lodge_status check_cam(const lodge_camera* c, const lodge_workspace* ws)
{
    if (!c) return LODGE_OK;   // the camera already set on the workspace
    if (ws && (c->width != ws->width || c->height != ws->height))
        return fail(LODGE_ERR_INVALID_ARG, "camera size differs from the workspace's");
    const float v[] = {c->fx, c->fy, c->cx, c->cy, c->znear, c->lim_x, c->lim_y};
    for (float x : v)
        if (!std::isfinite(x)) return fail(LODGE_ERR_INVALID_ARG, "camera has a non-finite intrinsic");
    if (!(c->fx > 0) || !(c->fy > 0) || !(c->znear > 0) || !(c->lim_x > 0) || !(c->lim_y > 0))
        return fail(LODGE_ERR_INVALID_ARG, "camera focal lengths, znear and limits must be > 0");
    return LODGE_OK;
}

lodge_status check_render_opts(const lodge_render_opts* opts, lodge_render_opts* o)
{
    *o = lodge_render_opts{0.3f, 1, nullptr};
    if (opts) *o = *opts;
    if (!(o->s2d >= 0.0f) || !std::isfinite(o->s2d)) return fail(LODGE_ERR_INVALID_ARG, "s2d must be finite and >= 0");
    return LODGE_OK;
}

// The stages of lodge_render on the views of a workspace: setup (camera,
// options, counters), projection, binning, sort, compositing.
lodge_status render_stages(const lodge_scene* scene, const lodge_selection& sel, const lodge_camera* cam,
                           const lodge_render_opts& o, const Views& v, bool keep_select_flag, float* image,
                           float* final_T, uint32_t* n_contrib, hipStream_t st, float* score)
{
    hipError_t e = hipSuccess;
    auto mark = [&](int k) -> hipError_t {
        return o.stage_events ? hipEventRecord(static_cast<hipEvent_t>(o.stage_events[k]), st) : hipSuccess;
    };
    if ((e = launch_render_setup(o, cam, v, keep_select_flag, st)) != hipSuccess)
        return hip_fail(e, "lodge_render: setup");
    if ((e = mark(0)) != hipSuccess) return hip_fail(e, "lodge_render: event");
    if ((e = launch_project(scene->levels, sel, v, st)) != hipSuccess) return hip_fail(e, "lodge_render: project");
    if ((e = mark(1)) != hipSuccess) return hip_fail(e, "lodge_render: event");
    if ((e = launch_bin(v, sel, st)) != hipSuccess) return hip_fail(e, "lodge_render: bin");
    if ((e = mark(2)) != hipSuccess) return hip_fail(e, "lodge_render: event");
    if ((e = launch_sort(v, st)) != hipSuccess) return hip_fail(e, "lodge_render: sort");
    if ((e = mark(3)) != hipSuccess) return hip_fail(e, "lodge_render: event");
    if (score) {
        if ((e = launch_importance(v, sel.ids, score, st)) != hipSuccess) return hip_fail(e, "lodge_importance");
    } else if ((e = launch_composite(v, image, final_T, n_contrib, st)) != hipSuccess) {
        return hip_fail(e, "lodge_render: composite");
    }
    if ((e = mark(4)) != hipSuccess) return hip_fail(e, "lodge_render: event");
    return LODGE_OK;
}

namespace {

lodge_status check_ws(const lodge_scene* s, const lodge_workspace* ws)
{
    if (!ws || !ws->base) return fail(LODGE_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws->base & 255) != 0) return fail(LODGE_ERR_INVALID_ARG, "workspace base not 256-byte aligned");
    if (ws->width <= 0 || ws->height <= 0 || ws->width > 16384 || ws->height > 16384)
        return fail(LODGE_ERR_INVALID_ARG, "workspace image size out of range");
    if (ws->max_instances >= (1ull << 32)) return fail(LODGE_ERR_INVALID_ARG, "max_instances must be < 2^32");
    if (ws->max_active >= (1u << 31)) return fail(LODGE_ERR_INVALID_ARG, "max_active must be < 2^31");
    if (tiles_of(ws->width, ws->height) > (uint64_t)kMaxTiles)
        return fail(LODGE_ERR_UNSUPPORTED, "image has more than 32768 16x16 tiles");
    const Layout L = make_layout(s->levels.total, ws->width, ws->height, ws->max_active, ws->max_instances);
    if (ws->bytes < L.total) return fail(LODGE_ERR_INVALID_ARG, "workspace smaller than lodge_workspace_size()");
    return LODGE_OK;
}

lodge_status check_sel(const lodge_selection* sel, const lodge_workspace* ws)
{
    if (!sel || !sel->ids || !sel->w || !sel->count) return fail(LODGE_ERR_INVALID_ARG, "selection buffers are NULL");
    if (sel->cap != ws->max_active) return fail(LODGE_ERR_INVALID_ARG, "selection cap != workspace max_active");
    return LODGE_OK;
}

}  // namespace

Layout make_layout(uint32_t n_total, int32_t width, int32_t height, uint32_t max_active, uint64_t max_instances)
{
    Layout L{};
    L.TX = (uint32_t)(width + kTile - 1) / kTile;
    L.TY = (uint32_t)(height + kTile - 1) / kTile;
    L.T = L.TX * L.TY;
    // selection blocks never straddle levels: at most one partial block per level
    L.sel_tiles = (n_total + kSelTile - 1) / kSelTile + LODGE_MAX_LEVELS;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += al(bytes); return o; };
    L.params = take(sizeof(FrameParams));
    L.info = take(sizeof(FrameInfo));
    L.wstats = take(16ull * 4 * L.T);
    L.chunk_sum = take(4ull * ((max_active + kProjChunk - 1) / kProjChunk + 1));
    L.chunk_vis = take(4ull * ((max_active + kProjChunk - 1) / kProjChunk + 1));
    L.scan_blk = take(16ull * (((max_active + kProjChunk - 1) / kProjChunk + kScanChunks - 1) / kScanChunks + 1));
    L.bin_blocks = (uint32_t)std::max<uint64_t>(1, (max_instances + kBinChunk - 1) / kBinChunk);
    L.bstart = take(4ull * (L.bin_blocks + 1));
    L.proj = take(48ull * max_active);
    L.depth = take(4ull * max_active);
    L.rect = take(8ull * max_active);
    L.vtiles = take(4ull * max_active + 16);
    L.vis_off = take(4ull * max_active + 16);
    L.vis_id = take(4ull * max_active + 16);
    L.inst = take(8ull * max_instances);
    L.hist = take(4ull * L.T * L.bin_blocks);
    L.tcount = take(4ull * L.T);
    L.ranges = take(8ull * L.T);
    L.order = take(4ull * L.T);
    L.large = take(12ull * L.T);
    L.sorted = take(4ull * max_instances);
    L.temp = take(8ull * max_instances);
    L.g2d = take(48ull * max_active);
    // last: the only regions whose size depends on the scene
    L.sel_cnt = take(4ull * L.sel_tiles);
    L.sel_off = take(4ull * L.sel_tiles);
    L.sel_bits = take(4ull * kSelBlock * L.sel_tiles);
    L.total = off;
    return L;
}

Views views_of(const lodge_workspace* ws, uint32_t n_total)
{
    Views v{};
    v.lay = make_layout(n_total, ws->width, ws->height, ws->max_active, ws->max_instances);
    char* b = static_cast<char*>(ws->base);
    v.params = reinterpret_cast<FrameParams*>(b + v.lay.params);
    v.info = reinterpret_cast<FrameInfo*>(b + v.lay.info);
    v.wstats = reinterpret_cast<uint4*>(b + v.lay.wstats);
    v.sel_cnt = reinterpret_cast<uint32_t*>(b + v.lay.sel_cnt);
    v.sel_off = reinterpret_cast<uint32_t*>(b + v.lay.sel_off);
    v.sel_bits = reinterpret_cast<uint32_t*>(b + v.lay.sel_bits);
    v.chunk_sum = reinterpret_cast<uint32_t*>(b + v.lay.chunk_sum);
    v.chunk_vis = reinterpret_cast<uint32_t*>(b + v.lay.chunk_vis);
    v.scan_blk = reinterpret_cast<uint4*>(b + v.lay.scan_blk);
    v.proj = reinterpret_cast<float4*>(b + v.lay.proj);
    v.depth = reinterpret_cast<float*>(b + v.lay.depth);
    v.rect = reinterpret_cast<uint2*>(b + v.lay.rect);
    v.vtiles = reinterpret_cast<uint32_t*>(b + v.lay.vtiles);
    v.vis_off = reinterpret_cast<uint32_t*>(b + v.lay.vis_off);
    v.vis_id = reinterpret_cast<uint32_t*>(b + v.lay.vis_id);
    v.bstart = reinterpret_cast<uint32_t*>(b + v.lay.bstart);
    v.inst = reinterpret_cast<uint2*>(b + v.lay.inst);
    v.hist = reinterpret_cast<uint32_t*>(b + v.lay.hist);
    v.tcount = reinterpret_cast<uint32_t*>(b + v.lay.tcount);
    v.ranges = reinterpret_cast<uint2*>(b + v.lay.ranges);
    v.order = reinterpret_cast<uint32_t*>(b + v.lay.order);
    v.large = reinterpret_cast<uint32_t*>(b + v.lay.large);
    v.sorted = reinterpret_cast<uint32_t*>(b + v.lay.sorted);
    v.temp = reinterpret_cast<unsigned long long*>(b + v.lay.temp);
    v.g2d = reinterpret_cast<float*>(b + v.lay.g2d);
    v.max_active = ws->max_active;
    v.max_instances = ws->max_instances;
    return v;
}

// Clears the render counters and records the options; a small kernel so a
// captured graph holds no memset.
namespace {
__global__ void k_render_setup(FrameParams* fp, FrameInfo* info, lodge_camera cam, int32_t has_cam, float s2d,
                               int32_t compensate, int32_t TX, int32_t TY, uint32_t keep_flags)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (has_cam) store_camera(&fp->cam, cam);
        fp->s2d = s2d;
        fp->compensate = compensate;
        fp->TX = TX;
        fp->TY = TY;
        info->n_front = 0;
        info->n_visible = 0;
        info->n_instances = 0;
        info->max_tile_len = 0;
        info->overflow &= keep_flags;
        info->n_large = 0;
        info->n_huge = 0;
        info->n_mid = 0;
        info->n_xl = 0;
        info->n_binned = 0;
        info->sort_next = 0;
        info->scan_done = 0;
    }
}
}  // namespace

namespace {
// The camera travels as a kernel argument: the copy is taken at launch, so
// the caller's struct can change right after the call returns.
__global__ void k_set_camera(lodge_camera cam, lodge_camera* dst)
{
    if (threadIdx.x == 0) store_camera(dst, cam);
}
}  // namespace

hipError_t launch_set_camera(const lodge_camera& cam, const Views& v, hipStream_t st)
{
    k_set_camera<<<1, 64, 0, st>>>(cam, &v.params->cam);
    return hipGetLastError();
}

hipError_t launch_render_setup(const lodge_render_opts& o, const lodge_camera* cam, const Views& v,
                               bool keep_select_flag, hipStream_t st)
{
    lodge_camera c{};
    if (cam) c = *cam;
    k_render_setup<<<1, 64, 0, st>>>(v.params, v.info, c, cam ? 1 : 0, o.s2d, o.compensate, (int32_t)v.lay.TX,
                                     (int32_t)v.lay.TY, keep_select_flag ? kOvfSelect : 0u);
    return hipGetLastError();
}

}  // namespace lodge

using namespace lodge;

extern "C" {

const char* lodge_status_string(lodge_status s)
{
    switch (s) {
    case LODGE_OK: return "ok";
    case LODGE_ERR_INVALID_ARG: return "invalid argument";
    case LODGE_ERR_CAPACITY: return "capacity exceeded";
    case LODGE_ERR_HIP: return "HIP runtime error";
    case LODGE_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* lodge_last_error(void) { return g_last_error.c_str(); }

const char* lodge_version(void) { return "lodge-gfx950 0.1"; }

lodge_status lodge_scene_create(const lodge_level* levels, int32_t L, const float* d, const lodge_chunks* chunks,
                                lodge_scene** out)
{
    if (!out) return fail(LODGE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!levels || L < 1 || L > LODGE_MAX_LEVELS) return fail(LODGE_ERR_INVALID_ARG, "need 1..8 levels");
    if (L > 1 && !d) return fail(LODGE_ERR_INVALID_ARG, "switch distances are NULL");
    lodge_scene* s = new lodge_scene();
    memset(s, 0, sizeof(*s));
    uint64_t total = 0;
    for (int l = 0; l < L; l++) {
        const lodge_level& v = levels[l];
        if (v.n < 0) { delete s; return fail(LODGE_ERR_INVALID_ARG, "negative level size"); }
        if (v.n >= (int64_t)1 << 30) {
            delete s;
            return fail(LODGE_ERR_UNSUPPORTED, "a level holds 2^30 or more Gaussians (planes are addressed with 32-bit "
                                               "byte offsets)");
        }
        if (v.sh_degree < 0 || v.sh_degree > 3) { delete s; return fail(LODGE_ERR_INVALID_ARG, "sh_degree must be 0..3"); }
        if (!(v.filter3d_var >= 0.0f) || !std::isfinite(v.filter3d_var)) {
            delete s;
            return fail(LODGE_ERR_INVALID_ARG, "filter3d_var must be finite and >= 0");
        }
        if (v.n > 0 && (!v.mean || !v.scale || !v.quat || !v.opacity || !v.sh)) {
            delete s;
            return fail(LODGE_ERR_INVALID_ARG, "level has a NULL parameter plane");
        }
        LevelDev& dv = s->levels.lv[l];
        dv.mean = v.mean; dv.scale = v.scale; dv.quat = v.quat; dv.opacity = v.opacity; dv.sh = v.sh;
        dv.n = (uint32_t)v.n;
        dv.base = (uint32_t)total;
        dv.sh_degree = v.sh_degree;
        dv.var = v.filter3d_var;
        total += (uint64_t)v.n;
        if (total >= (1ull << 32)) { delete s; return fail(LODGE_ERR_INVALID_ARG, "more than 2^32 - 1 Gaussians"); }
    }
    // unused level slots never match: base beyond every id
    for (int l = L; l < LODGE_MAX_LEVELS; l++) s->levels.lv[l].base = 0xffffffffu;
    for (int l = 0; l + 1 < L; l++) {
        if (!(d[l] > 0.0f) || !std::isfinite(d[l]) || (l > 0 && !(d[l] > d[l - 1]))) {
            delete s;
            return fail(LODGE_ERR_INVALID_ARG, "switch distances must be finite, > 0 and strictly increasing");
        }
        s->levels.d[l] = d[l];
    }
    s->levels.L = L;
    s->levels.total = (uint32_t)total;
    uint32_t blk = 0;
    for (int l = 0; l < L; l++) {
        s->levels.first_block[l] = blk;
        blk += (uint32_t)((levels[l].n + kSelTile - 1) / kSelTile);
    }
    for (int l = L; l <= LODGE_MAX_LEVELS; l++) s->levels.first_block[l] = blk;
    s->levels.sel_blocks = blk;
    if (chunks) {
        if (chunks->k < 1 || chunks->k > LODGE_MAX_CHUNKS || !chunks->center || !chunks->offset) {
            delete s;
            return fail(LODGE_ERR_INVALID_ARG, "chunks: need 1..128 centres and offsets");
        }
        if (!std::isfinite(chunks->band)) {
            delete s;
            return fail(LODGE_ERR_INVALID_ARG, "chunk blend band must be finite");
        }
        // Eq. 4 divides by |m_f - m_o|^2: centres must be finite and pairwise distinct
        for (int k = 0; k < chunks->k; k++) {
            const float* ck = chunks->center + 3 * k;
            if (!std::isfinite(ck[0]) || !std::isfinite(ck[1]) || !std::isfinite(ck[2])) {
                delete s;
                return fail(LODGE_ERR_INVALID_ARG, "chunk centres must be finite");
            }
            for (int j = 0; j < k; j++) {
                const float* cj = chunks->center + 3 * j;
                const float g0 = ck[0] - cj[0], g1 = ck[1] - cj[1], g2 = ck[2] - cj[2];
                const float den = (g0 * g0 + g1 * g1) + g2 * g2;
                if (!(den > 0.0f) || !std::isfinite(den)) {
                    delete s;
                    return fail(LODGE_ERR_INVALID_ARG, "chunk centres must be pairwise distinct (and their squared "
                                                       "distances finite and non-zero in FP32)");
                }
            }
        }
        s->chunks.K = chunks->k;
        s->chunks.band = chunks->band;
        for (int k = 0; k < chunks->k; k++) {
            s->chunks.c[k] = make_float4(chunks->center[3 * k], chunks->center[3 * k + 1], chunks->center[3 * k + 2],
                                         chunks->offset[k]);
            if (!std::isfinite(s->chunks.c[k].w) || s->chunks.c[k].w < 0.0f) {
                delete s;
                return fail(LODGE_ERR_INVALID_ARG, "chunk offsets must be finite and >= 0");
            }
        }
        s->has_chunks = true;
    }
    *out = s;
    return LODGE_OK;
}

void lodge_scene_destroy(lodge_scene* scene) { delete scene; }

int64_t lodge_scene_total(const lodge_scene* scene) { return scene ? (int64_t)scene->levels.total : -1; }

lodge_status lodge_workspace_size(const lodge_scene* scene, int32_t width, int32_t height, uint32_t max_active,
                                  uint64_t max_instances, size_t* bytes)
{
    if (!scene || !bytes) return fail(LODGE_ERR_INVALID_ARG, "scene or bytes is NULL");
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384)
        return fail(LODGE_ERR_INVALID_ARG, "image size out of range");
    if (max_instances >= (1ull << 32)) return fail(LODGE_ERR_INVALID_ARG, "max_instances must be < 2^32");
    if (max_active >= (1u << 31)) return fail(LODGE_ERR_INVALID_ARG, "max_active must be < 2^31");
    if (tiles_of(width, height) > (uint64_t)kMaxTiles)
        return fail(LODGE_ERR_UNSUPPORTED, "image has more than 32768 16x16 tiles");
    *bytes = make_layout(scene->levels.total, width, height, max_active, max_instances).total;
    return LODGE_OK;
}

namespace {
uint32_t sh_stride4(int32_t deg) { return (uint32_t)((3 * (deg + 1) * (deg + 1) + 3) / 4); }
}  // namespace

lodge_status lodge_pack_size(const lodge_scene* scene, size_t* bytes)
{
    if (!scene || !bytes) return fail(LODGE_ERR_INVALID_ARG, "scene or bytes is NULL");
    size_t b = 0;
    for (int l = 0; l < scene->levels.L; l++) {
        const LevelDev& L = scene->levels.lv[l];
        b += (size_t)L.n * (32 + 16 * (size_t)sh_stride4(L.sh_degree));
        b = (b + 255) & ~(size_t)255;
    }
    *bytes = b;
    return LODGE_OK;
}

lodge_status lodge_scene_pack(lodge_scene* scene, void* pack, size_t bytes, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    if (!pack) {   // detach: the projection reads the level planes again
        for (int l = 0; l < LODGE_MAX_LEVELS; l++) scene->levels.pk[l] = PackDev{nullptr, nullptr, 0};
        scene->levels.packed = 0;
        return LODGE_OK;
    }
    size_t need = 0;
    lodge_pack_size(scene, &need);
    if (bytes < need) return fail(LODGE_ERR_INVALID_ARG, "pack buffer smaller than lodge_pack_size()");
    if (reinterpret_cast<uintptr_t>(pack) & 255) return fail(LODGE_ERR_INVALID_ARG, "pack buffer not 256-byte aligned");
    LevelsArg lv = scene->levels;
    char* b = static_cast<char*>(pack);
    size_t off = 0;
    for (int l = 0; l < lv.L; l++) {
        const LevelDev& L = lv.lv[l];
        PackDev& P = lv.pk[l];
        P.sh_stride4 = sh_stride4(L.sh_degree);
        P.pgeo = reinterpret_cast<const float4*>(b + off);
        P.psh = reinterpret_cast<const float4*>(b + off + 32 * (size_t)L.n);
        off += (size_t)L.n * (32 + 16 * (size_t)P.sh_stride4);
        off = (off + 255) & ~(size_t)255;
    }
    const hipError_t e = launch_pack(lv, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "lodge_scene_pack");
    lv.packed = 1;
    scene->levels = lv;
    return LODGE_OK;
}

lodge_status lodge_set_camera(const lodge_workspace* ws, const lodge_camera* cam, void* stream)
{
    if (!ws || !ws->base) return fail(LODGE_ERR_INVALID_ARG, "workspace is NULL");
    if (!cam) return fail(LODGE_ERR_INVALID_ARG, "camera is NULL");
    lodge_status s;
    if ((s = check_cam(cam, ws)) != LODGE_OK) return s;
    const Views v = views_of(ws, 0);
    const hipError_t e = launch_set_camera(*cam, v, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_set_camera");
}

lodge_status lodge_select(const lodge_scene* scene, const lodge_camera* cam, int32_t mode, const lodge_workspace* ws,
                          lodge_selection* sel, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_cam(cam, nullptr)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    if (mode < LODGE_SELECT_ALL || mode > LODGE_SELECT_CHUNKED) return fail(LODGE_ERR_INVALID_ARG, "unknown mode");
    if (mode == LODGE_SELECT_CHUNKED && !scene->has_chunks)
        return fail(LODGE_ERR_INVALID_ARG, "chunked selection on a scene without chunks");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Views v = views_of(ws, scene->levels.total);
    hipError_t e = hipSuccess;
    if ((e = launch_select_setup(scene->levels, scene->chunks, mode, cam, v, st)) != hipSuccess)
        return hip_fail(e, "lodge_select: setup");
    if ((e = launch_select(scene->levels, v, *sel, st)) != hipSuccess) return hip_fail(e, "lodge_select");
    return LODGE_OK;
}

lodge_status lodge_chunk_sets_size(const lodge_scene* scene, size_t* bytes)
{
    if (!scene || !bytes) return fail(LODGE_ERR_INVALID_ARG, "scene or bytes is NULL");
    if (!scene->has_chunks) return fail(LODGE_ERR_INVALID_ARG, "the scene has no chunks");
    *bytes = (size_t)scene->chunks.K * std::max<uint32_t>(scene->levels.sel_blocks, 1) * kSelBlock * sizeof(uint16_t);
    return LODGE_OK;
}

lodge_status lodge_chunk_sets_build(const lodge_scene* scene, void* sets, size_t bytes, void* stream)
{
    size_t need = 0;
    lodge_status s = lodge_chunk_sets_size(scene, &need);
    if (s != LODGE_OK) return s;
    if (!sets || bytes < need) return fail(LODGE_ERR_INVALID_ARG, "chunk-set buffer is NULL or too small");
    if (reinterpret_cast<uintptr_t>(sets) % 4) return fail(LODGE_ERR_INVALID_ARG, "chunk-set buffer must be 4-byte aligned");
    const hipError_t e = launch_sets_build(scene->levels, scene->chunks, static_cast<uint16_t*>(sets),
                                           static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_chunk_sets_build");
}

lodge_status lodge_select_chunk_sets(const lodge_scene* scene, const void* sets, const lodge_camera* cam,
                                     const lodge_workspace* ws, lodge_selection* sel, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    if (!scene->has_chunks) return fail(LODGE_ERR_INVALID_ARG, "the scene has no chunks");
    if (!sets) return fail(LODGE_ERR_INVALID_ARG, "chunk sets are NULL");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_cam(cam, nullptr)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Views v = views_of(ws, scene->levels.total);
    hipError_t e = hipSuccess;
    if ((e = launch_select_setup(scene->levels, scene->chunks, LODGE_SELECT_CHUNKED, cam, v, st)) != hipSuccess)
        return hip_fail(e, "lodge_select_chunk_sets: setup");
    if ((e = launch_sets_mark(scene->levels, v, static_cast<const uint16_t*>(sets), st)) != hipSuccess)
        return hip_fail(e, "lodge_select_chunk_sets: mark");
    if ((e = launch_select_finish(scene->levels, v, *sel, st)) != hipSuccess)
        return hip_fail(e, "lodge_select_chunk_sets");
    return LODGE_OK;
}

lodge_status lodge_select_chunk(const lodge_scene* scene, const void* sets, int32_t k, const lodge_workspace* ws,
                                lodge_selection* sel, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    if (!scene->has_chunks) return fail(LODGE_ERR_INVALID_ARG, "the scene has no chunks");
    if (k < 0 || k >= scene->chunks.K) return fail(LODGE_ERR_INVALID_ARG, "chunk index out of range");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Views v = views_of(ws, scene->levels.total);
    hipError_t e = hipSuccess;
    if ((e = launch_select_setup(scene->levels, scene->chunks, LODGE_SELECT_CHUNKED, nullptr, v, st, k)) !=
        hipSuccess)
        return hip_fail(e, "lodge_select_chunk: setup");
    if (sets) {
        if ((e = launch_sets_mark(scene->levels, v, static_cast<const uint16_t*>(sets), st)) != hipSuccess)
            return hip_fail(e, "lodge_select_chunk: mark");
        if ((e = launch_select_finish(scene->levels, v, *sel, st)) != hipSuccess)
            return hip_fail(e, "lodge_select_chunk");
    } else if ((e = launch_select(scene->levels, v, *sel, st)) != hipSuccess) {
        return hip_fail(e, "lodge_select_chunk");
    }
    return LODGE_OK;
}

lodge_status lodge_chunk_sets_prune(const lodge_scene* scene, void* sets, size_t bytes, int32_t k, const float* score,
                                    float threshold, void* stream)
{
    size_t need = 0;
    lodge_status s = lodge_chunk_sets_size(scene, &need);
    if (s != LODGE_OK) return s;
    if (!sets || bytes < need) return fail(LODGE_ERR_INVALID_ARG, "chunk-set buffer is NULL or too small");
    if (reinterpret_cast<uintptr_t>(sets) % 4) return fail(LODGE_ERR_INVALID_ARG, "chunk-set buffer must be 4-byte aligned");
    if (k < 0 || k >= scene->chunks.K) return fail(LODGE_ERR_INVALID_ARG, "chunk index out of range");
    if (!score) return fail(LODGE_ERR_INVALID_ARG, "score is NULL");
    if (!std::isfinite(threshold)) return fail(LODGE_ERR_INVALID_ARG, "threshold must be finite");
    const hipError_t e = launch_sets_prune(scene->levels, static_cast<uint16_t*>(sets), k, score, threshold,
                                           static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_chunk_sets_prune");
}

lodge_status lodge_importance(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                              const lodge_render_opts* opts, const lodge_workspace* ws, float* score, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_cam(cam, ws)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    if (!score) return fail(LODGE_ERR_INVALID_ARG, "score is NULL");
    if (reinterpret_cast<uintptr_t>(score) % 4) return fail(LODGE_ERR_INVALID_ARG, "score must be 4-byte aligned");
    lodge_render_opts o;
    if ((s = check_render_opts(opts, &o)) != LODGE_OK) return s;
    const Views v = views_of(ws, scene->levels.total);
    return render_stages(scene, *sel, cam, o, v, true, nullptr, nullptr, nullptr, static_cast<hipStream_t>(stream),
                         score);
}

lodge_status lodge_render(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                          const lodge_render_opts* opts, const lodge_workspace* ws, float* image, float* final_T,
                          uint32_t* n_contrib, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_cam(cam, ws)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    if (!image || !final_T || !n_contrib) return fail(LODGE_ERR_INVALID_ARG, "output buffers are NULL");
    lodge_render_opts o;
    if ((s = check_render_opts(opts, &o)) != LODGE_OK) return s;
    const Views v = views_of(ws, scene->levels.total);
    return render_stages(scene, *sel, cam, o, v, true, image, final_T, n_contrib, static_cast<hipStream_t>(stream));
}

namespace {

// Synchronises the stream and copies the frame's info block; with_pairs also
// sums the compositor's per-(tile, quadrant) pair counters.
lodge_status read_info(const lodge_workspace* ws, lodge_frame_info* out, void* stream, bool with_pairs)
{
    if (!ws || !ws->base || !out) return fail(LODGE_ERR_INVALID_ARG, "workspace or out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "lodge_frame_info_read: sync");
    // the leading regions of the layout do not depend on the scene
    const Layout lay = make_layout(0, ws->width, ws->height, ws->max_active, ws->max_instances);
    const char* base = static_cast<const char*>(ws->base);
    FrameInfo fi;
    e = hipMemcpy(&fi, base + lay.info, sizeof(fi), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "lodge_frame_info_read: copy");
    if (with_pairs) {
        std::vector<uint4> ws4(4ull * lay.T);
        e = hipMemcpy(ws4.data(), base + lay.wstats, ws4.size() * sizeof(uint4), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "lodge_frame_info_read: copy counters");
        unsigned long long ev = 0, bl = 0, st = 0;
        for (const uint4& q : ws4) {
            ev += (unsigned long long)q.x | ((unsigned long long)q.y << 32);
            bl += q.z;
            st += q.w;
        }
        fi.pairs_evaluated = ev;
        fi.pairs_blended = bl;
        out->pixels_stopped = st;
    } else {
        out->pixels_stopped = 0;
    }
    out->n_selected = fi.n_selected;
    out->n_front = fi.n_front;
    out->n_visible = fi.n_visible;
    out->max_tile_len = fi.max_tile_len;
    out->n_instances = fi.n_instances;
    out->pairs_evaluated = fi.pairs_evaluated;
    out->pairs_blended = fi.pairs_blended;
    out->overflow = fi.overflow;
    out->f = fi.f;
    out->o = fi.o;
    out->t = fi.t;
    out->n_long = fi.n_large + fi.n_xl;
    out->n_merge = fi.n_huge;
    return LODGE_OK;
}

}  // namespace

lodge_status lodge_frame_info_read(const lodge_workspace* ws, lodge_frame_info* out, void* stream)
{
    return read_info(ws, out, stream, true);
}

lodge_status lodge_check(const lodge_workspace* ws, uint32_t* needed_active, uint64_t* needed_instances, void* stream)
{
    lodge_frame_info fi;
    lodge_status s = read_info(ws, &fi, stream, false);
    if (s != LODGE_OK) return s;
    if (needed_active) *needed_active = fi.n_selected;
    if (needed_instances) *needed_instances = fi.n_instances;
    if (fi.overflow & (kOvfSelect | kOvfInstances)) {
        char buf[160];
        snprintf(buf, sizeof buf, "capacity exceeded: selected %u (cap %u), instances %llu (cap %llu)", fi.n_selected,
                 ws->max_active, (unsigned long long)fi.n_instances, (unsigned long long)ws->max_instances);
        return fail(LODGE_ERR_CAPACITY, buf);
    }
    return LODGE_OK;
}

lodge_status lodge_debug_views(const lodge_workspace* ws, const uint32_t** sorted_ids, const uint32_t** tile_ranges,
                               const float** proj, const float** depth, const uint32_t** rect)
{
    if (!ws || !ws->base) return fail(LODGE_ERR_INVALID_ARG, "workspace is NULL");
    // every region but the trailing selection flags is independent of the scene size
    const Views v = views_of(ws, 0);
    if (sorted_ids) *sorted_ids = v.sorted;
    if (tile_ranges) *tile_ranges = reinterpret_cast<const uint32_t*>(v.ranges);
    if (proj) *proj = reinterpret_cast<const float*>(v.proj);
    if (depth) *depth = v.depth;
    if (rect) *rect = reinterpret_cast<const uint32_t*>(v.rect);
    return LODGE_OK;
}

lodge_status lodge_render_backward(const lodge_scene* scene, const lodge_selection* sel, const lodge_camera* cam,
                                   const lodge_render_opts* opts, const lodge_workspace* ws, const float* final_T,
                                   const uint32_t* n_contrib, const float* dL_dimage, int32_t grad_level,
                                   const lodge_grads* grads, void* stream)
{
    if (!scene) return fail(LODGE_ERR_INVALID_ARG, "scene is NULL");
    lodge_status s;
    if ((s = check_ws(scene, ws)) != LODGE_OK) return s;
    if ((s = check_cam(cam, ws)) != LODGE_OK) return s;
    if ((s = check_sel(sel, ws)) != LODGE_OK) return s;
    if (!final_T || !n_contrib || !dL_dimage || !grads)
        return fail(LODGE_ERR_INVALID_ARG, "final_T, n_contrib, dL_dimage and grads must be non-NULL");
    if (grad_level < -1 || grad_level >= scene->levels.L) return fail(LODGE_ERR_INVALID_ARG, "grad_level out of range");
    lodge_render_opts o{0.3f, 1, nullptr};
    if (opts) o = *opts;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Views v = views_of(ws, scene->levels.total);
    // the forward's camera and options are still in ws; a given camera replaces it
    hipError_t e = hipSuccess;
    if (cam && (e = launch_set_camera(*cam, v, st)) != hipSuccess) return hip_fail(e, "lodge_render_backward: camera");
    if ((e = launch_backward(scene->levels, *sel, v, final_T, n_contrib, dL_dimage, grad_level, grads, st,
                             o.stage_events)) != hipSuccess)
        return hip_fail(e, "lodge_render_backward");
    return LODGE_OK;
}

lodge_status lodge_activate(int64_t n, const float* log_scale, const float* quat_raw, const float* opacity_logit,
                            float* scale, float* quat, float* opacity, void* stream)
{
    if (n < 0) return fail(LODGE_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return LODGE_OK;
    if (!log_scale || !quat_raw || !opacity_logit || !scale || !quat || !opacity)
        return fail(LODGE_ERR_INVALID_ARG, "activate: NULL plane");
    const hipError_t e = launch_activate(n, log_scale, quat_raw, opacity_logit, scale, quat, opacity,
                                         static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_activate");
}

lodge_status lodge_activate_backward(int64_t n, const float* quat_raw, const float* scale, const float* opacity,
                                     const float* g_scale, const float* g_quat, const float* g_opacity,
                                     float* g_log_scale, float* g_quat_raw, float* g_opacity_logit, void* stream)
{
    if (n < 0) return fail(LODGE_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return LODGE_OK;
    if ((g_scale && (!scale || !g_log_scale)) || (g_quat && (!quat_raw || !g_quat_raw)) ||
        (g_opacity && (!opacity || !g_opacity_logit)))
        return fail(LODGE_ERR_INVALID_ARG, "activate_backward: a gradient is given without its inputs/outputs");
    const hipError_t e = launch_activate_backward(n, quat_raw, scale, opacity, g_scale, g_quat, g_opacity,
                                                  g_log_scale, g_quat_raw, g_opacity_logit,
                                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_activate_backward");
}

}  // extern "C"
