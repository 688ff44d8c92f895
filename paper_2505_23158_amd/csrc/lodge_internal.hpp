// Internal declarations of the gfx950 renderer: device-side argument
// structs, the workspace layout and the kernel launchers each translation
// unit provides.  Not part of the public ABI (see include/lodge.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lodge.h"

namespace lodge {

constexpr int kTile = 16;           // screen tiles are 16 x 16 pixels
constexpr int kMaxSh = 16;          // SH coefficients per channel at degree 3

// ---------------------------------------------------------------- arguments

// One level as the kernels see it (passed by value inside LevelsArg).
struct LevelDev {
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* sh;
    uint32_t n;
    uint32_t base;      // global id of the level's first Gaussian
    int32_t sh_degree;
    float var;          // Eq. 3 filter variance
};

// A level's packed copy (lodge_scene_pack), null when absent: per Gaussian
// two float4 (scale xyz, opacity), (quaternion wxyz), and sh_stride4 float4
// of its SH coefficients in [basis][channel] order.
struct PackDev {
    const float4* pgeo;
    const float4* psh;
    uint32_t sh_stride4;
};

struct LevelsArg {
    LevelDev lv[LODGE_MAX_LEVELS];
    int32_t L;
    uint32_t total;
    float d[LODGE_MAX_LEVELS];   // d_1 .. d_{L-1}
    uint32_t first_block[LODGE_MAX_LEVELS + 1];   // selection blocks: level l owns [first_block[l], first_block[l+1])
    uint32_t sel_blocks;
    int32_t packed;     // 1: the projection reads the packed copy of every level
    PackDev pk[LODGE_MAX_LEVELS];
};

struct ChunksArg {
    int32_t K;
    float band;
    float4 c[LODGE_MAX_CHUNKS];   // centre (x, y, z), offset r
};

// Frame parameters in device memory: the camera copy plus what the setup
// kernel derives from it.  Kernels read these instead of kernel arguments so
// that a captured graph re-reads the camera at every replay.
struct FrameParams {
    lodge_camera cam;
    int32_t mode;
    int32_t f, o;
    float t, w_o;
    float cf[3], co[3];              // centres the selection measures from
    float lo_f[LODGE_MAX_LEVELS], hi_f[LODGE_MAX_LEVELS];
    float lo_o[LODGE_MAX_LEVELS], hi_o[LODGE_MAX_LEVELS];
    float s2d;
    int32_t compensate;
    int32_t TX, TY;
};

// Device counters of one frame (mirrors lodge_frame_info, plus tickets).
struct FrameInfo {
    uint32_t n_selected;
    uint32_t n_front;
    uint32_t n_visible;
    unsigned long long n_instances;
    unsigned long long pairs_evaluated;   // filled on the host from the per-wave counters
    unsigned long long pairs_blended;
    uint32_t max_tile_len;
    uint32_t overflow;
    int32_t f, o;
    float t;
    uint32_t n_large;     // tiles with a list in (kSortSmall, kSortMid]
    uint32_t n_huge;      // tiles with a list longer than kSortLarge
    uint32_t n_mid;       // tiles with a list in (kSortWave, kSortSmall]
    uint32_t n_xl;        // tiles with a list in (kSortMid, kSortLarge]
    uint32_t n_binned;    // actives with at least one tile
    uint32_t sort_next;   // next work item of the per-tile sort
    uint32_t scan_done;   // chunk-scan blocks that have written their totals
};

enum : uint32_t { kOvfSelect = 1u, kOvfInstances = 2u, kOvfTile = 4u };

// Element at byte offset off of a plane whose base every lane holds alike:
// the base stays in scalar registers and only the 32-bit offset is a vector
// operand (no 64-bit address arithmetic per load).
typedef const __attribute__((address_space(1))) char gchar;
typedef const __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ float ld_plane(const float* plane, uint32_t off)
{
    return *(const gfloat*)((const gchar*)plane + off);
}

// The same, marked as streamed once (non-temporal: not kept in the caches).
__device__ __forceinline__ float ld_plane_stream(const float* plane, uint32_t off)
{
    return __builtin_nontemporal_load((const gfloat*)((const gchar*)plane + off));
}

// Field-by-field store of a camera held in kernel arguments (a struct
// assignment would stage the argument through private memory).
__device__ __forceinline__ void store_camera(lodge_camera* __restrict__ d, const lodge_camera& c)
{
    d->width = c.width;
    d->height = c.height;
    d->fx = c.fx;
    d->fy = c.fy;
    d->cx = c.cx;
    d->cy = c.cy;
#pragma unroll
    for (int k = 0; k < 9; k++) d->R[k] = c.R[k];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        d->t[k] = c.t[k];
        d->pos[k] = c.pos[k];
        d->bg[k] = c.bg[k];
    }
    d->znear = c.znear;
    d->lim_x = c.lim_x;
    d->lim_y = c.lim_y;
}

// ------------------------------------------------------------ workspace map

constexpr int kSelBlock = 256;
constexpr int kSelItems = 16;                       // per thread
constexpr int kSelTile = kSelBlock * kSelItems;     // Gaussians per selection block
constexpr int kSortWave = 256;                      // runs up to this: one wave, keys in registers
constexpr int kSortSmall = 2048;                    // runs up to this: 256 threads x 8 keys ("mid" queue)
constexpr int kSortMid = 4096;                      // runs up to this: 512 threads x 8 keys
constexpr int kSortLarge = 16384;                   // runs longer than this: the "huge" queue
constexpr int kBinChunk = 4096;                     // instances per binning block
constexpr int kScanChunks = 4096;                   // projection chunks per chunk-scan block
constexpr int kProjChunk = 64;                      // actives per projection chunk: one wave (instance-scan granule)
constexpr int kMaxTiles = 32768;                    // 16-bit-packed LDS tile histograms (e.g. 3840 x 2160)

struct Layout {
    size_t params, info, wstats, bstart, sel_cnt, sel_off, sel_bits, chunk_sum, chunk_vis, scan_blk, proj, depth, rect, vtiles, vis_off,
        vis_id, inst, hist, tcount, ranges, order, large, sorted, temp, g2d, total;
    uint32_t sel_tiles, TX, TY, T, bin_blocks;
};

Layout make_layout(uint32_t n_total, int32_t width, int32_t height, uint32_t max_active, uint64_t max_instances);

// Typed views of a workspace.
struct Views {
    FrameParams* params;
    FrameInfo* info;
    uint4* wstats;         // per (tile, quadrant): pairs evaluated (lo, hi), pairs blended, pixels stopped
    uint32_t* sel_cnt;     // per selection tile: member count
    uint32_t* sel_off;     // per selection tile: exclusive offset of its members
    uint32_t* sel_bits;    // [selection tiles][kSelBlock] two membership bits per item
    uint32_t* chunk_sum;   // per projection chunk: tile total -> exclusive instance offset
    uint32_t* chunk_vis;   // per projection chunk: actives with >= 1 tile -> exclusive offset among them
    uint4* scan_blk;       // per chunk-scan block: its totals -> its exclusive offsets
    float4* proj;          // [max_active][3]: (u, v, -A/2, -B), (-C/2, o, thr, r), (g, b, ex, ey); visible only
    float* depth;          // [max_active] camera depth (sort key), 0 when culled
    uint2* rect;           // [max_active] tile rect (x0 | y0 << 16, x1 | y1 << 16), empty when culled
    uint32_t* vtiles;      // tiles touched per active index
    uint32_t* vis_off;     // per active with >= 1 tile, in index order: its first instance
    uint32_t* vis_id;      // ... and its active index
    uint32_t* bstart;      // per binning block: the vis_off slot holding its first instance
    uint2* inst;           // [max_instances] (tile, active index) in emission order
    uint32_t* hist;        // [bin blocks][T] per-block tile counts -> per-block first slots
    uint32_t* tcount;      // per tile list length
    uint2* ranges;         // per tile [start, end)
    uint32_t* order;       // tiles by decreasing list length
    uint32_t* large;       // queues: [0, T) lists in (2048, 16384], [T, 2T) longer, [2T, 3T) in (256, 2048]
    uint32_t* sorted;      // [max_instances] active indices, tile-major
    unsigned long long* temp;   // [max_instances] merge scratch for very long lists
    float* g2d;            // [max_active][12] adjoint of the projected quantities
    Layout lay;
    uint32_t max_active;
    uint64_t max_instances;
};

Views views_of(const lodge_workspace* ws, uint32_t n_total);

// ----------------------------------------------------------------- launchers
// Each returns hipGetLastError() after enqueueing on `st`.

hipError_t launch_set_camera(const lodge_camera& cam, const Views& v, hipStream_t st);
// only_chunk >= 0: the set of that chunk alone (mode must be chunked): f = only_chunk, no second chunk, t = 1
hipError_t launch_select_setup(const LevelsArg& lv, const ChunksArg& ch, int32_t mode, const lodge_camera* cam,
                              const Views& v, hipStream_t st, int32_t only_chunk = -1);
hipError_t launch_select(const LevelsArg& lv, const Views& v, const lodge_selection& sel, hipStream_t st);
// scan + emit of the selection from the per-tile counts and packed bits already in the workspace
hipError_t launch_select_finish(const LevelsArg& lv, const Views& v, const lodge_selection& sel, hipStream_t st);
hipError_t launch_sets_build(const LevelsArg& lv, const ChunksArg& ch, uint16_t* sets, hipStream_t st);
hipError_t launch_sets_mark(const LevelsArg& lv, const Views& v, const uint16_t* sets, hipStream_t st);
// clears chunk k's bit of every member whose score (by global id) is below threshold
hipError_t launch_sets_prune(const LevelsArg& lv, uint16_t* sets, int32_t k, const float* score, float threshold,
                             hipStream_t st);
// keep_select_flag: keep the selection-overflow bit a lodge_select on the same workspace set
hipError_t launch_render_setup(const lodge_render_opts& o, const lodge_camera* cam, const Views& v,
                               bool keep_select_flag, hipStream_t st);
hipError_t launch_project(const LevelsArg& lv, const lodge_selection& sel, const Views& v, hipStream_t st);
hipError_t launch_bin(const Views& v, const lodge_selection& sel, hipStream_t st);
hipError_t launch_sort(const Views& v, hipStream_t st);
hipError_t launch_composite(const Views& v, float* image, float* final_T, uint32_t* n_contrib, hipStream_t st);
// the compositor's walk, max-accumulating each blended weight alpha T into score[sel_ids[a]]
hipError_t launch_importance(const Views& v, const uint32_t* sel_ids, float* score, hipStream_t st);
hipError_t launch_backward(const LevelsArg& lv, const lodge_selection& sel, const Views& v, const float* final_T,
                           const uint32_t* n_contrib, const float* dL_dimage, int32_t grad_level,
                           const lodge_grads* grads, hipStream_t st, void* const* events = nullptr);
// fills the packed copy of every level (layout in LevelDev)
hipError_t launch_pack(const LevelsArg& lv, hipStream_t st);
hipError_t launch_activate(int64_t n, const float* ls, const float* qr, const float* ol, float* s, float* q, float* o,
                           hipStream_t st);
hipError_t launch_activate_backward(int64_t n, const float* qr, const float* s, const float* o, const float* gs,
                                    const float* gq, const float* go, float* gls, float* gqr, float* gol,
                                    hipStream_t st);

// ------------------------------------------------------------ host helpers (api.hip)

// Records msg as the calling thread's last error and returns s.
lodge_status fail(lodge_status s, const std::string& msg);
lodge_status hip_fail(hipError_t e, const char* where);
uint64_t tiles_of(int32_t w, int32_t h);
// cam may be NULL (then OK); ws may be NULL (then the size is not checked).
lodge_status check_cam(const lodge_camera* c, const lodge_workspace* ws);
// Defaults (s2d 0.3, compensation on) for opts == NULL; validates s2d.
lodge_status check_render_opts(const lodge_render_opts* opts, lodge_render_opts* o);

}  // namespace lodge

// The scene behind the opaque handle of include/lodge.h.
struct lodge_scene {
    lodge::LevelsArg levels;
    lodge::ChunksArg chunks;
    bool has_chunks;
};

namespace lodge {

// The stages of lodge_render (setup, project, bin, sort, composite) on the
// views of a workspace; keep_select_flag as for launch_render_setup.
// With score non-NULL the last stage is the importance walk (no image).
lodge_status render_stages(const lodge_scene* scene, const lodge_selection& sel, const lodge_camera* cam,
                           const lodge_render_opts& o, const Views& v, bool keep_select_flag, float* image,
                           float* final_T, uint32_t* n_contrib, hipStream_t st, float* score = nullptr);

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Grid sizes that fill the chip (256 CUs) without depending on device counts.
constexpr int kPersistentBlocks = 2048;

}  // namespace lodge
