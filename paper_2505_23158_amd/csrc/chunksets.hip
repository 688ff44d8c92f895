// Precomputed per-chunk active sets (LODGE Sec. 3 "Reducing memory with
// chunk-based rendering": each chunk keeps the Gaussians that Eq. 2 selects
// at its centre, with every switch distance offset by the chunk's radius;
// "Opacity blending": a frame renders the union of the two nearest chunks'
// sets, weighted by Eq. 4).
//
// Storage: for chunk k, selection tile s (kSelTile Gaussians inside one
// level, as in the per-frame selection) and thread slot tid, one 16-bit word
// whose bit r says whether item i0 + r kSelBlock + tid belongs to chunk k's
// set.  That is one bit per Gaussian per chunk (3.3 MB per chunk at 26.55M
// Gaussians), laid out so that a frame reads, per thread, exactly the two
// words of its selection-tile slot.
//
//   k_sets_build  once: every tile loads its means, then for every chunk
//                 evaluates the chunk's membership with the same FP32
//                 operations as the per-frame selection, and stores the
//                 words.
//   k_sets_mark   per frame, replacing the mean pass of the selection: the
//                 two chunks' words interleave into the selection's packed
//                 (in_f, in_o) bits and give the tile's member count; the
//                 selection's scan and emit passes then run unchanged.
//
// Built with -ffp-contract=off: memberships must equal those of the
// per-frame selection bit for bit.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

__device__ __forceinline__ float dist2(float px, float py, float pz, float qx, float qy, float qz)
{
    const float dx = px - qx, dy = py - qy, dz = pz - qz;
    return (dx * dx + dy * dy) + dz * dz;
}

// Squared bounds of level l for a chunk of offset r, as the selection setup
// computes them: lo(0) = 0, lo(l) = (d_l + r)^2, hi(l) = lo(l+1), hi(L-1) = inf.
__device__ __forceinline__ void level_bounds(const LevelsArg& lv, int l, float r, float& lo, float& hi)
{
    float s;
    s = (l == 0) ? 0.0f : lv.d[l - 1] + r;
    lo = (l == 0) ? 0.0f : s * s;
    s = (l == lv.L - 1) ? 0.0f : lv.d[l] + r;
    hi = (l == lv.L - 1) ? INFINITY : s * s;
}

__global__ __launch_bounds__(kSelBlock) void k_sets_build(LevelsArg lv, ChunksArg ch, uint32_t ntiles,
                                                          uint16_t* __restrict__ sets)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && tile >= lv.first_block[j]) l = j;
    const LevelDev& L = lv.lv[l];
    const uint32_t n = L.n;
    const uint32_t i0 = (tile - lv.first_block[l]) * (uint32_t)kSelTile;
    float mx[kSelItems], my[kSelItems], mz[kSelItems];
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kSelBlock + tid;
        const bool ok = n > 0 && i < n;
        mx[r] = ok ? L.mean[i] : 0.0f;
        my[r] = ok ? L.mean[n + i] : 0.0f;
        mz[r] = ok ? L.mean[2 * (size_t)n + i] : 0.0f;
    }
    for (int k = 0; k < ch.K; k++) {
        const float4 c = ch.c[k];
        float lo, hi;
        level_bounds(lv, l, c.w, lo, hi);
        uint32_t word = 0;
#pragma unroll
        for (int r = 0; r < kSelItems; r++) {
            const uint32_t i = i0 + (uint32_t)r * kSelBlock + tid;
            const float d = dist2(mx[r], my[r], mz[r], c.x, c.y, c.z);
            if (i < n && lo <= d && d < hi) word |= 1u << r;
        }
        sets[((size_t)k * ntiles + tile) * kSelBlock + tid] = (uint16_t)word;
    }
}

// 16 bits -> the even bits of a 32-bit word
__device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__global__ __launch_bounds__(kSelBlock) void k_sets_mark(const FrameParams* fp, uint32_t ntiles,
                                                         const uint16_t* __restrict__ sets,
                                                         uint32_t* __restrict__ cnt, uint32_t* __restrict__ bits_out)
{
    __shared__ uint32_t s_wave[kSelBlock / 64];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    const int32_t f = fp->f, o = fp->o;
    // the two sets are streamed (read once per frame)
    const uint32_t wf = __builtin_nontemporal_load(sets + ((size_t)f * ntiles + tile) * kSelBlock + tid);
    const uint32_t wo = o >= 0 ? __builtin_nontemporal_load(sets + ((size_t)o * ntiles + tile) * kSelBlock + tid) : 0u;
    const uint32_t bits = spread16(wf) | (spread16(wo) << 1);
    uint32_t mine = (uint32_t)__popc(wf | wo);
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if (lane == 0) s_wave[wave] = mine;
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kSelBlock / 64; k++) total += s_wave[k];
    if (tid == 0) cnt[tile] = total;
    if (total != 0u) bits_out[(size_t)tile * kSelBlock + tid] = bits;
}

// Visibility filtering of one chunk's stored set: every member of chunk k
// whose importance score (by global id) is below the threshold leaves it.
__global__ __launch_bounds__(kSelBlock) void k_sets_prune(LevelsArg lv, uint32_t ntiles, uint16_t* __restrict__ sets,
                                                          int32_t k, const float* __restrict__ score, float thr)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && tile >= lv.first_block[j]) l = j;
    const uint32_t gbase = lv.lv[l].base + (tile - lv.first_block[l]) * (uint32_t)kSelTile;
    uint16_t* const wp = sets + ((size_t)k * ntiles + tile) * kSelBlock + tid;
    const uint32_t word = *wp;
    if (word == 0u) return;
    uint32_t keep = word;
#pragma unroll
    for (int r = 0; r < kSelItems; r++)
        if ((word >> r) & 1u)
            if (!(score[gbase + (uint32_t)r * kSelBlock + tid] >= thr)) keep &= ~(1u << r);
    if (keep != word) *wp = (uint16_t)keep;
}

}  // namespace

hipError_t launch_sets_prune(const LevelsArg& lv, uint16_t* sets, int32_t k, const float* score, float threshold,
                             hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);
    k_sets_prune<<<ntiles, kSelBlock, 0, st>>>(lv, ntiles, sets, k, score, threshold);
    return hipGetLastError();
}

hipError_t launch_sets_build(const LevelsArg& lv, const ChunksArg& ch, uint16_t* sets, hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);
    k_sets_build<<<ntiles, kSelBlock, 0, st>>>(lv, ch, ntiles, sets);
    return hipGetLastError();
}

hipError_t launch_sets_mark(const LevelsArg& lv, const Views& v, const uint16_t* sets, hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);
    k_sets_mark<<<ntiles, kSelBlock, 0, st>>>(v.params, ntiles, sets, v.sel_cnt, v.sel_bits);
    return hipGetLastError();
}

}  // namespace lodge
