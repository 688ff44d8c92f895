// Active-set selection (LODGE Sec. 3, Eq. 2 with the per-chunk offset
// thresholds of "Reducing memory with chunk-based rendering", and the
// two-chunk opacity weights of Eq. 4).
//
// k_select_setup  one wave finds the two nearest chunk centres and t, and
//                 turns the switch distances into squared FP32 bounds.
// k_select        one pass over every Gaussian of every level (each block
//                 inside one level, so its parameters and bounds are
//                 uniform): coalesced loads of the three mean planes,
//                 membership on squared FP32 distances, two bits per item
//                 packed per thread, and the tile's member count.
// k_select_scan   one block: exclusive scan of the tile counts.
// k_select_emit   tiles with members only: re-derives the in-tile order
//                 from the packed bits (ballots + an LDS scan) and writes
//                 ids (ascending global id) and weights.  The positions
//                 are read once; no block waits on another.
//
// Bit-exactness: this file is built with -ffp-contract=off, so each
// +, -, *, / and sqrt below is one IEEE-rounded FP32 operation, evaluated
// in the order written (the order the oracle uses as the definition).
#include "lodge_internal.hpp"

namespace lodge {

namespace {

__device__ __forceinline__ float dist2(float px, float py, float pz, float qx, float qy, float qz)
{
    const float dx = px - qx, dy = py - qy, dz = pz - qz;
    return (dx * dx + dy * dy) + dz * dz;
}

// lexicographic (d, k) minimum across the wave
__device__ __forceinline__ void wave_argmin(float& d, int& k)
{
    for (int off = 32; off > 0; off >>= 1) {
        const float od = __shfl_xor(d, off);
        const int ok = __shfl_xor(k, off);
        if (od < d || (od == d && ok < k)) { d = od; k = ok; }
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One wave.  With a camera argument (has_cam) the kernel also stores it into
// the frame parameters, which saves a launch.
// only_chunk >= 0 (chunked mode): the set of that chunk alone, f = only_chunk,
// no second chunk, t = 1 (every member weighs 1).
__global__ __launch_bounds__(64) void k_select_setup(ChunksArg ch, LevelsArg lv, int32_t mode, lodge_camera cam,
                                                     int32_t has_cam, FrameParams* fp, FrameInfo* info,
                                                     int32_t only_chunk)
{
    const int lane = threadIdx.x;
    const float px = has_cam ? cam.pos[0] : fp->cam.pos[0];
    const float py = has_cam ? cam.pos[1] : fp->cam.pos[1];
    const float pz = has_cam ? cam.pos[2] : fp->cam.pos[2];
    int f = -1, o = -1;
    float t = 1.0f;
    if (mode == LODGE_SELECT_CHUNKED && only_chunk >= 0) {
        f = only_chunk;
    } else if (mode == LODGE_SELECT_CHUNKED) {
        float d = INFINITY;
        int k = 0x7fffffff;
        for (int c = lane; c < ch.K; c += 64) {
            const float4 m = ch.c[c];
            const float dc = dist2(px, py, pz, m.x, m.y, m.z);
            if (dc < d || (dc == d && c < k)) { d = dc; k = c; }
        }
        wave_argmin(d, k);
        f = k;
        if (ch.K > 1) {
            float d2 = INFINITY;
            int k2 = 0x7fffffff;
            for (int c = lane; c < ch.K; c += 64) {
                if (c == f) continue;
                const float4 m = ch.c[c];
                const float dc = dist2(px, py, pz, m.x, m.y, m.z);
                if (dc < d2 || (dc == d2 && c < k2)) { d2 = dc; k2 = c; }
            }
            wave_argmin(d2, k2);
            o = k2;
            // Eq. 4: t_bar = ((c - m_o) . (m_f - m_o)) / |m_f - m_o|^2
            const float4 mf = ch.c[f], mo = ch.c[o];
            const float g0 = mf.x - mo.x, g1 = mf.y - mo.y, g2 = mf.z - mo.z;
            const float e0 = px - mo.x, e1 = py - mo.y, e2 = pz - mo.z;
            const float num = (e0 * g0 + e1 * g1) + e2 * g2;
            const float den = (g0 * g0 + g1 * g1) + g2 * g2;
            float tb = num / den;
            if (ch.band > 0.0f) tb = 0.5f + (tb - 0.5f) * (sqrtf(den) / ch.band);
            t = tb < 0.0f ? 0.0f : tb;
            t = t > 1.0f ? 1.0f : t;
        }
    }
    if (lane != 0) return;
    if (has_cam) store_camera(&fp->cam, cam);
    fp->mode = mode;
    fp->f = f;
    fp->o = o;
    fp->t = t;
    fp->w_o = 1.0f - t;
    float cf[3] = {0.0f, 0.0f, 0.0f}, co[3] = {0.0f, 0.0f, 0.0f};
    float rf = 0.0f, ro = 0.0f;
    if (mode == LODGE_SELECT_LOD_CAMERA) { cf[0] = px; cf[1] = py; cf[2] = pz; }
    if (mode == LODGE_SELECT_CHUNKED) {
        const float4 mf = ch.c[f];
        cf[0] = mf.x; cf[1] = mf.y; cf[2] = mf.z;
        rf = mf.w;
        if (o >= 0) {
            const float4 mo = ch.c[o];
            co[0] = mo.x; co[1] = mo.y; co[2] = mo.z;
            ro = mo.w;
        }
    }
    for (int j = 0; j < 3; j++) { fp->cf[j] = cf[j]; fp->co[j] = co[j]; }
    // squared bounds: lo(0) = 0, lo(l) = (d_l + r)^2, hi(l) = lo(l+1), hi(L-1) = inf
#pragma unroll
    for (int l = 0; l < LODGE_MAX_LEVELS; l++) {
        if (l >= lv.L) break;
        float s;
        s = (l == 0) ? 0.0f : lv.d[l - 1] + rf;
        fp->lo_f[l] = (l == 0) ? 0.0f : s * s;
        s = (l == lv.L - 1) ? 0.0f : lv.d[l] + rf;
        fp->hi_f[l] = (l == lv.L - 1) ? INFINITY : s * s;
        s = (l == 0) ? 0.0f : lv.d[l - 1] + ro;
        fp->lo_o[l] = (l == 0) ? 0.0f : s * s;
        s = (l == lv.L - 1) ? 0.0f : lv.d[l] + ro;
        fp->hi_o[l] = (l == lv.L - 1) ? INFINITY : s * s;
    }
    info->n_selected = 0;
    info->overflow = 0;
    info->f = f;
    info->o = o;
    info->t = t;
}

// Pass 1, one block per selection tile of kSelTile Gaussians (every tile
// inside one level, so level parameters and bounds are block-uniform).
// Thread tid holds items i0 + r * kSelBlock + tid, r < kSelItems, and packs
// their membership (in_f, in_o) as two bits per item into one word.  The
// tile's count is always written; the words only when it is non-zero.
__global__ __launch_bounds__(kSelBlock) void k_select(LevelsArg lv, const FrameParams* fp, uint32_t ntiles,
                                                      uint32_t* __restrict__ cnt, uint32_t* __restrict__ bits_out)
{
    __shared__ uint32_t s_wave[kSelBlock / 64];
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles) return;
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && tile >= lv.first_block[j]) l = j;
    const LevelDev& L = lv.lv[l];
    const uint32_t n = L.n;
    const uint32_t i0 = (tile - lv.first_block[l]) * (uint32_t)kSelTile;
    const int32_t mode = fp->mode;
    const bool all = mode == LODGE_SELECT_ALL;
    const bool two = (mode == LODGE_SELECT_CHUNKED) && (fp->o >= 0);
    const float cf[3] = {fp->cf[0], fp->cf[1], fp->cf[2]};
    const float co[3] = {fp->co[0], fp->co[1], fp->co[2]};
    const float lof = fp->lo_f[l], hif = fp->hi_f[l], loo = fp->lo_o[l], hio = fp->hi_o[l];

    // all loads first, then the tests: block-uniform plane bases (scalar
    // registers) plus 32-bit lane byte offsets (a level holds fewer than 2^30
    // Gaussians), so no address is formed in 64-bit vector arithmetic; in the
    // level's last, partial tile the indices are clamped into the level so no
    // load sits in a branch
    float mx[kSelItems], my[kSelItems], mz[kSelItems];
    if (!all && n > 0) {
        const float* __restrict__ px = L.mean;
        const float* __restrict__ py = L.mean + n;
        const float* __restrict__ pz = L.mean + 2 * (size_t)n;
        if (i0 + (uint32_t)kSelTile <= n) {
            const uint32_t o0 = (i0 + tid) * 4u;
#pragma unroll
            for (int r = 0; r < kSelItems; r++) {
                const uint32_t o = o0 + (uint32_t)r * (kSelBlock * 4u);
                mx[r] = ld_plane_stream(px, o);
                my[r] = ld_plane_stream(py, o);
                mz[r] = ld_plane_stream(pz, o);
            }
        } else {
#pragma unroll
            for (int r = 0; r < kSelItems; r++) {
                const uint32_t o = min(i0 + (uint32_t)r * kSelBlock + tid, n - 1) * 4u;
                mx[r] = ld_plane_stream(px, o);
                my[r] = ld_plane_stream(py, o);
                mz[r] = ld_plane_stream(pz, o);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < kSelItems; r++) mx[r] = my[r] = mz[r] = 0.0f;
    }
    uint32_t bits = 0, mine = 0;
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kSelBlock + tid;
        uint32_t s = 0;
        if (i < n) {
            if (all) {
                s = 1;
            } else {
                const float df = dist2(mx[r], my[r], mz[r], cf[0], cf[1], cf[2]);
                if (lof <= df && df < hif) s |= 1u;
                if (two) {
                    const float dq = dist2(mx[r], my[r], mz[r], co[0], co[1], co[2]);
                    if (loo <= dq && dq < hio) s |= 2u;
                }
            }
        }
        bits |= s << (2 * r);
        mine += s != 0u ? 1u : 0u;
    }
    const uint32_t wsum = wave_sum(mine);
    if (lane == 0) s_wave[wave] = wsum;
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kSelBlock / 64; k++) total += s_wave[k];
    if (tid == 0) cnt[tile] = total;
    if (total != 0u) bits_out[(size_t)tile * kSelBlock + tid] = bits;
}

// One block: exclusive scan of the tile counts -> tile offsets, the active
// count and the capacity flag.  Each thread takes a contiguous run of tiles.
constexpr int kSelScanThreads = 1024;

__global__ __launch_bounds__(kSelScanThreads) void k_select_scan(FrameInfo* info, const uint32_t* __restrict__ cnt,
                                                                 uint32_t* __restrict__ off, uint32_t ntiles,
                                                                 uint32_t cap, uint32_t* count_out)
{
    // up to kPer counts per thread are held in registers, their loads issued
    // together; beyond that (more than kPer x 1024 tiles) the run is re-read
    constexpr int kPer = 8;
    __shared__ uint32_t s_w[kSelScanThreads / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (ntiles + kSelScanThreads - 1) / kSelScanThreads;
    const uint32_t c0 = min(ntiles, tid * per), c1 = min(ntiles, c0 + per);
    uint32_t v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; q++) v[q] = c0 + q < c1 ? cnt[c0 + q] : 0u;
    uint32_t local = 0;
#pragma unroll
    for (int q = 0; q < kPer; q++) local += v[q];
    for (uint32_t c = c0 + kPer; c < c1; c++) local += cnt[c];
    // block scan: wave scans, then the wave totals
    uint32_t inc = local;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o);
        if ((int)lane >= o) inc += u;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kSelScanThreads / 64; k++) {
        const uint32_t x = s_w[k];
        before += (uint32_t)k < wave ? x : 0u;
        total += x;
    }
    uint32_t run = before + inc - local;   // totals stay below 2^32: at most n_total Gaussians
#pragma unroll
    for (int q = 0; q < kPer; q++)
        if (c0 + q < c1) {
            off[c0 + q] = run;
            run += v[q];
        }
    for (uint32_t c = c0 + kPer; c < c1; c++) {
        off[c] = run;
        run += cnt[c];
    }
    if (tid == 0) {
        *count_out = total;
        info->n_selected = total;
        if (total > cap) atomicOr(&info->overflow, kOvfSelect);
    }
}

// Pass 2, one block per tile with a non-zero count: the membership words
// give each (item round, wave) count by ballots; an LDS scan in the item
// order (round, wave, lane) places every member at its ascending-id slot.
__global__ __launch_bounds__(kSelBlock) void k_select_emit(LevelsArg lv, const FrameParams* fp, uint32_t ntiles,
                                                           const uint32_t* __restrict__ cnt,
                                                           const uint32_t* __restrict__ off,
                                                           const uint32_t* __restrict__ bits_in, uint32_t* ids,
                                                           float* w, uint32_t cap)
{
    __shared__ uint32_t s_cnt[kSelItems * 4];
    const uint32_t tile = blockIdx.x;
    if (tile >= ntiles || cnt[tile] == 0u) return;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && tile >= lv.first_block[j]) l = j;
    const uint32_t gbase = lv.lv[l].base + (tile - lv.first_block[l]) * (uint32_t)kSelTile;
    const uint32_t bits = __builtin_nontemporal_load(bits_in + (size_t)tile * kSelBlock + tid);   // read once
    // read before the barriers below, so the loads overlap the in-tile scan
    const uint32_t excl = off[tile];
    const float t = fp->t, w_o = fp->w_o;
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const unsigned long long m = __ballot(((bits >> (2 * r)) & 3u) != 0u);
        if (lane == 0) s_cnt[r * 4 + wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t v = lane < (uint32_t)(kSelItems * 4) ? s_cnt[lane] : 0u;
        uint32_t inc = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o);
            if ((int)lane >= o) inc += u;
        }
        if (lane < (uint32_t)(kSelItems * 4)) s_cnt[lane] = inc - v;
    }
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t s = (bits >> (2 * r)) & 3u;
        const unsigned long long m = __ballot(s != 0u);
        if (s != 0u) {
            const uint32_t pos = excl + s_cnt[r * 4 + wave] + (uint32_t)__popcll(m & lt);
            if (pos < cap) {
                ids[pos] = gbase + (uint32_t)r * kSelBlock + tid;
                w[pos] = (s == 3u) ? 1.0f : (s == 1u ? t : w_o);
            }
        }
    }
}

}  // namespace

hipError_t launch_select_setup(const LevelsArg& lv, const ChunksArg& ch, int32_t mode, const lodge_camera* cam,
                              const Views& v, hipStream_t st, int32_t only_chunk)
{
    lodge_camera c{};
    if (cam) c = *cam;
    k_select_setup<<<1, 64, 0, st>>>(ch, lv, mode, c, cam ? 1 : 0, v.params, v.info, only_chunk);
    return hipGetLastError();
}

hipError_t launch_select(const LevelsArg& lv, const Views& v, const lodge_selection& sel, hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);   // an empty scene still runs (count 0)
    k_select<<<ntiles, kSelBlock, 0, st>>>(lv, v.params, ntiles, v.sel_cnt, v.sel_bits);
    return launch_select_finish(lv, v, sel, st);
}

hipError_t launch_select_finish(const LevelsArg& lv, const Views& v, const lodge_selection& sel, hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);
    k_select_scan<<<1, kSelScanThreads, 0, st>>>(v.info, v.sel_cnt, v.sel_off, ntiles, sel.cap, sel.count);
    k_select_emit<<<ntiles, kSelBlock, 0, st>>>(lv, v.params, ntiles, v.sel_cnt, v.sel_off, v.sel_bits, sel.ids,
                                                sel.w, sel.cap);
    return hipGetLastError();
}

}  // namespace lodge
