// Tile binning (LODGE Sec. 3 "Preliminaries: 3D Gaussian Splatting": each
// projected Gaussian is assigned to every 16 x 16 tile its rectangle
// overlaps; each tile's Gaussians are then depth sorted).
//
// k_scan_inst   exclusive scan of tiles-touched over the visible list
//               (single pass, decoupled look-back) -> instance offsets and
//               the instance count M.
// k_tiles       one block: 2-D prefix sums of the difference grid give each
//               tile's list length; a scan gives each tile's [start, end),
//               the emission cursors, a longest-first processing order for
//               compositing and the lists of tiles too long for the small
//               LDS sort.
// k_emit        load-balanced expansion: each thread takes instances, finds
//               its Gaussian by binary search over an LDS window of the
//               offsets, and claims a slot in its tile's run with an atomic.
//               Slot order inside a run is arbitrary; the per-tile sort
//               restores the total order (depth bits, active index).
#include "lodge_internal.hpp"

namespace lodge {

namespace {

// Decoupled look-back over 64-bit flag words: status in bits 62-63 (1 = block
// aggregate, 2 = inclusive prefix), value in bits 0-61.
constexpr unsigned long long kValMask = (1ull << 62) - 1ull;

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ unsigned long long lookback64(unsigned long long* flags, int32_t tile, uint32_t lane)
{
    unsigned long long prefix = 0;
    int32_t pred = tile - 1;
    while (true) {
        const int32_t idx = pred - (int32_t)lane;
        unsigned long long v = 2ull << 62;
        if (idx >= 0) v = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t st = (uint32_t)(v >> 62);
        if (__ballot(st == 0u) != 0ull) continue;          // a predecessor has not published yet
        const unsigned long long inc = __ballot(st == 2u);
        unsigned long long val = v & kValMask;
        if (inc != 0ull) {
            const int first = __ffsll((long long)inc) - 1;
            if ((int)lane > first) val = 0;
            prefix += wave_sum64(val);
            break;
        }
        prefix += wave_sum64(val);
        pred -= 64;
    }
    return prefix;
}

// In-place exclusive scan of vtiles[0, n_visible); total -> info->n_instances.
__global__ __launch_bounds__(kScanBlock) void k_scan_inst(FrameInfo* info, unsigned long long* flags,
                                                          uint32_t* __restrict__ vt, uint64_t max_instances)
{
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kScanBlock / 64];
    __shared__ unsigned long long s_excl;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(&info->scan_ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t n = info->n_visible;
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (tile >= ntiles) {
        if (tile == 0 && tid == 0) info->n_instances = 0;   // nothing visible
        return;
    }
    // each thread owns kScanItems consecutive items
    const uint32_t first = tile * kScanTile + tid * kScanItems;
    uint32_t x[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const uint32_t idx = first + k;
        x[k] = idx < n ? vt[idx] : 0u;
        sum += x[k];
    }
    // block exclusive scan of the per-thread sums
    uint32_t inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off);
        if ((int)lane >= off) inc += o;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t wave_excl = 0, block_total = 0;
#pragma unroll
    for (int wv = 0; wv < kScanBlock / 64; wv++) {
        const uint32_t s = s_wave[wv];
        if (wv < (int)wave) wave_excl += s;
        block_total += s;
    }
    if (wave == 0) {
        unsigned long long prefix = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&flags[0], (2ull << 62) | block_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&flags[tile], (1ull << 62) | block_total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            prefix = lookback64(flags, (int32_t)tile, lane);
            if (lane == 0)
                __hip_atomic_store(&flags[tile], (2ull << 62) | (prefix + block_total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_excl = prefix;
            if (tile == ntiles - 1) {
                const unsigned long long M = prefix + block_total;
                info->n_instances = M;
                if (M > max_instances) atomicOr(&info->overflow, kOvfInstances);
            }
        }
    }
    __syncthreads();
    // offsets only matter when M fits the instance capacity (< 2^32)
    uint32_t run = (uint32_t)s_excl + wave_excl + (inc - sum);
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        const uint32_t idx = first + k;
        if (idx < n) vt[idx] = run;
        run += x[k];
    }
}

// Single block: per-tile lengths from the difference grid, ranges, cursors,
// processing order (longest class first) and the long-list work queues.
constexpr int kTilesThreads = 1024;

__global__ __launch_bounds__(kTilesThreads) void k_tiles(const FrameParams* fp, FrameInfo* info,
                                                         int32_t* __restrict__ diff, uint2* __restrict__ ranges,
                                                         uint32_t* __restrict__ cursor, uint32_t* __restrict__ order,
                                                         uint32_t* __restrict__ large, uint64_t max_instances)
{
    __shared__ uint32_t s_part[kTilesThreads];
    __shared__ uint32_t s_cls[4], s_cls_base[4], s_max, s_nl, s_nh;
    const int32_t TX = fp->TX, TY = fp->TY, P = TX + 1;
    const uint32_t T = (uint32_t)(TX * TY);
    const uint32_t tid = threadIdx.x;
    if (tid < 4) s_cls[tid] = 0;
    if (tid == 0) { s_max = 0; s_nl = 0; s_nh = 0; }
    // prefix along x within each row, then along y within each column
    for (int32_t y = tid; y < TY; y += kTilesThreads) {
        int32_t run = 0;
        for (int32_t x = 0; x < TX; x++) { run += diff[y * P + x]; diff[y * P + x] = run; }
    }
    __syncthreads();
    for (int32_t x = tid; x < TX; x += kTilesThreads) {
        int32_t run = 0;
        for (int32_t y = 0; y < TY; y++) { run += diff[y * P + x]; diff[y * P + x] = run; }
    }
    __syncthreads();
    const bool ovf = info->n_instances > max_instances;
    // exclusive scan over tiles in row-major order; each thread a contiguous chunk
    const uint32_t per = (T + kTilesThreads - 1) / kTilesThreads;
    const uint32_t t0 = tid * per, t1 = min(T, t0 + per);
    uint32_t local = 0, lmax = 0;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = (uint32_t)diff[(t / TX) * P + (t % TX)];
        local += c;
        lmax = max(lmax, c);
    }
    s_part[tid] = local;
    atomicMax(&s_max, lmax);
    __syncthreads();
    for (int off = 1; off < kTilesThreads; off <<= 1) {
        const uint32_t o = tid >= (uint32_t)off ? s_part[tid - off] : 0u;
        __syncthreads();
        s_part[tid] += o;
        __syncthreads();
    }
    uint32_t run = s_part[tid] - local;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = ovf ? 0u : (uint32_t)diff[(t / TX) * P + (t % TX)];
        ranges[t] = make_uint2(run, run + c);
        cursor[t] = run;
        const uint32_t cls = c > 1024u ? 0u : (c > 256u ? 1u : (c > 64u ? 2u : 3u));
        atomicAdd(&s_cls[cls], 1u);
        if (c > (uint32_t)kSortLarge) large[T + atomicAdd(&s_nh, 1u)] = t;
        else if (c > (uint32_t)kSortSmall) large[atomicAdd(&s_nl, 1u)] = t;
        run += c;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t b = 0;
        for (int k = 0; k < 4; k++) { s_cls_base[k] = b; b += s_cls[k]; s_cls[k] = 0; }
        info->max_tile_len = s_max;
        info->n_large = s_nl;
        info->n_huge = s_nh;
    }
    __syncthreads();
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = ranges[t].y - ranges[t].x;
        const uint32_t cls = c > 1024u ? 0u : (c > 256u ? 1u : (c > 64u ? 2u : 3u));
        order[s_cls_base[cls] + atomicAdd(&s_cls[cls], 1u)] = t;
    }
}

constexpr int kEmitThreads = 256;
constexpr int kEmitItems = 4;
constexpr int kEmitChunk = kEmitThreads * kEmitItems;

__device__ __forceinline__ uint32_t upper_bound_g(const uint32_t* a, uint32_t n, uint32_t key)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit(const FrameParams* fp, const FrameInfo* info,
                                                        const uint32_t* __restrict__ off,
                                                        const uint32_t* __restrict__ vis,
                                                        const float4* __restrict__ proj,
                                                        uint32_t* __restrict__ cursor, uint32_t* __restrict__ sorted,
                                                        uint64_t max_instances)
{
    __shared__ uint32_t s_off[kEmitChunk + 1];
    __shared__ uint32_t s_lo, s_cnt;
    const uint32_t nvis = info->n_visible;
    const unsigned long long M = info->n_instances;
    if (M > max_instances || nvis == 0) return;
    const int32_t TX = fp->TX;
    const uint32_t nchunks = (uint32_t)((M + kEmitChunk - 1) / kEmitChunk);
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const uint32_t j0 = c * kEmitChunk;
        const uint32_t j1 = (uint32_t)min((unsigned long long)j0 + kEmitChunk, M);   // exclusive
        if (threadIdx.x == 0) {
            const uint32_t lo = upper_bound_g(off, nvis, j0) - 1;
            const uint32_t hi = upper_bound_g(off, nvis, j1 - 1) - 1;
            s_lo = lo;
            const uint32_t c = hi - lo + 1;   // <= kEmitChunk: every visible Gaussian has >= 1 instance
            s_cnt = c <= (uint32_t)kEmitChunk ? c : (uint32_t)kEmitChunk;
        }
        __syncthreads();
        const uint32_t lo = s_lo, cnt = s_cnt;
        for (uint32_t k = threadIdx.x; k < cnt; k += kEmitThreads) s_off[k] = off[lo + k];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kEmitItems; it++) {
            const uint32_t j = j0 + it * kEmitThreads + threadIdx.x;
            if (j < j1) {
                // last window entry with s_off <= j
                uint32_t a_lo = 0, a_hi = cnt;
                while (a_lo < a_hi) {
                    const uint32_t mid = (a_lo + a_hi) >> 1;
                    if (s_off[mid] <= j) a_lo = mid + 1; else a_hi = mid;
                }
                const uint32_t vi = lo + a_lo - 1;
                const uint32_t k = j - s_off[a_lo - 1];
                const uint32_t a = vis[vi];
                const float4 r2 = proj[3 * (size_t)a + 2];
                const uint32_t p0 = __float_as_uint(r2.z), p1 = __float_as_uint(r2.w);
                const uint32_t x0 = p0 & 0xffffu, y0 = p0 >> 16, x1 = p1 & 0xffffu;
                const uint32_t wr = x1 - x0;
                const uint32_t row = k / wr;
                const uint32_t tile = (y0 + row) * (uint32_t)TX + x0 + (k - row * wr);
                const uint32_t dst = atomicAdd(&cursor[tile], 1u);
                if (dst < max_instances) sorted[dst] = a;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_bin(const Views& v, hipStream_t st)
{
    k_scan_inst<<<v.lay.scan_tiles, kScanBlock, 0, st>>>(v.info, v.scan_flags, v.vtiles, v.max_instances);
    k_tiles<<<1, kTilesThreads, 0, st>>>(v.params, v.info, v.diff, v.ranges, v.cursor, v.order, v.large,
                                         v.max_instances);
    uint32_t blocks = (uint32_t)((v.max_instances + kEmitChunk - 1) / kEmitChunk);
    if (blocks < 1) blocks = 1;
    if (blocks > (uint32_t)kPersistentBlocks) blocks = kPersistentBlocks;
    k_emit<<<blocks, kEmitThreads, 0, st>>>(v.params, v.info, v.vtiles, v.vis, v.proj, v.cursor, v.sorted,
                                            v.max_instances);
    return hipGetLastError();
}

}  // namespace lodge
