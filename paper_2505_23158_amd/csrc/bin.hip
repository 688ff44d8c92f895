// Tile binning (LODGE Sec. 3 "Preliminaries: 3D Gaussian Splatting": each
// projected Gaussian is assigned to every 16 x 16 tile its rectangle
// overlaps; each tile's Gaussians are then depth sorted).
//
// A counting sort by tile built without device-scope atomics (which are
// slow on the die-spanning L2 of this part): block-local LDS histograms,
// coalesced column passes over a [block][tile] matrix, and LDS ranks.
//
//   k_chunk_scan  one block: exclusive scan of the per-chunk tile totals the
//                 projection wrote -> chunk offsets and the instance count M.
//   k_inst_off    per chunk (one wave): scan of the tile counts + chunk
//                 offset -> exclusive instance offsets of every active.
//   k_emit_hist   block b takes instances [b C, (b+1) C): finds each one's
//                 Gaussian by binary search over an LDS window of the
//                 offsets, writes (tile, index) pairs and its tile histogram
//                 (packed 16-bit LDS counters) as row b of the matrix.
//   k_col_sum     per tile: total count over the blocks (16 tiles x 16 row
//                 groups per block, row reads contiguous across tiles).
//   k_tile_scan   one block: exclusive scan of the tile totals -> [start,
//                 end) per tile, a longest-first processing order, the
//                 queues of tiles too long for the small LDS sort.
//   k_col_offset  per tile: running offsets down the column -> each block's
//                 first slot in each tile's run.
//   k_scatter     block b re-reads its pairs and places each at its block's
//                 offset plus an LDS rank.  Order inside a run is arbitrary;
//                 the per-tile sort restores (depth bits, active index).
#include "lodge_internal.hpp"

namespace lodge {

namespace {

// One block: exclusive scan of the per-chunk tile totals written by the
// projection (one per 64 actives) -> chunk offsets and M.  Each thread
// takes a contiguous run of chunks; the run totals are scanned in LDS.
constexpr int kChunkScanThreads = 1024;

__global__ __launch_bounds__(kChunkScanThreads) void k_chunk_scan(FrameInfo* info, uint32_t* __restrict__ csum,
                                                                 const uint32_t* __restrict__ count, uint32_t cap,
                                                                 uint64_t max_instances)
{
    __shared__ unsigned long long s_part[kChunkScanThreads];
    const uint32_t n = min(*count, cap);
    const uint32_t nc = (n + kProjChunk - 1) / kProjChunk;
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nc + kChunkScanThreads - 1) / kChunkScanThreads;
    const uint32_t c0 = min(nc, tid * per), c1 = min(nc, c0 + per);
    unsigned long long local = 0;
    for (uint32_t c = c0; c < c1; c++) local += csum[c];
    s_part[tid] = local;
    __syncthreads();
    for (int off = 1; off < kChunkScanThreads; off <<= 1) {
        const unsigned long long o = tid >= (uint32_t)off ? s_part[tid - off] : 0ull;
        __syncthreads();
        s_part[tid] += o;
        __syncthreads();
    }
    unsigned long long run = s_part[tid] - local;
    for (uint32_t c = c0; c < c1; c++) {
        const uint32_t v = csum[c];
        csum[c] = (uint32_t)run;    // offsets only matter when M fits the instance capacity (< 2^32)
        run += v;
    }
    if (tid == kChunkScanThreads - 1) {
        const unsigned long long M = s_part[tid];
        info->n_instances = M;
        if (M > max_instances) atomicOr(&info->overflow, kOvfInstances);
    }
}

// Per chunk of kProjChunk (= 64) actives, one wave: inclusive wave scan of
// their tile counts plus the chunk offset -> exclusive instance offsets, in place.
__global__ __launch_bounds__(256) void k_inst_off(const FrameInfo* info, uint32_t* __restrict__ vt,
                                                  const uint32_t* __restrict__ coff,
                                                  const uint32_t* __restrict__ count, uint32_t cap,
                                                  uint64_t max_instances)
{
    static_assert(kProjChunk == 64, "one wave per chunk");
    if (info->n_instances > max_instances) return;
    const uint32_t n = min(*count, cap);
    const uint32_t nc = (n + kProjChunk - 1) / kProjChunk;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < nc; c += waves) {
        const uint32_t a = c * kProjChunk + lane;
        const uint32_t x = a < n ? vt[a] : 0u;
        uint32_t inc = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if ((int)lane >= off) inc += o;
        }
        if (a < n) vt[a] = coff[c] + inc - x;
    }
}

__device__ __forceinline__ uint32_t upper_bound_g(const uint32_t* a, uint32_t n, uint32_t key)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t blocks_of(unsigned long long M)
{
    return (uint32_t)((M + kBinChunk - 1) / kBinChunk);
}

// 16-bit counter t of a packed LDS histogram: add 1, return the old count.
__device__ __forceinline__ uint32_t hist_inc(uint32_t* h, uint32_t t)
{
    const uint32_t sh = (t & 1u) << 4;
    return (atomicAdd(&h[t >> 1], 1u << sh) >> sh) & 0xffffu;
}

__device__ __forceinline__ uint32_t hist_get(const uint32_t* h, uint32_t t)
{
    return (h[t >> 1] >> ((t & 1u) << 4)) & 0xffffu;
}

constexpr int kBinThreads = 1024;
constexpr int kWindow = 16384;   // LDS window of instance offsets (active indices)

__global__ __launch_bounds__(kBinThreads) void k_emit_hist(const FrameParams* fp, const FrameInfo* info,
                                                           const uint32_t* __restrict__ off,
                                                           const uint32_t* __restrict__ count, uint32_t cap,
                                                           const uint2* __restrict__ rect, uint2* __restrict__ inst,
                                                           uint32_t* __restrict__ hist, uint64_t max_instances)
{
    __shared__ uint32_t s_hist[kMaxTiles / 2];
    __shared__ uint32_t s_off[kWindow];
    __shared__ uint32_t s_lo, s_cnt;
    const unsigned long long M = info->n_instances;
    if (M == 0 || M > max_instances) return;
    const uint32_t n_act = min(*count, cap);
    const int32_t TX = fp->TX;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t B = blocks_of(M);
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const uint32_t j0 = b * kBinChunk;
        const uint32_t j1 = (uint32_t)min((unsigned long long)j0 + kBinChunk, M);
        for (uint32_t k = threadIdx.x; k < (T + 1) / 2; k += kBinThreads) s_hist[k] = 0;
        if (threadIdx.x == 0) {
            const uint32_t lo = upper_bound_g(off, n_act, j0) - 1;
            const uint32_t hi = upper_bound_g(off, n_act, j1 - 1) - 1;
            s_lo = lo;
            s_cnt = hi - lo + 1;
        }
        __syncthreads();
        const uint32_t lo = s_lo, cnt = s_cnt;
        const bool in_lds = cnt <= (uint32_t)kWindow;
        if (in_lds)
            for (uint32_t k = threadIdx.x; k < cnt; k += kBinThreads) s_off[k] = off[lo + k];
        __syncthreads();
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += kBinThreads) {
            // last active index whose offset is <= j (zero-tile entries share offsets: take the last)
            uint32_t a;
            if (in_lds) {
                uint32_t l = 0, h = cnt;
                while (l < h) {
                    const uint32_t mid = (l + h) >> 1;
                    if (s_off[mid] <= j) l = mid + 1; else h = mid;
                }
                a = lo + l - 1;
            } else {
                a = upper_bound_g(off, n_act, j) - 1;
            }
            const uint32_t k = j - off[a];
            const uint2 rc = rect[a];
            const uint32_t p0 = rc.x, p1 = rc.y;
            const uint32_t x0 = p0 & 0xffffu, y0 = p0 >> 16, wr = (p1 & 0xffffu) - x0;
            const uint32_t row = k / wr;
            const uint32_t tile = (y0 + row) * (uint32_t)TX + x0 + (k - row * wr);
            inst[j] = make_uint2(tile, a);
            hist_inc(s_hist, tile);
        }
        __syncthreads();
        uint32_t* row_out = hist + (size_t)b * T;
        for (uint32_t t = threadIdx.x; t < T; t += kBinThreads) row_out[t] = hist_get(s_hist, t);
        __syncthreads();
    }
}

// Column passes over the [B][T] matrix: a block takes 16 tiles x 16 groups
// of consecutive rows, so row reads are contiguous across the tile lanes and
// every tile's column is walked by 16 threads at once.
constexpr int kColTiles = 16, kColGroups = 16;

// tile totals
__global__ __launch_bounds__(256) void k_col_sum(const FrameParams* fp, const FrameInfo* info,
                                                 const uint32_t* __restrict__ hist, uint32_t* __restrict__ tcount,
                                                 uint64_t max_instances)
{
    __shared__ uint32_t s_part[kColGroups][kColTiles];
    const unsigned long long M = info->n_instances;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t tl = threadIdx.x % kColTiles, g = threadIdx.x / kColTiles;
    const uint32_t t = blockIdx.x * kColTiles + tl;
    uint32_t s = 0;
    if (t < T && M <= max_instances) {
        const uint32_t B = blocks_of(M);
        const uint32_t R = (B + kColGroups - 1) / kColGroups;
        const uint32_t b0 = g * R, b1 = min(B, b0 + R);
        for (uint32_t b = b0; b < b1; b++) s += hist[(size_t)b * T + t];
    }
    s_part[g][tl] = s;
    __syncthreads();
    if (g == 0 && t < T) {
        uint32_t tot = 0;
        for (int k = 0; k < kColGroups; k++) tot += s_part[k][tl];
        tcount[t] = tot;
    }
}

// per-(block, tile) first slot: tile start + running count down the column
__global__ __launch_bounds__(256) void k_col_offset(const FrameParams* fp, const FrameInfo* info,
                                                    const uint2* __restrict__ ranges, uint32_t* __restrict__ hist,
                                                    uint64_t max_instances)
{
    __shared__ uint32_t s_part[kColGroups][kColTiles];
    const unsigned long long M = info->n_instances;
    if (M == 0 || M > max_instances) return;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t tl = threadIdx.x % kColTiles, g = threadIdx.x / kColTiles;
    const uint32_t t = blockIdx.x * kColTiles + tl;
    const uint32_t B = blocks_of(M);
    const uint32_t R = (B + kColGroups - 1) / kColGroups;
    const uint32_t b0 = min(B, g * R), b1 = min(B, b0 + R);
    uint32_t s = 0;
    if (t < T)
        for (uint32_t b = b0; b < b1; b++) s += hist[(size_t)b * T + t];
    s_part[g][tl] = s;
    __syncthreads();
    if (t >= T) return;
    uint32_t run = ranges[t].x;
    for (uint32_t k = 0; k < g; k++) run += s_part[k][tl];
    for (uint32_t b = b0; b < b1; b++) {
        const size_t i = (size_t)b * T + t;
        const uint32_t c = hist[i];
        hist[i] = run;
        run += c;
    }
}

// One block: exclusive scan of the tile totals -> ranges, processing order,
// long-list queues, longest list.
constexpr int kTilesThreads = 1024;

__global__ __launch_bounds__(kTilesThreads) void k_tile_scan(const FrameParams* fp, FrameInfo* info,
                                                             const uint32_t* __restrict__ tcount,
                                                             uint2* __restrict__ ranges, uint32_t* __restrict__ order,
                                                             uint32_t* __restrict__ large)
{
    __shared__ uint32_t s_part[kTilesThreads];
    __shared__ uint32_t s_cls[4], s_cls_base[4], s_max, s_nl, s_nh;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t tid = threadIdx.x;
    if (tid < 4) s_cls[tid] = 0;
    if (tid == 0) { s_max = 0; s_nl = 0; s_nh = 0; }
    const uint32_t per = (T + kTilesThreads - 1) / kTilesThreads;
    const uint32_t t0 = min(T, tid * per), t1 = min(T, t0 + per);
    uint32_t local = 0, lmax = 0;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = tcount[t];
        local += c;
        lmax = max(lmax, c);
    }
    s_part[tid] = local;
    __syncthreads();
    atomicMax(&s_max, lmax);
    for (int off = 1; off < kTilesThreads; off <<= 1) {
        const uint32_t o = tid >= (uint32_t)off ? s_part[tid - off] : 0u;
        __syncthreads();
        s_part[tid] += o;
        __syncthreads();
    }
    uint32_t run = s_part[tid] - local;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = tcount[t];
        ranges[t] = make_uint2(run, run + c);
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
        const uint32_t c = tcount[t];
        const uint32_t cls = c > 1024u ? 0u : (c > 256u ? 1u : (c > 64u ? 2u : 3u));
        order[s_cls_base[cls] + atomicAdd(&s_cls[cls], 1u)] = t;
    }
}

__global__ __launch_bounds__(kBinThreads) void k_scatter(const FrameParams* fp, const FrameInfo* info,
                                                         const uint2* __restrict__ inst,
                                                         const uint32_t* __restrict__ hist,
                                                         uint32_t* __restrict__ sorted, uint64_t max_instances)
{
    __shared__ uint32_t s_rank[kMaxTiles / 2];
    const unsigned long long M = info->n_instances;
    if (M == 0 || M > max_instances) return;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t B = blocks_of(M);
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const uint32_t j0 = b * kBinChunk;
        const uint32_t j1 = (uint32_t)min((unsigned long long)j0 + kBinChunk, M);
        for (uint32_t k = threadIdx.x; k < (T + 1) / 2; k += kBinThreads) s_rank[k] = 0;
        __syncthreads();
        const uint32_t* row = hist + (size_t)b * T;
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += kBinThreads) {
            const uint2 e = inst[j];
            const uint32_t slot = row[e.x] + hist_inc(s_rank, e.x);
            if (slot < max_instances) sorted[slot] = e.y;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_bin(const Views& v, const lodge_selection& sel, hipStream_t st)
{
    k_chunk_scan<<<1, kChunkScanThreads, 0, st>>>(v.info, v.chunk_sum, sel.count, sel.cap, v.max_instances);
    const uint32_t cg = std::max<uint32_t>(1, std::min<uint32_t>(4096, (v.max_active + 255) / 256));
    k_inst_off<<<cg, 256, 0, st>>>(v.info, v.vtiles, v.chunk_sum, sel.count, sel.cap, v.max_instances);
    const uint32_t bmax = std::max<uint32_t>(1, (uint32_t)((v.max_instances + kBinChunk - 1) / kBinChunk));
    const uint32_t grid = std::min<uint32_t>(bmax, 1024);
    k_emit_hist<<<grid, kBinThreads, 0, st>>>(v.params, v.info, v.vtiles, sel.count, sel.cap, v.rect, v.inst, v.hist,
                                              v.max_instances);
    const uint32_t tb = (v.lay.T + kColTiles - 1) / kColTiles;
    k_col_sum<<<tb, 256, 0, st>>>(v.params, v.info, v.hist, v.tcount, v.max_instances);
    k_tile_scan<<<1, kTilesThreads, 0, st>>>(v.params, v.info, v.tcount, v.ranges, v.order, v.large);
    k_col_offset<<<tb, 256, 0, st>>>(v.params, v.info, v.ranges, v.hist, v.max_instances);
    k_scatter<<<grid, kBinThreads, 0, st>>>(v.params, v.info, v.inst, v.hist, v.sorted, v.max_instances);
    return hipGetLastError();
}

}  // namespace lodge
