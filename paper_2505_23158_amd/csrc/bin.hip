// Tile binning (LODGE Sec. 3 "Preliminaries: 3D Gaussian Splatting": each
// projected Gaussian is assigned to every 16 x 16 tile its rectangle
// overlaps; each tile's Gaussians are then depth sorted).
//
// A counting sort by tile: block-local LDS histograms and LDS ranks, with
// device-scope atomics only where they are few (one per binning block and
// tile it touches, about 200 blocks x a few hundred tiles at 1080p).
//
//   k_chunk_scan  exclusive scans of the per-chunk totals the projection
//                 wrote (tiles; actives with a tile): offsets inside blocks
//                 of 4096 chunks, then, in the last block to finish, the
//                 blocks' offsets, the instance count M and the binned
//                 count; clears the tile totals.
//   k_inst_off    per chunk (one wave): scan of the tile counts + chunk
//                 offset -> exclusive instance offsets; the actives with a
//                 tile are compacted in index order as (first instance,
//                 index), and each binning block gets the compacted slot its
//                 first instance belongs to.
//   k_emit_hist   block b takes instances [b C, (b+1) C): finds each one's
//                 Gaussian by binary search over an LDS window of the
//                 compacted offsets (at most C + 1 of them, since every
//                 compacted active has an instance), writes (tile, index)
//                 pairs and counts them per tile (packed 16-bit LDS
//                 counters); for each tile it touched, one atomic add of its
//                 count to the tile total returns the block's first slot
//                 inside the tile's run (row b of the [block][tile] matrix).
//   k_tile_scan   one block: exclusive scan of the tile totals -> [start,
//                 end) per tile, a longest-first processing order, the
//                 queues of tiles too long for the small LDS sort.
//   k_scatter     block b re-reads its pairs and places each at its tile's
//                 start + its block's slot + an LDS rank.  Order inside a run
//                 is arbitrary; the per-tile sort restores (depth bits,
//                 active index).
#include "lodge_internal.hpp"

namespace lodge {

namespace {

// Exclusive scans of the two per-chunk totals the projection wrote (one
// chunk per 64 actives): tiles -> chunk instance offsets and M; actives with
// a tile -> chunk offsets of their compaction.  Block b takes chunks
// [b kScanChunks, (b + 1) kScanChunks), 4 per thread (coalesced uint4), and
// writes offsets local to the block plus its two totals; the last block to
// finish (one atomic per block, no waiting) scans the block totals into
// per-block offsets, M and the binned count.  Consumers add the block offset.
constexpr int kChunkScanThreads = 1024;
static_assert(kScanChunks == 4 * kChunkScanThreads, "four chunks per thread");

__device__ __forceinline__ uint4 load4(const uint32_t* __restrict__ p, uint32_t c, uint32_t nc)
{
    if (c + 3 < nc) return *reinterpret_cast<const uint4*>(p + c);
    return make_uint4(c < nc ? p[c] : 0u, c + 1 < nc ? p[c + 1] : 0u, c + 2 < nc ? p[c + 2] : 0u, 0u);
}

__device__ __forceinline__ void store4(uint32_t* __restrict__ p, uint32_t c, uint32_t nc, uint4 v)
{
    if (c + 3 < nc) {
        *reinterpret_cast<uint4*>(p + c) = v;
    } else {
        if (c < nc) p[c] = v.x;
        if (c + 1 < nc) p[c + 1] = v.y;
        if (c + 2 < nc) p[c + 2] = v.z;
    }
}

__global__ __launch_bounds__(kChunkScanThreads) void k_chunk_scan(const FrameParams* fp, FrameInfo* info,
                                                                 uint32_t* __restrict__ csum,
                                                                 uint32_t* __restrict__ cvis, uint4* blk,
                                                                 const uint32_t* __restrict__ count, uint32_t cap,
                                                                 uint32_t* __restrict__ tcount, uint64_t max_instances)
{
    constexpr int NW = kChunkScanThreads / 64, kPer = 8;
    __shared__ uint32_t s_w[2][NW];
    __shared__ unsigned long long s_t[NW];
    __shared__ uint32_t s_last;
    const uint32_t n = min(*count, cap);
    const uint32_t nc = (n + kProjChunk - 1) / kProjChunk;
    const uint32_t nb = max(1u, (nc + kScanChunks - 1) / kScanChunks);   // block 0 runs even with no chunk
    const uint32_t b = blockIdx.x;
    if (b >= nb) return;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (b == 0) {
        // tile totals: accumulated by the binning blocks' atomics
        const uint32_t T = (uint32_t)(fp->TX * fp->TY);
        for (uint32_t t = tid; t < T; t += kChunkScanThreads) tcount[t] = 0;
    }
    const uint32_t c = b * kScanChunks + 4 * tid;
    const uint4 v = load4(csum, c, nc), w = load4(cvis, c, nc);
    const uint32_t own = (v.x + v.y) + (v.z + v.w), vown = (w.x + w.y) + (w.z + w.w);
    uint32_t inc = own, vinc = vown;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o), vu = __shfl_up(vinc, o);
        if ((int)lane >= o) {
            inc += u;
            vinc += vu;
        }
    }
    if (lane == 63) {
        s_w[0][wave] = inc;
        s_w[1][wave] = vinc;
    }
    __syncthreads();
    uint32_t before = 0, vbefore = 0, vtotal = 0;
    unsigned long long total = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
        const uint32_t x = s_w[0][k], y = s_w[1][k];
        before += (uint32_t)k < wave ? x : 0u;
        total += x;
        vbefore += (uint32_t)k < wave ? y : 0u;
        vtotal += y;
    }
    // offsets only matter when M fits the instance capacity (< 2^32)
    const uint32_t e0 = before + inc - own, f0 = vbefore + vinc - vown;
    store4(csum, c, nc, make_uint4(e0, e0 + v.x, e0 + v.x + v.y, e0 + v.x + v.y + v.z));
    store4(cvis, c, nc, make_uint4(f0, f0 + w.x, f0 + w.x + w.y, f0 + w.x + w.y + w.z));
    if (tid == 0) {
        blk[b] = make_uint4((uint32_t)total, (uint32_t)(total >> 32), vtotal, 0u);
        __threadfence();   // the totals are visible before the count says so
        s_last = atomicAdd(&info->scan_done, 1u) == nb - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (s_last == 0u) return;
    // the last block: exclusive scan of the nb block totals, kPer per thread
    // (nb <= kPer x 1024 for any max_active < 2^31)
    __threadfence();
    const volatile uint4* vb = blk;
    const uint32_t per = (nb + kChunkScanThreads - 1) / kChunkScanThreads;
    const uint32_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    unsigned long long bt[kPer];
    uint32_t bv[kPer];
    unsigned long long st = 0;
    uint32_t sv = 0;
#pragma unroll
    for (int q = 0; q < kPer; q++) {
        bt[q] = 0;
        bv[q] = 0;
        if (b0 + q < b1) {
            const uint32_t lo = vb[b0 + q].x, hi = vb[b0 + q].y;
            bt[q] = ((unsigned long long)hi << 32) | lo;
            bv[q] = vb[b0 + q].z;
        }
        st += bt[q];
        sv += bv[q];
    }
    unsigned long long it = st;
    uint32_t iv = sv;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long ut = __shfl_up(it, o);
        const uint32_t uv = __shfl_up(iv, o);
        if ((int)lane >= o) {
            it += ut;
            iv += uv;
        }
    }
    __syncthreads();
    if (lane == 63) {
        s_t[wave] = it;
        s_w[1][wave] = iv;
    }
    __syncthreads();
    unsigned long long tb = 0, tt = 0;
    uint32_t vb0 = 0, vt = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) {
        tb += (uint32_t)k < wave ? s_t[k] : 0ull;
        tt += s_t[k];
        vb0 += (uint32_t)k < wave ? s_w[1][k] : 0u;
        vt += s_w[1][k];
    }
    unsigned long long rt = tb + it - st;
    uint32_t rv = vb0 + iv - sv;
#pragma unroll
    for (int q = 0; q < kPer; q++)
        if (b0 + q < b1) {
            blk[b0 + q] = make_uint4((uint32_t)rt, rv, 0u, 0u);
            rt += bt[q];
            rv += bv[q];
        }
    if (tid == 0) {
        info->n_instances = tt;
        info->n_binned = vt;
        if (tt > max_instances) atomicOr(&info->overflow, kOvfInstances);
    }
}

// Per chunk of kProjChunk (= 64) actives, one wave: inclusive wave scan of
// their tile counts plus the chunk offset -> exclusive instance offsets; the
// actives with a tile are compacted, in index order, into (vis_off, vis_id).
__global__ __launch_bounds__(256) void k_inst_off(const FrameInfo* info, const uint32_t* __restrict__ vt,
                                                  const uint32_t* __restrict__ coff,
                                                  const uint32_t* __restrict__ cvis,
                                                  const uint4* __restrict__ blk,
                                                  const uint32_t* __restrict__ count, uint32_t cap,
                                                  uint32_t* __restrict__ vis_off, uint32_t* __restrict__ vis_id,
                                                  uint32_t* __restrict__ bstart, uint64_t max_instances)
{
    static_assert(kProjChunk == 64, "one wave per chunk");
    if (info->n_instances > max_instances) return;
    const uint32_t n = min(*count, cap);
    const uint32_t nc = (n + kProjChunk - 1) / kProjChunk;
    const uint32_t lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < nc; c += waves) {
        const uint32_t a = c * kProjChunk + lane;
        const uint32_t x = a < n ? __builtin_nontemporal_load(vt + a) : 0u;   // read once
        uint32_t inc = x;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if ((int)lane >= off) inc += o;
        }
        const uint4 bo = blk[c / kScanChunks];   // the chunk-scan block's offsets
        const uint32_t o = bo.x + coff[c] + inc - x;
        const unsigned long long m = __ballot(x > 0u);
        if (x > 0u) {
            const uint32_t s = bo.y + cvis[c] + (uint32_t)__popcll(m & lt);
            vis_off[s] = o;
            vis_id[s] = a;
            // the binning block starting at instance b kBinChunk is owned by
            // the active whose run [o, o + x) holds that instance
            for (uint32_t b = (o + kBinChunk - 1) / kBinChunk; (unsigned long long)b * kBinChunk < o + x; b++)
                bstart[b] = s;
        }
    }
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
// Every compacted active holds at least one instance, so a binning block's
// instances belong to at most kBinChunk + 1 of them.
constexpr uint32_t kWindow = kBinChunk + 1;

// Dynamic LDS of the binning kernels, sized for the frame's tile count so
// that two blocks share a compute unit at 1080p: the tile histogram (16-bit
// counters, (T + 1) / 2 words), then for k_emit_hist the offset and id windows.
__host__ __device__ constexpr uint32_t emit_lds_words(uint32_t T) { return (T + 1) / 2 + 2 * kWindow; }
__host__ __device__ constexpr uint32_t scatter_lds_words(uint32_t T) { return (T + 1) / 2; }

// last index i in [0, n) with a[i] <= key (a ascending, a[0] <= key)
__device__ __forceinline__ uint32_t last_le(const uint32_t* a, uint32_t n, uint32_t key)
{
    uint32_t l = 0, h = n;
    while (l < h) {
        const uint32_t mid = (l + h) >> 1;
        if (a[mid] <= key) l = mid + 1; else h = mid;
    }
    return l - 1;
}

__global__ __launch_bounds__(kBinThreads) void k_emit_hist(const FrameParams* fp, const FrameInfo* info,
                                                           const uint32_t* __restrict__ vis_off,
                                                           const uint32_t* __restrict__ vis_id,
                                                           const uint32_t* __restrict__ bstart,
                                                           const uint2* __restrict__ rect, uint2* __restrict__ inst,
                                                           uint32_t* __restrict__ hist, uint32_t* __restrict__ tcount,
                                                           uint64_t max_instances)
{
    constexpr int kPer = kBinChunk / kBinThreads;   // instances per thread, processed together
    extern __shared__ uint32_t s_lds[];   // emit_lds_words(T)
    const unsigned long long M = info->n_instances;
    if (M == 0 || M > max_instances) return;
    const uint32_t n_bin = info->n_binned;
    const int32_t TX = fp->TX;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t B = blocks_of(M);
    // packed 16-bit tile counters first (T <= kMaxTiles), then the windows
    uint32_t* const s_hist = s_lds;
    uint32_t* const s_off = s_lds + (T + 1) / 2;
    uint32_t* const s_id = s_off + kWindow;
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const uint32_t j0 = b * kBinChunk;
        const uint32_t j1 = (uint32_t)min((unsigned long long)j0 + kBinChunk, M);
        for (uint32_t k = threadIdx.x; k < (T + 1) / 2; k += kBinThreads) s_hist[k] = 0;
        // compacted actives [lo, hi] hold the block's instances (hi may be one past the last)
        const uint32_t lo = bstart[b];
        const uint32_t hi = b + 1 < B ? bstart[b + 1] : n_bin - 1;
        const uint32_t cnt = min(hi - lo + 1, kWindow);
        // the window: every load of a pass issued before its LDS stores
        for (uint32_t k0 = 0; k0 < cnt; k0 += kPer * kBinThreads) {
            uint32_t o[kPer], g[kPer];
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                const uint32_t k = k0 + q * kBinThreads + threadIdx.x;
                o[q] = k < cnt ? __builtin_nontemporal_load(vis_off + lo + k) : 0u;   // read once
                g[q] = k < cnt ? __builtin_nontemporal_load(vis_id + lo + k) : 0u;
            }
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                const uint32_t k = k0 + q * kBinThreads + threadIdx.x;
                if (k < cnt) {
                    s_off[k] = o[q];
                    s_id[k] = g[q];
                }
            }
        }
        __syncthreads();
        // each instance's active: the last whose first instance is <= it
        uint32_t a[kPer], kk[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint32_t j = j0 + threadIdx.x + q * kBinThreads;
            a[q] = 0;
            kk[q] = 0;
            if (j < j1) {
                const uint32_t l = last_le(s_off, cnt, j);
                a[q] = s_id[l];
                kk[q] = j - s_off[l];
            }
        }
        uint2 rc[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) rc[q] = rect[a[q]];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint32_t j = j0 + threadIdx.x + q * kBinThreads;
            if (j >= j1) continue;
            const uint32_t x0 = rc[q].x & 0xffffu, y0 = rc[q].x >> 16, wr = (rc[q].y & 0xffffu) - x0;
            const uint32_t row = kk[q] / wr;
            const uint32_t tile = (y0 + row) * (uint32_t)TX + x0 + (kk[q] - row * wr);
            inst[j] = make_uint2(tile, a[q]);
            hist_inc(s_hist, tile);
        }
        __syncthreads();
        // the block's first slot in each touched tile's run (the order of
        // blocks inside a run is that of the atomics; the sort restores it)
        // (eight atomics in flight per thread before their results are stored)
        uint32_t* row_out = hist + (size_t)b * T;
        for (uint32_t t0 = 0; t0 < T; t0 += 8 * kBinThreads) {
            uint32_t c[8], r[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const uint32_t t = t0 + q * kBinThreads + threadIdx.x;
                c[q] = t < T ? hist_get(s_hist, t) : 0u;
            }
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const uint32_t t = t0 + q * kBinThreads + threadIdx.x;
                r[q] = c[q] != 0u ? atomicAdd(&tcount[t], c[q]) : 0u;
            }
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const uint32_t t = t0 + q * kBinThreads + threadIdx.x;
                if (c[q] != 0u) row_out[t] = r[q];
            }
        }
        __syncthreads();
    }
}

// One block: exclusive scan of the tile totals -> ranges, processing order,
// long-list queues, longest list.
constexpr int kTilesThreads = 1024;

// Sort queue of a tile list, as one unit in a packed count of four 16-bit
// fields (T <= kMaxTiles < 2^16): (kSortSmall, kSortMid] in bits 0-15, huge
// (above kSortLarge) in 16-31, mid (kSortWave, kSortSmall] in 32-47, and
// (kSortMid, kSortLarge] in 48-63.
constexpr unsigned long long kQMask = 0xffffull;
__device__ __forceinline__ unsigned long long queue_unit(uint32_t c)
{
    return c > (uint32_t)kSortLarge ? 1ull << 16
         : c > (uint32_t)kSortMid   ? 1ull << 48
         : c > (uint32_t)kSortSmall ? 1ull : c > (uint32_t)kSortWave ? 1ull << 32 : 0ull;
}

// Length class of a tile list in the compositing order (longest first).
__device__ __forceinline__ uint32_t length_class(uint32_t c)
{
    return c > 1024u ? 0u : (c > 256u ? 1u : (c > 64u ? 2u : 3u));
}

// Exclusive scan over the block of three 64-bit values at once (wave scans,
// wave totals in LDS, two barriers); returns the prefixes and the totals.
template <int NT>
__device__ __forceinline__ void block_scan3(unsigned long long (&v)[3], unsigned long long (*s_w)[NT / 64],
                                            unsigned long long (&total)[3])
{
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long inc[3] = {v[0], v[1], v[2]};
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const unsigned long long u = __shfl_up(inc[c], o);
            if ((int)lane >= o) inc[c] += u;
        }
    }
    if (lane == 63)
        for (int c = 0; c < 3; c++) s_w[c][wave] = inc[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; c++) {
        unsigned long long before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; w++) {
            const unsigned long long x = s_w[c][w];
            before += (uint32_t)w < wave ? x : 0ull;
            tot += x;
        }
        total[c] = tot;
        v[c] = before + inc[c] - v[c];
    }
    __syncthreads();
}

// One block over all tiles, each thread a contiguous run of them:
// exclusive scan of the list lengths -> [start, end) per tile;
// the compositing order (four length classes, longest first, tile order
// inside a class) and the queues of lists too long for the per-tile LDS
// sort, all placed by scans of packed per-thread counts (no atomics).
__global__ __launch_bounds__(kTilesThreads) void k_tile_scan(const FrameParams* fp, FrameInfo* info,
                                                             const uint32_t* __restrict__ tcount,
                                                             uint2* __restrict__ ranges, uint32_t* __restrict__ order,
                                                             uint32_t* __restrict__ large)
{
    __shared__ unsigned long long s_w[3][kTilesThreads / 64];
    __shared__ uint32_t s_max[kTilesThreads / 64];
    __shared__ uint32_t s_c[kMaxTiles];   // 128 KB: this kernel is one block
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (T + kTilesThreads - 1) / kTilesThreads;
    const uint32_t t0 = min(T, tid * per), t1 = min(T, t0 + per);
    // the tile totals staged in LDS by coalesced loads, eight in flight per
    // thread, so the per-thread runs below read LDS, not global memory
    for (uint32_t g0 = 0; g0 < T; g0 += 8 * kTilesThreads) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const uint32_t t = g0 + q * kTilesThreads + tid;
            v[q] = t < T ? tcount[t] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const uint32_t t = g0 + q * kTilesThreads + tid;
            if (t < T) s_c[t] = v[q];
        }
    }
    __syncthreads();
    // cls: four 16-bit length-class counts; big: four 16-bit queue counts
    // (bits 0-15 runs in (2048, 4096], 16-31 over 16384, 32-47 in (256, 2048],
    // 48-63 in (4096, 16384]; see queue_unit)
    unsigned long long sum = 0, cls = 0, big = 0;
    uint32_t lmax = 0;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = s_c[t];
        sum += c;
        lmax = max(lmax, c);
        cls += 1ull << (16 * length_class(c));
        big += queue_unit(c);
    }
    for (int o = 32; o > 0; o >>= 1) lmax = max(lmax, (uint32_t)__shfl_xor(lmax, o));
    if (lane == 0) s_max[wave] = lmax;
    unsigned long long sc[3] = {sum, cls, big}, tot[3];
    block_scan3<kTilesThreads>(sc, s_w, tot);
    unsigned long long run = sc[0], cpos = sc[1];
    const unsigned long long bpos = sc[2], cls_tot = tot[1], big_tot = tot[2];
    uint32_t base[4];
    {
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            base[k] = b;
            b += (uint32_t)(cls_tot >> (16 * k)) & 0xffffu;
        }
    }
    uint32_t nl = (uint32_t)(bpos & kQMask), nh = (uint32_t)((bpos >> 16) & kQMask),
             nm = (uint32_t)((bpos >> 32) & kQMask), nx = (uint32_t)((bpos >> 48) & kQMask);
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t c = s_c[t];
        // offsets only matter when the total fits the instance capacity (< 2^32)
        ranges[t] = make_uint2((uint32_t)run, (uint32_t)(run + c));
        run += c;
        const uint32_t q = length_class(c);
        order[base[q] + ((uint32_t)(cpos >> (16 * q)) & 0xffffu)] = t;
        cpos += 1ull << (16 * q);
        // (kSortMid, kSortLarge] fills the first region from its end
        if (c > (uint32_t)kSortLarge) large[T + nh++] = t;
        else if (c > (uint32_t)kSortMid) large[T - 1 - nx++] = t;
        else if (c > (uint32_t)kSortSmall) large[nl++] = t;
        else if (c > (uint32_t)kSortWave) large[2 * T + nm++] = t;
    }
    if (tid == 0) {
        uint32_t m = 0;
        for (int w = 0; w < kTilesThreads / 64; w++) m = max(m, s_max[w]);
        info->max_tile_len = m;
        info->n_large = (uint32_t)(big_tot & kQMask);
        info->n_huge = (uint32_t)((big_tot >> 16) & kQMask);
        info->n_mid = (uint32_t)((big_tot >> 32) & kQMask);
        info->n_xl = (uint32_t)((big_tot >> 48) & kQMask);
    }
}

__global__ __launch_bounds__(kBinThreads) void k_scatter(const FrameParams* fp, const FrameInfo* info,
                                                         const uint2* __restrict__ inst,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint2* __restrict__ ranges,
                                                         uint32_t* __restrict__ sorted, uint64_t max_instances)
{
    extern __shared__ uint32_t s_lds[];   // scatter_lds_words(T)
    uint32_t* const s_rank = s_lds;
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
        // the block's instances, kPer per thread: each round of loads is
        // issued before any of its results is used
        constexpr int kPer = kBinChunk / kBinThreads;
        uint2 e[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint32_t j = j0 + q * kBinThreads + threadIdx.x;
            unsigned long long v = 0;
            if (j < j1) v = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(inst) + j);   // read once
            e[q] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
        }
        uint32_t base[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint32_t j = j0 + q * kBinThreads + threadIdx.x;
            base[q] = j < j1 ? ranges[e[q].x].x + row[e[q].x] : 0u;
        }
#pragma unroll
        for (int q = 0; q < kPer; q++) {
            const uint32_t j = j0 + q * kBinThreads + threadIdx.x;
            if (j < j1) {
                const uint32_t slot = base[q] + hist_inc(s_rank, e[q].x);
                if (slot < max_instances) sorted[slot] = e[q].y;
            }
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_bin(const Views& v, const lodge_selection& sel, hipStream_t st)
{
    const uint32_t sb = std::max<uint32_t>(1, ((v.max_active + kProjChunk - 1) / kProjChunk + kScanChunks - 1) / kScanChunks);
    k_chunk_scan<<<sb, kChunkScanThreads, 0, st>>>(v.params, v.info, v.chunk_sum, v.chunk_vis, v.scan_blk, sel.count,
                                                   sel.cap, v.tcount, v.max_instances);
    const uint32_t cg = std::max<uint32_t>(1, std::min<uint32_t>(4096, (v.max_active + 255) / 256));
    k_inst_off<<<cg, 256, 0, st>>>(v.info, v.vtiles, v.chunk_sum, v.chunk_vis, v.scan_blk, sel.count, sel.cap,
                                   v.vis_off, v.vis_id, v.bstart, v.max_instances);
    const uint32_t bmax = std::max<uint32_t>(1, (uint32_t)((v.max_instances + kBinChunk - 1) / kBinChunk));
    const uint32_t grid = std::min<uint32_t>(bmax, 1024);
    // more than 64 KB of dynamic LDS must be allowed explicitly (up to 4K frames)
    static thread_local int dev_cached = -1;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != dev_cached) {
        if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_emit_hist),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(4 * emit_lds_words(kMaxTiles)))) != hipSuccess)
            return e;
        dev_cached = dev;
    }
    k_emit_hist<<<grid, kBinThreads, 4 * emit_lds_words(v.lay.T), st>>>(v.params, v.info, v.vis_off, v.vis_id,
                                                                         v.bstart, v.rect, v.inst, v.hist, v.tcount,
                                                                         v.max_instances);
    k_tile_scan<<<1, kTilesThreads, 0, st>>>(v.params, v.info, v.tcount, v.ranges, v.order, v.large);
    k_scatter<<<grid, kBinThreads, 4 * scatter_lds_words(v.lay.T), st>>>(v.params, v.info, v.inst, v.hist, v.ranges,
                                                                          v.sorted, v.max_instances);
    return hipGetLastError();
}

}  // namespace lodge
