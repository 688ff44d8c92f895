// Per-tile sort of the binned instances (LODGE Sec. 3 "Preliminaries":
// the Gaussians of each tile are sorted in depth before blending).
//
// Each tile's run holds active indices in arbitrary order.  The key of
// index a is (float bits of its camera depth) << 32 | a: depth > znear > 0,
// so the bit pattern orders like the value, and the index makes the order
// total (ties in depth are broken by active index, i.e. by global id).
//
// Short runs are sorted by bitonic networks held in registers: each thread
// keeps E consecutive keys; stages whose partner is in the same thread
// compare registers, and stages whose partner is in another lane exchange
// keys with lane permutes (DPP quad permutes, swizzles, gfx950 lane swaps).
// Longer runs are cut into 512-key pieces, each sorted by one wave in
// registers, and the pieces are merged in LDS by merge-path rounds.  One
// launch, k_sort, sorts every run, by length band:
//   <= 256         one wave, 1-4 keys per lane: no LDS, no barrier;
//   (256, 2048]    four waves: 512-key wave sorts, two merge rounds;
//   (2048, 4096]   eight waves: 512-key wave sorts, three merge rounds;
//   (4096, 8192]   both halves sorted so, then one merge-path merge of the
//                  two from the block's 64 KB of LDS into the run;
//   > 8192         8192-key chunks sorted so, then merge passes in
//                  global memory where each key finds its output slot by
//                  binary search in the sibling run.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

constexpr int kSortThreads = 512;
constexpr int kSortLds = 8192;   // keys of LDS per block (64 KB): two blocks per compute unit

// Indices come from the emission pass; one outside [0, cap) would be a
// binning bug, so it sorts last instead of being dereferenced.
__device__ __forceinline__ unsigned long long key_of(const float* __restrict__ depth, uint32_t a, uint32_t cap)
{
    if (a >= cap) return ~0ull;
    return ((unsigned long long)__float_as_uint(depth[a]) << 32) | a;
}

// 32-bit value of lane (lane ^ D) of the wave.  Distances 1 and 2 are quad
// permutes (DPP); 4 and 8 are swizzles through the LDS unit (no memory
// access, and no VALU slot, which this VALU-bound network is short of); 16
// and 32 are gfx950 lane-swaps of the value with a copy of
// itself (permlane16_swap trades rows 1 and 3 of the first operand with rows
// 0 and 2 of the second, permlane32_swap the upper half of the first with the
// lower half of the second), after which the partner's value sits in the
// second result below the swapped boundary and in the first above it.
template <int D>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    if constexpr (D == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    } else if constexpr (D == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else if constexpr (D == 4 || D == 8) {
        // swizzle in bit mode (and 0x1f, xor D inside 32 lanes): one LDS-unit
        // instruction instead of two row shifts and a select on the VALU
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (D << 10) | 0x1F);
    } else if constexpr (D == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (__lane_id() & 16) ? r[0] : r[1];
    } else {
        static_assert(D == 32, "lane distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (__lane_id() & 32) ? r[0] : r[1];
    }
}

template <int D>
__device__ __forceinline__ unsigned long long xor_lane64(unsigned long long v)
{
    const uint32_t lo = xor_lane<D>((uint32_t)v), hi = xor_lane<D>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long xor_lane64_dyn(unsigned long long v, uint32_t d)
{
    switch (d) {
        case 1: return xor_lane64<1>(v);
        case 2: return xor_lane64<2>(v);
        case 4: return xor_lane64<4>(v);
        case 8: return xor_lane64<8>(v);
        case 16: return xor_lane64<16>(v);
        default: return xor_lane64<32>(v);
    }
}

// Compare-exchange seen from one side: the key this position keeps, given
// its own key x and its partner's y (keys are unique, so ties never matter).
__device__ __forceinline__ unsigned long long keep(unsigned long long x, unsigned long long y, bool keep_min)
{
    return ((y < x) == keep_min) ? y : x;
}

// Ascending bitonic sort of the NT x E keys of the block (thread t holds
// positions t E ... t E + E - 1).  lds: 2 NT E keys when NT E > 64 E (a
// partner in another wave), unused otherwise.
template <int NT, int E, int LOG2P>
__device__ __forceinline__ void bitonic_regs(unsigned long long (&x)[E], unsigned long long* lds)
{
    static_assert((NT * E) == (1 << LOG2P), "NT x E must be 2^LOG2P");
    constexpr int P = NT * E;
    const uint32_t t = threadIdx.x % NT;   // several NT = 64 groups (waves) may share a block
    int buf = 0;
#pragma unroll
    for (int lk = 1; lk <= LOG2P; lk++) {
        const uint32_t k = 1u << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; lj--) {
            const uint32_t j = 1u << lj;
            if (j >= 64u * E) {
                // partner in another wave: exchange through LDS
                unsigned long long* s = lds + buf * P;
#pragma unroll
                for (int e = 0; e < E; e++) s[t * E + e] = x[e];
                __syncthreads();
                unsigned long long y[E];
#pragma unroll
                for (int e = 0; e < E; e++) y[e] = s[(t * E + e) ^ j];
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const uint32_t i = t * E + e;
                    x[e] = keep(x[e], y[e], ((i & j) == 0) == ((i & k) == 0));
                }
                buf ^= 1;
            } else if (j >= (uint32_t)E) {
                // partner in lane t ^ (j / E) of this wave: all exchanges issued, then compared
                unsigned long long y[E];
#pragma unroll
                for (int e = 0; e < E; e++) y[e] = xor_lane64_dyn(x[e], j / E);
#pragma unroll
                for (int e = 0; e < E; e++) {
                    const uint32_t i = t * E + e;
                    x[e] = keep(x[e], y[e], ((i & j) == 0) == ((i & k) == 0));
                }
            } else {
                // partner in this thread
#pragma unroll
                for (int e = 0; e < E; e++) {
                    if ((e & (int)j) != 0) continue;
                    const uint32_t i = t * E + e;
                    const unsigned long long a = x[e], b = x[e ^ j];
                    const bool up = (i & k) == 0;
                    x[e] = keep(a, b, up);
                    x[e ^ j] = keep(b, a, !up);
                }
            }
        }
    }
}

template <int NT, int E, int LOG2P>
__device__ __forceinline__ void sort_run_regs(unsigned long long* lds, const float* __restrict__ depth,
                                              uint32_t* __restrict__ run, uint32_t n, uint32_t cap)
{
    unsigned long long x[E];
    const uint32_t t = threadIdx.x % NT;
    // branch-free, so that the E index loads, then the E depth loads, are
    // each issued together rather than one wait per key
    uint32_t idx[E];
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        idx[e] = i < n ? run[i] : 0xffffffffu;
    }
    uint32_t dep[E];
#pragma unroll
    for (int e = 0; e < E; e++) dep[e] = __float_as_uint(depth[idx[e] < cap ? idx[e] : 0u]);
#pragma unroll
    for (int e = 0; e < E; e++) x[e] = idx[e] < cap ? ((unsigned long long)dep[e] << 32) | idx[e] : ~0ull;
    bitonic_regs<NT, E, LOG2P>(x, lds);
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        if (i < n) run[i] = x[e] == ~0ull ? 0xffffffffu : (uint32_t)x[e];
    }
}

// position of key x among the sorted run b[0, n): number of keys < x
__device__ __forceinline__ uint32_t rank_in(const uint32_t* __restrict__ b, uint32_t n, unsigned long long x,
                                            const float* __restrict__ proj, uint32_t cap)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key_of(proj, b[mid], cap) < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// A run of up to NW x 512 keys, sorted by a group of NW waves (the NW x 64
// threads from group_base on): each wave sorts 512 keys of it in registers
// (64 lanes x 8, the bitonic network with no LDS stage and no barrier; waves
// past the run's end only pad), then log2(NW) merge-path rounds in LDS
// double the sorted runs.  Each thread makes 8 outputs of a round: a binary
// search on its diagonal finds how many come from the left run (equal keys
// go left first), then 8 merge steps.  Only the ceil(n / 512) chunks that
// hold keys are sorted; the rest are all-padding (~0, sorting last).  s: 2 x
// NW x 512 keys of LDS for the group.  Every thread of the block calls this
// (the rounds end at block barriers), with the same NW.
template <int NW>
__device__ __forceinline__ void sort_run_merge(unsigned long long* s, const float* __restrict__ depth,
                                               uint32_t* __restrict__ run, uint32_t n, uint32_t cap)
{
    constexpr int E = 8, CH = 64 * E, P = NW * CH, NT = NW * 64;
    static_assert(kSortThreads % NT == 0, "groups tile the block");
    const uint32_t t = threadIdx.x % NT;
    const uint32_t w = t >> 6, lane = t & 63;
    const uint32_t nch = (n + CH - 1) / CH;
    unsigned long long x[E];
    if (w < nch) {   // wave-uniform
        const uint32_t c0 = w * CH, m = min(n - c0, (uint32_t)CH);
        uint32_t idx[E], dep[E];
#pragma unroll
        for (int e = 0; e < E; e++) {
            const uint32_t i = lane * E + e;
            idx[e] = i < m ? run[c0 + i] : 0xffffffffu;
        }
#pragma unroll
        for (int e = 0; e < E; e++) dep[e] = __float_as_uint(depth[idx[e] < cap ? idx[e] : 0u]);
#pragma unroll
        for (int e = 0; e < E; e++) x[e] = idx[e] < cap ? ((unsigned long long)dep[e] << 32) | idx[e] : ~0ull;
        bitonic_regs<64, E, 9>(x, nullptr);
    } else {
#pragma unroll
        for (int e = 0; e < E; e++) x[e] = ~0ull;
    }
#pragma unroll
    for (int e = 0; e < E; e++) s[w * CH + lane * E + e] = x[e];
    __syncthreads();
    unsigned long long* src = s;
    unsigned long long* dst = s + P;
#pragma unroll 1
    for (uint32_t L = CH; L < (uint32_t)P; L <<= 1) {
        const uint32_t o0 = t * E;
        const uint32_t pair0 = o0 & ~(2 * L - 1), d = o0 - pair0;
        const unsigned long long* A = src + pair0;
        const unsigned long long* B = A + L;
        uint32_t lo = d > L ? d - L : 0u, hi = d < L ? d : L;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A[mid] <= B[d - mid - 1]) lo = mid + 1; else hi = mid;
        }
        uint32_t i = lo, j = d - lo;
#pragma unroll
        for (int e = 0; e < E; e++) {
            const unsigned long long a = i < L ? A[i] : ~0ull, b = j < L ? B[j] : ~0ull;
            const bool take_a = i < L && (j >= L || a <= b);
            dst[o0 + e] = take_a ? a : b;
            i += take_a ? 1u : 0u;
            j += take_a ? 0u : 1u;
        }
        __syncthreads();
        unsigned long long* tmp = src; src = dst; dst = tmp;
    }
    for (uint32_t p = t; p < n; p += NT) run[p] = src[p] == ~0ull ? 0xffffffffu : (uint32_t)src[p];
}

// A run in (kSortMid, kSortLds]: both halves (the first kSortMid keys and
// the rest) are sorted in place by the merge sort above, then read back into
// LDS as keys, which just fills it, and merged by merge path straight into
// the run: each thread finds where its E outputs start on the diagonal and
// writes them in order.
__device__ __forceinline__ void sort_run_halves(unsigned long long* s, const float* __restrict__ depth,
                                                uint32_t* __restrict__ run, uint32_t n, uint32_t cap)
{
    constexpr uint32_t H = kSortMid, E = kSortLds / kSortThreads;
    sort_run_merge<kSortThreads / 64>(s, depth, run, H, cap);
    __syncthreads();   // the first sort's last LDS reads, before the second's writes
    sort_run_merge<kSortThreads / 64>(s, depth, run + H, n - H, cap);
    __syncthreads();   // the sorted halves are in the run, for every thread
    const uint32_t m = n - H;
    // keys back into LDS, eight per thread in flight: index loads, then depth loads
#pragma unroll 1
    for (uint32_t e0 = 0; e0 < E; e0 += 8) {
        uint32_t idx[8], dep[8];
#pragma unroll
        for (uint32_t e = 0; e < 8; e++) {
            const uint32_t k = (e0 + e) * kSortThreads + threadIdx.x;
            idx[e] = k < n ? run[k] : 0xffffffffu;
        }
#pragma unroll
        for (uint32_t e = 0; e < 8; e++) dep[e] = __float_as_uint(depth[idx[e] < cap ? idx[e] : 0u]);
#pragma unroll
        for (uint32_t e = 0; e < 8; e++) {
            const uint32_t k = (e0 + e) * kSortThreads + threadIdx.x;
            if (k < n) s[k] = idx[e] < cap ? ((unsigned long long)dep[e] << 32) | idx[e] : ~0ull;
        }
    }
    __syncthreads();
    const unsigned long long* A = s;
    const unsigned long long* B = s + H;
    const uint32_t d = threadIdx.x * E;
    if (d < n) {
        uint32_t lo = d > m ? d - m : 0u, hi = d < H ? d : H;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (A[mid] <= B[d - mid - 1]) lo = mid + 1; else hi = mid;
        }
        uint32_t i = lo, j = d - lo;
#pragma unroll 2
        for (uint32_t e = 0; e < E; e++) {
            const unsigned long long a = i < H ? A[i] : ~0ull, b = j < m ? B[j] : ~0ull;
            const bool take_a = i < H && (j >= m || a <= b);
            const unsigned long long x = take_a ? a : b;
            if (d + e < n) run[d + e] = x == ~0ull ? 0xffffffffu : (uint32_t)x;
            i += take_a ? 1u : 0u;
            j += take_a ? 0u : 1u;
        }
    }
    __syncthreads();   // LDS and the run are free for the next step
}

// A run longer than kSortLds: kSortLds-key chunks sorted as above, then
// merge passes in global memory (ping-pong with scratch) where each key
// finds its output slot by binary search in the sibling run.
__device__ __forceinline__ void sort_huge_run(unsigned long long* s, const float* __restrict__ proj,
                                              uint32_t* __restrict__ run, uint32_t* __restrict__ tmp, uint32_t n,
                                              uint32_t cap)
{
    uint32_t* src = run;
    uint32_t* dst = tmp;
    for (uint32_t c0 = 0; c0 < n; c0 += kSortLds) {
        const uint32_t len = min((uint32_t)kSortLds, n - c0);
        if (len > (uint32_t)kSortMid) {
            sort_run_halves(s, proj, src + c0, len, cap);
        } else {
            sort_run_merge<kSortThreads / 64>(s, proj, src + c0, len, cap);
            __syncthreads();
        }
    }
    // merge passes: run pairs [i, i + w) and [i + w, i + 2w)
    for (uint32_t w = kSortLds; w < n; w <<= 1) {
        for (uint32_t k = threadIdx.x; k < n; k += kSortThreads) {
            const uint32_t pair = k / (2 * w) * (2 * w);
            const uint32_t mid = min(pair + w, n), end = min(pair + 2 * w, n);
            const unsigned long long x = key_of(proj, src[k], cap);
            uint32_t out;
            if (k < mid) out = pair + (k - pair) + rank_in(src + mid, end - mid, x, proj, cap);
            else out = pair + (k - mid) + rank_in(src + pair, mid - pair, x, proj, cap);
            out = out < n ? out : n - 1;
            dst[out] = src[k];
        }
        __syncthreads();
        uint32_t* t = src; src = dst; dst = t;
    }
    if (src != run)
        for (uint32_t k = threadIdx.x; k < n; k += kSortThreads) run[k] = src[k];
    __syncthreads();
}

// All runs in one launch of 512-thread blocks with 64 KB of LDS, two per
// compute unit.  Work items, longest first, are handed out by a counter
// (one atomic per item, not per key):
//   n_huge items   one run > 16384, by LDS chunks and merge passes;
//   n_xl items     one run in (4096, 16384]: up to 8192 by two merge sorts
//                  and an LDS merge, longer by such chunks and merge passes;
//   n_large items  one run in (2048, 4096], by wave sorts and merges;
//   n_mid / 2      two queued runs in (256, 2048], one per 256 threads
//                  (their merge rounds in step: the block barriers match);
//   T / 8          eight tiles, one per wave, sorted if 1 < n <= 256.
// Every block leaves once the items run out.
__global__ __launch_bounds__(kSortThreads) void k_sort(const FrameParams* __restrict__ fp, FrameInfo* info,
                                                       const uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ queues,
                                                       const float* __restrict__ depth, uint32_t* __restrict__ sorted,
                                                       uint32_t* __restrict__ scratch, uint32_t cap)
{
    static_assert(2 * kSortMid <= kSortLds && 2 * 2 * kSortSmall <= kSortLds, "LDS per item");
    constexpr uint32_t kWaves = kSortThreads / 64, kGroups = kSortThreads / 256;
    __shared__ unsigned long long s[kSortLds];
    __shared__ uint32_t s_item;
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t nl = info->n_large, nh = info->n_huge, nm = info->n_mid, nx = info->n_xl;
    // the longest runs first: huge, then (4096, 16384], then (2048, 4096]
    const uint32_t i_xl = nh, i_large = i_xl + nx, i_mid = i_large + nl,
                   i_wave = i_mid + (nm + kGroups - 1) / kGroups, n_items = i_wave + (T + kWaves - 1) / kWaves;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&info->sort_next, 1u);
        __syncthreads();
        const uint32_t i = s_item;
        __syncthreads();
        if (i >= n_items) break;
        if (i < i_mid) {
            const uint32_t tile = i < i_xl ? queues[T + i] : i < i_large ? queues[T - 1 - (i - i_xl)] : queues[i - i_large];
            const uint2 r = ranges[tile];
            const uint32_t n = r.y - r.x;
            if (n <= (uint32_t)kSortMid)
                sort_run_merge<kSortThreads / 64>(s, depth, sorted + r.x, n, cap);
            else if (n <= (uint32_t)kSortLds) sort_run_halves(s, depth, sorted + r.x, n, cap);
            else sort_huge_run(s, depth, sorted + r.x, scratch + r.x, n, cap);
        } else if (i < i_wave) {
            const uint32_t g = threadIdx.x / 256, q = kGroups * (i - i_mid) + g;
            uint2 r = make_uint2(0u, 0u);   // an empty run still steps through the network
            if (q < nm) r = ranges[queues[2 * T + q]];
            sort_run_merge<kSortSmall / 512>(s + g * 2 * kSortSmall, depth, sorted + r.x, r.y - r.x, cap);
        } else {
            const uint32_t t = kWaves * (i - i_wave) + threadIdx.x / 64;
            const uint2 r = t < T ? ranges[t] : make_uint2(0u, 0u);
            const uint32_t n = r.y - r.x;
            uint32_t* run = sorted + r.x;
            // the lane index is threadIdx.x % 64 inside sort_run_regs<64, ...>
            if (n > 1 && n <= 64) sort_run_regs<64, 1, 6>(nullptr, depth, run, n, cap);
            else if (n > 64 && n <= 128) sort_run_regs<64, 2, 7>(nullptr, depth, run, n, cap);
            else if (n > 128 && n <= (uint32_t)kSortWave) sort_run_regs<64, 4, 8>(nullptr, depth, run, n, cap);
        }
        __syncthreads();   // LDS is reused by the next item
    }
}

}  // namespace

hipError_t launch_sort(const Views& v, hipStream_t st)
{
    // two 64 KB-LDS blocks per compute unit
    static thread_local int dev_cached = -1, cus = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != dev_cached) {
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        dev_cached = dev;
    }
    k_sort<<<std::max(1, 2 * cus), kSortThreads, 0, st>>>(v.params, v.info, v.ranges, v.large, v.depth, v.sorted,
                                                      reinterpret_cast<uint32_t*>(v.temp), v.max_active);
    return hipGetLastError();
}

}  // namespace lodge
