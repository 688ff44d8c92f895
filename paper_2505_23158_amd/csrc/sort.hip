// Per-tile sort of the binned instances (LODGE Sec. 3 "Preliminaries":
// the Gaussians of each tile are sorted in depth before blending).
//
// Each tile's run holds active indices in arbitrary order.  The key of
// index a is (float bits of its camera depth) << 32 | a: depth > znear > 0,
// so the bit pattern orders like the value, and the index makes the order
// total (ties in depth are broken by active index, i.e. by global id).
//
//   k_sort_small  one 256-thread block per tile, runs <= 2048: bitonic
//                 network on 64-bit keys in LDS (16 KB).
//   k_sort_large  1024-thread blocks over the queue of runs in (2048, 16384]:
//                 the same network in 128 KB of LDS (gfx950 allows 160 KB).
//   k_sort_huge   runs > 16384: 16384-key chunks sorted in LDS, then merge
//                 passes in global memory where each key finds its output
//                 slot by binary search in the sibling run.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

// Indices come from the emission pass; one outside [0, cap) would be a
// binning bug, so it sorts last instead of being dereferenced.
__device__ __forceinline__ unsigned long long key_of(const float* __restrict__ depth, uint32_t a, uint32_t cap)
{
    if (a >= cap) return ~0ull;
    return ((unsigned long long)__float_as_uint(depth[a]) << 32) | a;
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t n)
{
    uint32_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

// Ascending bitonic sort of s[0, P), P a power of two; all threads of the block take part.
template <int NT>
__device__ __forceinline__ void bitonic_lds(unsigned long long* s, uint32_t P)
{
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t p = threadIdx.x; p < (P >> 1); p += NT) {
                const uint32_t i = (p / j) * (2 * j) + (p % j);
                const uint32_t q = i + j;
                const unsigned long long x = s[i], y = s[q];
                const bool up = (i & k) == 0;
                if ((x > y) == up) { s[i] = y; s[q] = x; }
            }
            __syncthreads();
        }
    }
}

template <int NT, int CAP>
__device__ __forceinline__ void sort_run(unsigned long long* s, const float* __restrict__ proj,
                                         uint32_t* __restrict__ run, uint32_t n, uint32_t cap)
{
    const uint32_t P = next_pow2(n);
    for (uint32_t k = threadIdx.x; k < P; k += NT) s[k] = k < n ? key_of(proj, run[k], cap) : ~0ull;
    __syncthreads();
    bitonic_lds<NT>(s, P);
    for (uint32_t k = threadIdx.x; k < n; k += NT) run[k] = s[k] == ~0ull ? 0xffffffffu : (uint32_t)s[k];
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_sort_small(const FrameParams* fp, const uint2* __restrict__ ranges,
                                                    const float* __restrict__ proj, uint32_t* __restrict__ sorted,
                                                    uint32_t cap)
{
    __shared__ unsigned long long s[kSortSmall];
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint2 r = ranges[t];
        const uint32_t n = r.y - r.x;
        if (n <= 1 || n > (uint32_t)kSortSmall) continue;
        uint32_t* run = sorted + r.x;
        if (n <= 256) {
            // rank sort: keys are unique, so each key's rank is the number of smaller keys
            const uint32_t i = threadIdx.x;
            unsigned long long mine = ~0ull;
            if (i < n) s[i] = mine = key_of(proj, run[i], cap);
            __syncthreads();
            uint32_t rank = 0;
            if (i < n)
                for (uint32_t j = 0; j < n; j++) rank += s[j] < mine ? 1u : 0u;
            __syncthreads();
            if (i < n) run[rank] = mine == ~0ull ? 0xffffffffu : (uint32_t)mine;
            __syncthreads();
        } else {
            sort_run<256, kSortSmall>(s, proj, run, n, cap);
        }
    }
}

__global__ __launch_bounds__(1024) void k_sort_large(const FrameInfo* info, const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ large,
                                                     const float* __restrict__ proj, uint32_t* __restrict__ sorted,
                                                     uint32_t cap)
{
    __shared__ unsigned long long s[kSortLarge];
    const uint32_t nl = info->n_large;
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint2 r = ranges[large[q]];
        sort_run<1024, kSortLarge>(s, proj, sorted + r.x, r.y - r.x, cap);
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

__global__ __launch_bounds__(1024) void k_sort_huge(const FrameParams* fp, const FrameInfo* info,
                                                    const uint2* __restrict__ ranges, const uint32_t* __restrict__ large,
                                                    const float* __restrict__ proj, uint32_t* __restrict__ sorted,
                                                    uint32_t* __restrict__ scratch, uint32_t cap)
{
    __shared__ unsigned long long s[kSortLarge];
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t nh = info->n_huge;
    for (uint32_t q = blockIdx.x; q < nh; q += gridDim.x) {
        const uint2 r = ranges[large[T + q]];
        const uint32_t n = r.y - r.x;
        uint32_t* src = sorted + r.x;
        uint32_t* dst = scratch + r.x;
        // sorted chunks in place
        for (uint32_t c0 = 0; c0 < n; c0 += kSortLarge)
            sort_run<1024, kSortLarge>(s, proj, src + c0, min((uint32_t)kSortLarge, n - c0), cap);
        // merge passes: run pairs [i, i + w) and [i + w, i + 2w)
        for (uint32_t w = kSortLarge; w < n; w <<= 1) {
            for (uint32_t k = threadIdx.x; k < n; k += 1024) {
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
            uint32_t* tmp = src; src = dst; dst = tmp;
        }
        if (src != sorted + r.x)
            for (uint32_t k = threadIdx.x; k < n; k += 1024) sorted[r.x + k] = src[k];
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_sort(const Views& v, hipStream_t st)
{
    k_sort_small<<<v.lay.T, 256, 0, st>>>(v.params, v.ranges, v.depth, v.sorted, v.max_active);
    k_sort_large<<<256, 1024, 0, st>>>(v.info, v.ranges, v.large, v.depth, v.sorted, v.max_active);
    k_sort_huge<<<64, 1024, 0, st>>>(v.params, v.info, v.ranges, v.large, v.depth, v.sorted,
                                     reinterpret_cast<uint32_t*>(v.temp), v.max_active);
    return hipGetLastError();
}

}  // namespace lodge
