// Per-tile sort of the binned instances (LODGE Sec. 3 "Preliminaries":
// the Gaussians of each tile are sorted in depth before blending).
//
// Each tile's run holds active indices in arbitrary order.  The key of
// index a is (float bits of its camera depth) << 32 | a: depth > znear > 0,
// so the bit pattern orders like the value, and the index makes the order
// total (ties in depth are broken by active index, i.e. by global id).
//
// Runs up to 4096 keys are sorted by a bitonic network held in registers:
// each thread keeps E consecutive keys; stages whose partner is in the same
// thread compare registers, stages whose partner is in another lane of the
// wave exchange keys with lane shuffles, and only stages whose partner is in
// another wave go through LDS (double-buffered, one barrier per stage).
//
//   k_sort_wave   runs <= 256, one wave each (four per block), 1-4 keys per
//                 lane: no LDS, no barrier.
//   k_sort_mid    queued runs in (256, 2048], 256 threads x 8 keys.
//   k_sort_big    queued runs in (2048, 4096], 1024 threads x 4 keys.
//   k_sort_big8   queued runs in (4096, 8192], 1024 threads x 8 keys.
//   k_sort_large  queued runs in (8192, 16384]: the bitonic network in 128 KB
//                 of LDS, 1024 threads (gfx950 allows 160 KB).
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

// 32-bit value of lane (lane ^ D) of the wave.  Distances 1 and 2 are quad
// permutes and 4 and 8 two row shifts plus a select (DPP: register-speed, no
// LDS round trip); 16 swizzles within 32 lanes; 32 goes through bpermute.
template <int D>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    if constexpr (D == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    } else if constexpr (D == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    } else if constexpr (D == 4 || D == 8) {
        // row_shl:D reads lane + D, row_shr:D reads lane - D (both stay inside the 16-lane row here)
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x100 + D, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x110 + D, 0xF, 0xF, false);
        return (__lane_id() & D) ? dn : up;
    } else if constexpr (D == 16) {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);   // bit mode: xor 16 within 32 lanes
    } else {
        return (uint32_t)__shfl_xor((int)v, D);
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
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        x[e] = i < n ? key_of(depth, run[i], cap) : ~0ull;
    }
    bitonic_regs<NT, E, LOG2P>(x, lds);
#pragma unroll
    for (int e = 0; e < E; e++) {
        const uint32_t i = t * E + e;
        if (i < n) run[i] = x[e] == ~0ull ? 0xffffffffu : (uint32_t)x[e];
    }
}

__global__ __launch_bounds__(256) void k_sort_wave(const FrameParams* fp, const uint2* __restrict__ ranges,
                                                   const float* __restrict__ depth, uint32_t* __restrict__ sorted,
                                                   uint32_t cap)
{
    const uint32_t T = (uint32_t)(fp->TX * fp->TY);
    const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= T) return;
    const uint2 r = ranges[t];
    const uint32_t n = r.y - r.x;
    if (n <= 1 || n > (uint32_t)kSortWave) return;
    uint32_t* run = sorted + r.x;
    // the lane index is threadIdx.x % 64 inside sort_run_regs<64, ...>
    if (n <= 64) sort_run_regs<64, 1, 6>(nullptr, depth, run, n, cap);
    else if (n <= 128) sort_run_regs<64, 2, 7>(nullptr, depth, run, n, cap);
    else sort_run_regs<64, 4, 8>(nullptr, depth, run, n, cap);
}

__global__ __launch_bounds__(256) void k_sort_mid(const FrameInfo* info, const uint2* __restrict__ ranges,
                                                  const uint32_t* __restrict__ mid, const float* __restrict__ depth,
                                                  uint32_t* __restrict__ sorted, uint32_t cap)
{
    __shared__ unsigned long long s[2 * kSortSmall];
    const uint32_t nm = info->n_mid;
    for (uint32_t q = blockIdx.x; q < nm; q += gridDim.x) {
        const uint2 r = ranges[mid[q]];
        sort_run_regs<256, kSortSmall / 256, 11>(s, depth, sorted + r.x, r.y - r.x, cap);
        __syncthreads();   // LDS is reused by the next run
    }
}

__global__ __launch_bounds__(1024) void k_sort_big(const FrameInfo* info, const uint2* __restrict__ ranges,
                                                  const uint32_t* __restrict__ large, const float* __restrict__ depth,
                                                  uint32_t* __restrict__ sorted, uint32_t cap)
{
    __shared__ unsigned long long s[2 * kSortMid];
    const uint32_t nl = info->n_large;
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint2 r = ranges[large[q]];
        const uint32_t n = r.y - r.x;
        if (n > (uint32_t)kSortMid) continue;
        sort_run_regs<1024, kSortMid / 1024, 12>(s, depth, sorted + r.x, n, cap);
        __syncthreads();
    }
}

// Queued runs in (4096, 8192]: 1024 threads x 8 keys in registers, 128 KB
// of LDS for the double-buffered cross-wave stages.
__global__ __launch_bounds__(1024) void k_sort_big8(const FrameInfo* info, const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ large,
                                                    const float* __restrict__ depth, uint32_t* __restrict__ sorted,
                                                    uint32_t cap)
{
    __shared__ unsigned long long s[2 * 2 * kSortMid];
    const uint32_t nl = info->n_large;
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint2 r = ranges[large[q]];
        const uint32_t n = r.y - r.x;
        if (n <= (uint32_t)kSortMid || n > 2u * kSortMid) continue;
        sort_run_regs<1024, 2 * kSortMid / 1024, 13>(s, depth, sorted + r.x, n, cap);
        __syncthreads();
    }
}

// Runs in (kSortSmall, kSortLarge], in two length bands: each instantiation
// takes the queued runs in (LO, CAP] and allocates only the LDS that CAP
// needs, so that more blocks fit a CU.
template <int LO, int CAP>
__global__ __launch_bounds__(1024) void k_sort_large(const FrameInfo* info, const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ large,
                                                     const float* __restrict__ proj, uint32_t* __restrict__ sorted,
                                                     uint32_t cap)
{
    __shared__ unsigned long long s[CAP];
    const uint32_t nl = info->n_large;
    for (uint32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const uint2 r = ranges[large[q]];
        const uint32_t n = r.y - r.x;
        if (n <= (uint32_t)LO || n > (uint32_t)CAP) continue;
        sort_run<1024, CAP>(s, proj, sorted + r.x, n, cap);
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
    k_sort_wave<<<(v.lay.T + 3) / 4, 256, 0, st>>>(v.params, v.ranges, v.depth, v.sorted, v.max_active);
    k_sort_mid<<<1024, 256, 0, st>>>(v.info, v.ranges, v.large + 2 * v.lay.T, v.depth, v.sorted, v.max_active);
    k_sort_big<<<512, 1024, 0, st>>>(v.info, v.ranges, v.large, v.depth, v.sorted, v.max_active);
    k_sort_big8<<<256, 1024, 0, st>>>(v.info, v.ranges, v.large, v.depth, v.sorted, v.max_active);
    k_sort_large<2 * kSortMid, kSortLarge><<<256, 1024, 0, st>>>(v.info, v.ranges, v.large, v.depth, v.sorted,
                                                                  v.max_active);
    k_sort_huge<<<64, 1024, 0, st>>>(v.params, v.info, v.ranges, v.large, v.depth, v.sorted,
                                     reinterpret_cast<uint32_t*>(v.temp), v.max_active);
    return hipGetLastError();
}

}  // namespace lodge
