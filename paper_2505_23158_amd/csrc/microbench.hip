// Measurement and verification helpers, not part of the method: the rates
// the kernels' roofline fractions are also reported against, measured on the
// device at hand instead of taken from its data sheet, and the FP32 division
// and square root the bit-exact stages rely on.
//
// k_stream_copy  a coalesced device copy, 16-byte non-temporal accesses, four
//                loads per thread in flight before the stores: the HBM rate
//                of a kernel that reads and writes once (bytes read + bytes
//                written over the time).
// k_stream_read  the same loads summed per thread, one float written per
//                thread: the HBM rate of a kernel that only reads.
// k_fma_chains   independent chains of dependent FP32 FMAs per lane, enough
//                of them and enough waves to cover the FMA latency: the rate
//                at which the SIMDs retire non-packed VALU lane-ops (one FMA
//                counted as one).
// k_div_sqrt     q = a / b and r = sqrt(a) per element, built with the
//                library's flags: the selection, rectangles and depths match
//                the oracle bit for bit only if both are correctly rounded.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));   // a 16-byte access the nontemporal builtins take

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 4;
constexpr int kFmaThreads = 256;
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(kCopyThreads) void k_stream_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                              size_t n4)
{
    const size_t stride = (size_t)gridDim.x * kCopyThreads;
    size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * stride < n4; i += kCopyUnroll * stride) {
        v4f v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n4; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(kCopyThreads) void k_stream_read(const v4f* __restrict__ src, float* __restrict__ out,
                                                              size_t n4)
{
    const size_t stride = (size_t)gridDim.x * kCopyThreads;
    size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x;
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (; i + (kCopyUnroll - 1) * stride < n4; i += kCopyUnroll * stride) {
        v4f v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) acc += v[u];
    }
    for (; i < n4; i += stride) acc += __builtin_nontemporal_load(src + i);
    out[(size_t)blockIdx.x * kCopyThreads + threadIdx.x] = (acc.x + acc.y) + (acc.z + acc.w);
}

// Each chain runs x <- fma(x, a, b) iters times; the chains' sum is written
// so that no FMA is dead.
__global__ __launch_bounds__(kFmaThreads) void k_fma_chains(float* __restrict__ out, uint32_t iters, float a,
                                                            float b)
{
    const uint32_t t = blockIdx.x * kFmaThreads + threadIdx.x;
    float x[kFmaChains];
#pragma unroll
    for (int c = 0; c < kFmaChains; c++) x[c] = (float)c;
    for (uint32_t k = 0; k < iters; k++) {
#pragma unroll
        for (int c = 0; c < kFmaChains; c++) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kFmaChains; c++) s += x[c];
    out[t] = s;
}

__global__ __launch_bounds__(256) void k_div_sqrt(const float* __restrict__ a, const float* __restrict__ b,
                                                  float* __restrict__ q, float* __restrict__ r, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        q[i] = a[i] / b[i];
        r[i] = sqrtf(a[i]);
    }
}

}  // namespace

}  // namespace lodge

using namespace lodge;

extern "C" {

lodge_status lodge_microbench_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    if (bytes == 0) return LODGE_OK;
    if (!src || !dst || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
        return fail(LODGE_ERR_INVALID_ARG, "microbench_copy: 16-byte aligned non-NULL buffers and bytes % 16 == 0");
    const size_t n4 = bytes / 16;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "microbench_copy");
    // 64 blocks per compute unit: the fastest of 4..256 on the 1-2 GiB copies measured
    const size_t want = (n4 + kCopyThreads * kCopyUnroll - 1) / (kCopyThreads * kCopyUnroll);
    const uint32_t blocks = (uint32_t)std::max<size_t>(1, std::min<size_t>(want, (size_t)cus * 64));
    k_stream_copy<<<blocks, kCopyThreads, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const v4f*>(src), static_cast<v4f*>(dst), n4);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "microbench_copy");
    return LODGE_OK;
}

lodge_status lodge_microbench_read_blocks(size_t bytes, uint32_t* blocks)
{
    if (!blocks) return fail(LODGE_ERR_INVALID_ARG, "microbench_read_blocks: blocks is NULL");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "microbench_read_blocks");
    // 16 blocks per compute unit: the fastest of 4..256 on the 1-2 GiB reads measured
    const size_t n4 = bytes / 16;
    const size_t want = (n4 + kCopyThreads * kCopyUnroll - 1) / (kCopyThreads * kCopyUnroll);
    *blocks = (uint32_t)std::max<size_t>(1, std::min<size_t>(want, (size_t)cus * 16));
    return LODGE_OK;
}

lodge_status lodge_microbench_read(const void* src, size_t bytes, float* out, uint32_t blocks, void* stream)
{
    if (!src || !out || blocks == 0 || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16)
        return fail(LODGE_ERR_INVALID_ARG, "microbench_read: 16-byte aligned src, bytes % 16 == 0, out, blocks > 0");
    k_stream_read<<<blocks, kCopyThreads, 0, static_cast<hipStream_t>(stream)>>>(static_cast<const v4f*>(src), out,
                                                                              bytes / 16);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "microbench_read");
    return LODGE_OK;
}

lodge_status lodge_fp32_div_sqrt(const float* a, const float* b, float* q, float* r, size_t n, void* stream)
{
    if (n == 0) return LODGE_OK;
    if (!a || !b || !q || !r) return fail(LODGE_ERR_INVALID_ARG, "fp32_div_sqrt: NULL buffer");
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + 255) / 256, 65536);
    k_div_sqrt<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(a, b, q, r, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fp32_div_sqrt");
    return LODGE_OK;
}

lodge_status lodge_microbench_fma(float* out, uint32_t blocks, uint32_t iters, float a, float b, void* stream)
{
    if (!out || blocks == 0) return fail(LODGE_ERR_INVALID_ARG, "microbench_fma: out non-NULL and blocks > 0");
    k_fma_chains<<<blocks, kFmaThreads, 0, static_cast<hipStream_t>(stream)>>>(out, iters, a, b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "microbench_fma");
    return LODGE_OK;
}

}  // extern "C"
