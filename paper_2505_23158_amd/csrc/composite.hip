// Front-to-back alpha compositing (LODGE Sec. 3 "Preliminaries", Eq. 1:
// alpha = o G(p), G = exp(-1/2 (p - mu')^T Sigma'^-1 (p - mu'))).
//
// One 256-thread block per 16 x 16 tile, one pixel per thread, tiles taken
// longest-list first.  The tile's sorted run is staged through LDS in
// batches of 256 (each thread gathers one Gaussian's 36 bytes: centre,
// conic, opacity, colour); every thread then walks the batch in order.
// Per entry: power = -1/2 (A dx^2 + C dy^2) - B dx dy; skip if power > 0;
// alpha = min(0.99, o exp(power)); skip if alpha < 1/255; stop (without
// blending) once T (1 - alpha) < 1e-4; else C += rgb alpha T, T *= 1 - alpha.
// The block leaves its run once every pixel has stopped.
//
// Most evaluated pairs fall below alpha = 1/255 (small splats covering a
// few pixels of a tile), so the exponential is skipped when power is below
// ln(1 / (255 o)) by a margin (1e-3) far larger than the rounding of either
// side: that decision is then the same as the one alpha would give.
#include "lodge_internal.hpp"
#include "splat.hpp"

namespace lodge {

namespace {

constexpr int kBatch = 256;

__global__ __launch_bounds__(256) void k_composite(const FrameParams* __restrict__ fp, FrameInfo* info,
                                                   const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ sorted,
                                                   const float4* __restrict__ proj, float* __restrict__ image,
                                                   float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                                   uint32_t cap)
{
    __shared__ float4 s_geo[kBatch];   // u, v, -A/2, -B
    __shared__ float4 s_col[kBatch];   // -C/2, o, skip threshold, r
    __shared__ float2 s_gb[kBatch];    // g, b
    __shared__ uint32_t s_eval[4], s_blend[4];

    const int32_t W = fp->cam.width, H = fp->cam.height, TX = fp->TX;
    const uint32_t tile = order[blockIdx.x];
    const uint32_t tx = tile % (uint32_t)TX, ty = tile / (uint32_t)TX;
    const uint32_t x = tx * kTile + (threadIdx.x & 15), y = ty * kTile + (threadIdx.x >> 4);
    const bool inside = (int32_t)x < W && (int32_t)y < H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint2 rg = ranges[tile];
    const uint32_t len = rg.y - rg.x;

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, nblend = 0, neval = len;
    bool done = !inside;

    for (uint32_t b0 = 0; b0 < len; b0 += kBatch) {
        if (__syncthreads_count(done) == 256) break;
        const uint32_t k = b0 + threadIdx.x;
        if (k < len) {
            uint32_t a = sorted[rg.x + k];
            a = a < cap ? a : 0u;   // an index outside the active set would be a binning bug
            stage_splat(proj, a, s_geo[threadIdx.x], s_col[threadIdx.x], s_gb[threadIdx.x]);
        }
        __syncthreads();
        if (!done) {
            const uint32_t nb = min((uint32_t)kBatch, len - b0);
            for (uint32_t j = 0; j < nb; j++) {
                const float4 g = s_geo[j];
                const float4 c = s_col[j];
                float dx, dy, G;
                bool clamped;
                const float alpha = splat_alpha(g, c, px, py, dx, dy, G, clamped);
                if (alpha < 0.0f) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kTStop) {
                    done = true;
                    neval = b0 + j + 1;
                    break;
                }
                const float wgt = alpha * T;
                const float2 gb = s_gb[j];
                cr += c.w * wgt;
                cg += gb.x * wgt;
                cb += gb.y * wgt;
                T = Tn;
                last = b0 + j + 1;
                nblend++;
            }
        }
    }
    if (inside) {
        const size_t p = (size_t)y * W + x;
        const size_t HW = (size_t)W * H;
        image[p] = cr + T * fp->cam.bg[0];
        image[HW + p] = cg + T * fp->cam.bg[1];
        image[2 * HW + p] = cb + T * fp->cam.bg[2];
        final_T[p] = T;
        n_contrib[p] = last;
    } else {
        neval = 0;
    }
    // counters: wave sums, then one atomic per block
    uint32_t e = neval, bl = nblend;
    for (int off = 32; off > 0; off >>= 1) {
        e += __shfl_xor(e, off);
        bl += __shfl_xor(bl, off);
    }
    if ((threadIdx.x & 63) == 0) { s_eval[threadIdx.x >> 6] = e; s_blend[threadIdx.x >> 6] = bl; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long se = (unsigned long long)s_eval[0] + s_eval[1] + s_eval[2] + s_eval[3];
        const unsigned long long sb = (unsigned long long)s_blend[0] + s_blend[1] + s_blend[2] + s_blend[3];
        if (se) atomicAdd(&info->pairs_evaluated, se);
        if (sb) atomicAdd(&info->pairs_blended, sb);
    }
}

}  // namespace

hipError_t launch_composite(const Views& v, float* image, float* final_T, uint32_t* n_contrib, hipStream_t st)
{
    k_composite<<<v.lay.T, 256, 0, st>>>(v.params, v.info, v.ranges, v.order, v.sorted, v.proj, image, final_T,
                                         n_contrib, v.max_active);
    return hipGetLastError();
}

}  // namespace lodge
