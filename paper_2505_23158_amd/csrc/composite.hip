// Front-to-back alpha compositing (LODGE Sec. 3 "Preliminaries", Eq. 1:
// alpha = o G(p), G = exp(-1/2 (p - mu')^T Sigma'^-1 (p - mu'))).
//
// One 256-thread block per 16 x 16 tile, taken longest-list first; each of
// the four waves owns one 8 x 8 quadrant, one pixel per lane.  The tile's
// sorted run is staged through LDS in batches of 256: each thread gathers
// one splat's record and tests it against the four quadrants with the
// half-extents (ex, ey) of the ellipse where its alpha can reach 1/255;
// ballots then build one ordered list per quadrant, so a wave walks only
// the splats that can touch its pixels.  Per (pixel, splat): power =
// -1/2 (A dx^2 + C dy^2) - B dx dy; skip if power > 0 or below the splat's
// threshold ln(1/(255 o)) - 1e-3 (alpha < 1/255 there, so exp is not
// needed); alpha = min(0.99, o exp(power)); skip if alpha < 1/255; stop
// (without blending) once T (1 - alpha) < 1e-4; else C += rgb alpha T,
// T *= 1 - alpha.  Skipping a splat for a whole quadrant changes no
// decision: every pixel of the quadrant would have skipped it (the test has
// a margin far above the rounding of the extents).
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
    __shared__ float4 s_geo[kBatch];        // u, v, -A/2, -B
    __shared__ float4 s_col[kBatch];        // -C/2, o, threshold, r
    __shared__ float2 s_gb[kBatch];         // g, b
    __shared__ uint16_t s_list[4][kBatch];  // per quadrant: batch slots in list order
    __shared__ uint32_t s_cnt[4][4];        // [quadrant][staging wave]
    __shared__ uint32_t s_eval[4], s_blend[4];

    const int32_t W = fp->cam.width, H = fp->cam.height, TX = fp->TX;
    const uint32_t tile = order[blockIdx.x];
    const uint32_t tx = tile % (uint32_t)TX, ty = tile / (uint32_t)TX;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t qx0 = tx * kTile + (wave & 1u) * 8u, qy0 = ty * kTile + (wave >> 1) * 8u;
    const uint32_t x = qx0 + (lane & 7u), y = qy0 + (lane >> 3);
    const bool inside = (int32_t)x < W && (int32_t)y < H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    // quadrant centres of the pixel-centre boxes (half-width 3.5 px)
    float qcx[4], qcy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        qcx[q] = (float)(tx * kTile + (q & 1) * 8) + 4.0f;
        qcy[q] = (float)(ty * kTile + (q >> 1) * 8) + 4.0f;
    }
    const uint2 rg = ranges[tile];
    const uint32_t len = rg.y - rg.x;
    const unsigned long long lt = (1ull << lane) - 1ull;

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, nblend = 0, neval = len;
    bool done = !inside;

    for (uint32_t b0 = 0; b0 < len; b0 += kBatch) {
        if (__syncthreads_count(done) == 256) break;
        const uint32_t i = threadIdx.x;
        const uint32_t k = b0 + i;
        bool hit[4] = {false, false, false, false};
        if (k < len) {
            uint32_t a = sorted[rg.x + k];
            a = a < cap ? a : 0u;   // an index outside the active set would be a binning bug
            const float4 r0 = proj[3 * (size_t)a];
            const float4 r1 = proj[3 * (size_t)a + 1];
            const float4 r2 = proj[3 * (size_t)a + 2];
            s_geo[i] = make_float4(r0.x, r0.y, -0.5f * r0.z, -r0.w);
            s_col[i] = make_float4(-0.5f * r1.x, r1.y, r2.w, r1.z);
            s_gb[i] = make_float2(r1.w, r2.x);
            const float ex = r2.y, ey = r2.z;
            if (ex >= 0.0f) {
                const float mx = ex + 3.5f + 0.01f + 1e-3f * ex, my = ey + 3.5f + 0.01f + 1e-3f * ey;
#pragma unroll
                for (int q = 0; q < 4; q++) hit[q] = fabsf(r0.x - qcx[q]) <= mx && fabsf(r0.y - qcy[q]) <= my;
            }
        }
        unsigned long long m[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            m[q] = __ballot(hit[q]);
            if (lane == 0) s_cnt[q][wave] = (uint32_t)__popcll(m[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (hit[q]) {
                uint32_t pos = (uint32_t)__popcll(m[q] & lt);
                for (uint32_t w = 0; w < wave; w++) pos += s_cnt[q][w];
                s_list[q][pos] = (uint16_t)i;
            }
        }
        __syncthreads();
        if (!done) {
            const uint32_t n = s_cnt[wave][0] + s_cnt[wave][1] + s_cnt[wave][2] + s_cnt[wave][3];
            for (uint32_t j = 0; j < n; j++) {
                const uint32_t e = s_list[wave][j];
                const float4 g = s_geo[e];
                const float4 c = s_col[e];
                float dx, dy, G;
                bool clamped;
                const float alpha = splat_alpha(g, c, px, py, dx, dy, G, clamped);
                if (alpha < 0.0f) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kTStop) {
                    done = true;
                    neval = b0 + e + 1;
                    break;
                }
                const float wgt = alpha * T;
                const float2 gb = s_gb[e];
                cr = __builtin_fmaf(c.w, wgt, cr);
                cg = __builtin_fmaf(gb.x, wgt, cg);
                cb = __builtin_fmaf(gb.y, wgt, cb);
                T = Tn;
                last = b0 + e + 1;
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
    uint32_t ev = neval, bl = nblend;
    for (int off = 32; off > 0; off >>= 1) {
        ev += __shfl_xor(ev, off);
        bl += __shfl_xor(bl, off);
    }
    if (lane == 0) { s_eval[wave] = ev; s_blend[wave] = bl; }
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
