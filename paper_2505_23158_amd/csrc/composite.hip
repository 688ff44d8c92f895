// Front-to-back alpha compositing (LODGE Sec. 3 "Preliminaries", Eq. 1:
// alpha = o G(p), G = exp(-1/2 (p - mu')^T Sigma'^-1 (p - mu'))).
//
// Each 16 x 16 tile is split into four 8 x 8 quadrants and every quadrant is
// one wave, one pixel per lane, working on its own: the waves of a block
// share no data and never wait for each other, so a quadrant that reaches
// full opacity stops at once.  Blocks take tiles longest-list first.
//
// A wave walks its tile's sorted run in batches of 64.  Each lane gathers
// one splat's record and tests whether its alpha can reach 1/255 anywhere
// in the quadrant: a bounding-box test on the ellipse where it can
// (half-extents ex, ey from the projection), then the exact minimum of the
// conic quadratic form over the box of the quadrant's pixel centres.  A
// ballot compacts the survivors, in list order, into the wave's LDS slice;
// the wave then walks them.  Per (pixel, splat): power = -1/2 (A dx^2 +
// C dy^2) - B dx dy; skip if power > 0 or below the splat's threshold
// ln(1/(255 o)) - 1e-3 (alpha < 1/255 there, so exp is not needed);
// alpha = min(0.99, o exp(power)); skip if alpha < 1/255; stop (without
// blending) once T (1 - alpha) < 1e-4; else C += rgb alpha T,
// T *= 1 - alpha.  A splat dropped for a quadrant changes no decision: the
// test keeps every splat that any pixel of the quadrant would not skip,
// with a margin above the rounding of both computations.
//
// Per-wave pair counters go to one slot each (no atomics); the host sums
// them when the frame info is read.
#include "lodge_internal.hpp"
#include "splat.hpp"

namespace lodge {

namespace {

// Can the splat's alpha reach 1/255 at some point of the box [bx0, bx1] x
// [by0, by1]?  r0 = (u, v, A, B), r1 = (C, ...), r2 = (.., ex, ey, thr) as
// written by the projection; alpha >= 1/255 needs q(d) = A dx^2 + 2B dx dy
// + C dy^2 <= rho = -2 thr.
__device__ __forceinline__ bool reaches_box(const float4& r0, const float4& r1, const float4& r2, float bx0,
                                            float bx1, float by0, float by1)
{
    const float ex = r2.y, ey = r2.z;
    if (!(ex >= 0.0f)) return false;   // alpha below 1/255 everywhere (or a non-finite record)
    const float u = r0.x, v = r0.y;
    const float mx = ex + 1e-3f * ex + 0.01f, my = ey + 1e-3f * ey + 0.01f;
    if (u + mx < bx0 || u - mx > bx1 || v + my < by0 || v - my > by1) return false;
    const float du0 = bx0 - u, du1 = bx1 - u, dv0 = by0 - v, dv1 = by1 - v;
    if (du0 <= 0.0f && du1 >= 0.0f && dv0 <= 0.0f && dv1 >= 0.0f) return true;   // centre inside
    // the convex form is smallest on the boundary: minimise along each edge
    // (an approximate reciprocal moves the edge minimiser by an ulp, which
    // changes the form only to second order: far inside the margin below)
    const float A = r0.z, B = r0.w, C = r1.x;
    const float rho = -2.0f * r2.w;
    const float nba = -B * __builtin_amdgcn_rcpf(A), nbc = -B * __builtin_amdgcn_rcpf(C);
    float qmin = INFINITY;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const float x = e ? du1 : du0;
        const float y = fminf(fmaxf(nbc * x, dv0), dv1);
        qmin = fminf(qmin, (A * x) * x + (2.0f * B * x) * y + (C * y) * y);
    }
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const float y = e ? dv1 : dv0;
        const float x = fminf(fmaxf(nba * y, du0), du1);
        qmin = fminf(qmin, (A * x) * x + (2.0f * B * x) * y + (C * y) * y);
    }
    // rounding of this minimum and of the per-pixel power both grow with the
    // conditioning of the form; lam bounds the largest covariance eigenvalue
    const float lam = (ex * ex + ey * ey) / rho;
    const float gamma = 1e-5f * (1.0f + lam);
    if (!(gamma < 0.5f)) return true;
    return qmin * (1.0f - gamma) <= rho + 1e-3f * rho;
}

__global__ __launch_bounds__(256) void k_composite(const FrameParams* __restrict__ fp,
                                                   const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ sorted,
                                                   const float4* __restrict__ proj, float* __restrict__ image,
                                                   float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                                   uint4* __restrict__ wstats, uint32_t cap)
{
    __shared__ float4 s_a[4][64];   // per wave: u, v, -A/2, -B
    __shared__ float4 s_b[4][64];   // -C/2, o, threshold, r
    __shared__ float4 s_c[4][64];   // g, b, list position + 1 (bits), -

    const int32_t W = fp->cam.width, H = fp->cam.height, TX = fp->TX;
    const uint32_t tile = order[blockIdx.x];
    const uint32_t tx = tile % (uint32_t)TX, ty = tile / (uint32_t)TX;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t qx0 = tx * kTile + (wave & 1u) * 8u, qy0 = ty * kTile + (wave >> 1) * 8u;
    const uint32_t x = qx0 + (lane & 7u), y = qy0 + (lane >> 3);
    const bool inside = (int32_t)x < W && (int32_t)y < H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, bx1 = bx0 + 7.0f, by0 = (float)qy0 + 0.5f, by1 = by0 + 7.0f;
    const uint2 rg = ranges[tile];
    const uint32_t len = rg.y - rg.x;
    const unsigned long long lt = (1ull << lane) - 1ull;
    float4* const sa = s_a[wave];
    float4* const sb = s_b[wave];
    float4* const sc = s_c[wave];

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, nblend = 0, neval = len;
    bool done = !inside;

    for (uint32_t b0 = 0; b0 < len; b0 += 64) {
        if (__ballot(!done) == 0ull) break;
        const uint32_t k = b0 + lane;
        bool hit = false;
        float4 r0, r1, r2;
        if (k < len) {
            uint32_t a = sorted[rg.x + k];
            a = a < cap ? a : 0u;   // an index outside the active set would be a binning bug
            r0 = proj[3 * (size_t)a];
            r1 = proj[3 * (size_t)a + 1];
            r2 = proj[3 * (size_t)a + 2];
            hit = reaches_box(r0, r1, r2, bx0, bx1, by0, by1);
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            const uint32_t pos = (uint32_t)__popcll(m & lt);
            sa[pos] = make_float4(r0.x, r0.y, -0.5f * r0.z, -r0.w);
            sb[pos] = make_float4(-0.5f * r1.x, r1.y, r2.w, r1.z);
            sc[pos] = make_float4(r1.w, r2.x, __uint_as_float(k + 1u), 0.0f);
        }
        // the wave's own LDS slice: order its writes before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t n = (uint32_t)__popcll(m);
        if (!done) {
            for (uint32_t j = 0; j < n; j++) {
                const float4 g = sa[j];
                const float4 c = sb[j];
                float dx, dy, G;
                bool clamped;
                const float alpha = splat_alpha(g, c, px, py, dx, dy, G, clamped);
                if (alpha < 0.0f) continue;
                const float Tn = T * (1.0f - alpha);
                if (Tn < kTStop) {
                    done = true;
                    neval = __float_as_uint(sc[j].z);
                    break;
                }
                const float4 e = sc[j];
                const float wgt = alpha * T;
                cr = __builtin_fmaf(c.w, wgt, cr);
                cg = __builtin_fmaf(e.x, wgt, cg);
                cb = __builtin_fmaf(e.y, wgt, cb);
                T = Tn;
                last = __float_as_uint(e.z);
                nblend++;
            }
        }
        // every lane is past its reads before the next batch overwrites the slice
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
    // per-wave counters, one slot per (tile, quadrant)
    unsigned long long ev = neval;
    uint32_t bl = nblend;
    for (int off = 32; off > 0; off >>= 1) {
        ev += __shfl_xor(ev, off);
        bl += __shfl_xor(bl, off);
    }
    if (lane == 0) wstats[4 * tile + wave] = make_uint4((uint32_t)ev, (uint32_t)(ev >> 32), bl, 0u);
}

}  // namespace

hipError_t launch_composite(const Views& v, float* image, float* final_T, uint32_t* n_contrib, hipStream_t st)
{
    k_composite<<<v.lay.T, 256, 0, st>>>(v.params, v.ranges, v.order, v.sorted, v.proj, image, final_T, n_contrib,
                                         v.wstats, v.max_active);
    return hipGetLastError();
}

}  // namespace lodge
