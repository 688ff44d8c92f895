// Per-(pixel, splat) evaluation shared by the compositing kernel and its
// adjoint, so both take exactly the same skip / clamp / stop decisions.
//
// A staged splat is three LDS words: geo = (u, v, -A/2, -B),
// col = (-C/2, o_eff, skip threshold, r), gb = (g, b), where (A, B, C) is the
// conic and the skip threshold, from the projection, is ln(1 / (255 o_eff))
// - 1e-3 (+inf when o_eff <= 0): a power below it cannot give alpha >= 1/255,
// so exp is not evaluated for it.  Explicit fmaf keeps the arithmetic
// identical wherever this is inlined (the files are built without FMA
// contraction).
#pragma once

#include <hip/hip_runtime.h>

namespace lodge {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 0.0001f;

__device__ __forceinline__ void stage_splat(const float4* __restrict__ proj, uint32_t a, float4& geo, float4& col,
                                            float2& gb)
{
    const float4 r0 = proj[3 * (size_t)a];
    const float4 r1 = proj[3 * (size_t)a + 1];
    const float4 r2 = proj[3 * (size_t)a + 2];
    geo = make_float4(r0.x, r0.y, -0.5f * r0.z, -r0.w);
    col = make_float4(-0.5f * r1.x, r1.y, r2.w, r1.z);
    gb = make_float2(r1.w, r2.x);
}

__device__ __forceinline__ float splat_power(const float4& geo, const float4& col, float px, float py, float& dx,
                                             float& dy)
{
    dx = geo.x - px;
    dy = geo.y - py;
    return __builtin_fmaf(geo.z * dx, dx, __builtin_fmaf(col.x * dy, dy, (geo.w * dx) * dy));
}

// alpha of the splat at this pixel, or a negative value if it is skipped
// (power > 0, power below the threshold, or alpha < 1/255).  G and the clamp
// state are returned for the adjoint.
__device__ __forceinline__ float splat_alpha(const float4& geo, const float4& col, float px, float py, float& dx,
                                             float& dy, float& G, bool& clamped)
{
    const float power = splat_power(geo, col, px, py, dx, dy);
    if (power > 0.0f || power < col.z) return -1.0f;
    G = __expf(power);
    const float og = col.y * G;
    clamped = og > kAlphaMax;
    const float alpha = clamped ? kAlphaMax : og;
    return alpha < kAlphaMin ? -1.0f : alpha;
}

// The same decision as splat_alpha without branches: alpha (clamped at
// kAlphaMax) and whether the pair counts; exp is evaluated either way.
__device__ __forceinline__ bool splat_keep(const float4& geo, const float4& col, float px, float py, float& alpha)
{
    float dx, dy;
    const float power = splat_power(geo, col, px, py, dx, dy);
    const float og = col.y * __expf(power);
    alpha = og > kAlphaMax ? kAlphaMax : og;
    return !(power > 0.0f || power < col.z) && !(alpha < kAlphaMin);
}

}  // namespace lodge
