// Per-(pixel, splat) evaluation shared by the compositing kernel and its
// adjoint, so both take exactly the same skip / clamp / stop decisions.
//
// A projected record is three float4, in the form the compositor reads:
// (u, v, -A/2, -B), (-C/2, o_eff, skip threshold, r), (g, b, ex, ey), where
// (A, B, C) is the conic, (ex, ey) the half-extents of the ellipse where
// alpha can reach 1/255, and the skip threshold, from the projection, is
// ln(1 / (255 o_eff)) - 1e-3 (+inf when o_eff <= 0): a power below it cannot
// give alpha >= 1/255, so exp is not evaluated for it.  Explicit fmaf keeps
// the arithmetic identical wherever this is inlined (the files are built
// without FMA contraction).
#pragma once

#include <hip/hip_runtime.h>

namespace lodge {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 0.0001f;

__device__ __forceinline__ float splat_power(const float4& geo, const float4& col, float px, float py, float& dx,
                                             float& dy)
{
    dx = geo.x - px;
    dy = geo.y - py;
    return __builtin_fmaf(dx, __builtin_fmaf(geo.w, dy, geo.z * dx), (col.x * dy) * dy);
}

// Whether the pair counts, and its alpha (clamped at kAlphaMax), without
// branches: the pair counts when power <= 0 and alpha >= amin.  exp is
// evaluated either way, so the splat's power threshold is not tested: a
// power below it gives o exp(power) < e^-0.001 / 255, far enough below
// 1/255 for any rounding of exp, and the alpha test rejects the pair.  amin
// is kAlphaMin, or +inf for a pixel that takes no more splats (every finite
// alpha is then below it).
__device__ __forceinline__ bool splat_keep(const float4& geo, const float4& col, float px, float py, float amin,
                                           float& alpha)
{
    float dx, dy;
    const float power = splat_power(geo, col, px, py, dx, dy);
    const float og = col.y * __expf(power);
    alpha = fminf(og, kAlphaMax);
    return !(power > 0.0f) && !(alpha < amin);
}

// Culling of a splat against a box of pixel centres, shared by the
// compositor and its adjoint: a splat rejected for a box is one that no
// pixel of the box would keep.  Per-splat terms of the test:
struct BoxTest {
    float u, v, mx, my;   // centre and bounding half-extents (with margin)
    float A, B, C;        // conic
    float nba, nbc;       // edge minimisers: x = -B y / A, y = -B x / C
    float lim;            // accept if the minimum of the form is <= lim
    bool any;             // alpha can reach 1/255 somewhere
};

// r0, r1, r2: a projected record (above); alpha >= 1/255 needs
// q(d) = A dx^2 + 2B dx dy + C dy^2 <= -2 thr.  The conic is recovered by
// exact scalings of the stored coefficients.
__device__ __forceinline__ BoxTest box_test(const float4& r0, const float4& r1, const float4& r2)
{
    BoxTest b;
    const float ex = r2.z, ey = r2.w;
    b.any = ex >= 0.0f;   // false: alpha below 1/255 everywhere (or a non-finite record)
    b.u = r0.x;
    b.v = r0.y;
    b.mx = ex + 1e-3f * ex + 0.01f;
    b.my = ey + 1e-3f * ey + 0.01f;
    b.A = -2.0f * r0.z;
    b.B = -r0.w;
    b.C = -2.0f * r1.x;
    // an approximate reciprocal moves an edge minimiser by an ulp, which
    // changes the form only to second order: far inside the margin below
    b.nba = -b.B * __builtin_amdgcn_rcpf(b.A);
    b.nbc = -b.B * __builtin_amdgcn_rcpf(b.C);
    // rounding of the minimum and of the per-pixel power both grow with the
    // conditioning of the form; lam bounds the largest covariance eigenvalue
    // (approximate reciprocals: their ulp errors are far inside these margins)
    const float rho = -2.0f * r1.z;
    const float lam = (ex * ex + ey * ey) * __builtin_amdgcn_rcpf(rho);
    const float gamma = 1.001e-5f * (1.0f + lam);
    b.lim = gamma < 0.5f ? (rho + 1e-3f * rho) * __builtin_amdgcn_rcpf(1.0f - gamma) : INFINITY;
    return b;
}

// Does the bounding box of the splat's alpha >= 1/255 ellipse meet [bx0, bx1] x [by0, by1]?
__device__ __forceinline__ bool box_overlaps(const BoxTest& b, float bx0, float bx1, float by0, float by1)
{
    return !(b.u + b.mx < bx0 || b.u - b.mx > bx1 || b.v + b.my < by0 || b.v - b.my > by1);
}

// Can the splat reach alpha >= 1/255 at a point of [bx0, bx1] x [by0, by1]?
__device__ __forceinline__ bool reaches(const BoxTest& b, float bx0, float bx1, float by0, float by1)
{
    if (!b.any || !box_overlaps(b, bx0, bx1, by0, by1)) return false;
    const float du0 = bx0 - b.u, du1 = bx1 - b.u, dv0 = by0 - b.v, dv1 = by1 - b.v;
    if (du0 <= 0.0f && du1 >= 0.0f && dv0 <= 0.0f && dv1 >= 0.0f) return true;   // centre inside
    // the convex form is smallest on the boundary: minimise along each edge
    float qmin = INFINITY;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const float x = e ? du1 : du0;
        const float y = fminf(fmaxf(b.nbc * x, dv0), dv1);
        qmin = fminf(qmin, (b.A * x) * x + (2.0f * b.B * x) * y + (b.C * y) * y);
    }
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const float y = e ? dv1 : dv0;
        const float x = fminf(fmaxf(b.nba * y, du0), du1);
        qmin = fminf(qmin, (b.A * x) * x + (2.0f * b.B * x) * y + (b.C * y) * y);
    }
    return qmin <= b.lim;
}

}  // namespace lodge
