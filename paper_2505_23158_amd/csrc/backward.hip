// Adjoint of lodge_render (the rasterizer's backward pass used by the
// per-level fine-tuning of the paper's supplementary "LOD structure
// optimization steps": only the parameters of G_l are updated).
//
// k_bwd_setup      zero the per-active 2-D gradient records.
// k_composite_bwd  one wave per 8 x 8 quadrant of a tile (four per block,
//                  never waiting for each other), one pixel per lane,
//                  walking the tile's sorted run back to front from the
//                  largest n_contrib of the quadrant, in batches of 64 whose
//                  entries are culled for the quadrant exactly as the
//                  compositor culls them.  The transmittance before entry k
//                  is recovered from the stored final T by division,
//                  T_k = T_{k+1} / (1 - alpha_k), rather than stored per pair.
//                  With S_k the colour behind entry k (plus T_final * bg):
//                    dC/dc_k = alpha_k T_k,  dC/dalpha_k = c_k T_k - S_k / (1 - alpha_k).
//                  The colour behind enters only through D = dC . S, so
//                  dC/dalpha_k = T_k (dC . c_k) - D / (1 - alpha_k), one
//                  reciprocal per pair.  Per entry the quadrant's nine
//                  gradients are summed over the wave by a transposed
//                  reduction (only where some pixel contributed) and added
//                  with one atomic instruction of nine lanes.
// k_project_bwd    one thread per visible active Gaussian whose 2-D gradient is
//                  not zero: the chain rule from
//                  (u, v, conic, o_eff, rgb) back through the 2-D filter, the
//                  EWA covariance, the camera and the Eq. 3 filter to the
//                  activated parameters; each Gaussian occurs once per frame,
//                  so its gradient is added without atomics.
#include "lodge_internal.hpp"
#include "splat.hpp"

namespace lodge {

namespace {

constexpr int kG2 = 12;   // floats per 2-D gradient record: u, v, A, B, C, o, r, g, b (+3 pad)

__global__ void k_bwd_setup(float* __restrict__ g2d, const uint32_t* __restrict__ count, uint32_t cap)
{
    const uint32_t n = min(*count, cap) * (uint32_t)kG2;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) g2d[i] = 0.0f;
}

// Lane exchanges of the reduction below.  permlane32_swap / permlane16_swap
// (gfx950) trade the upper half of the first operand with the lower half of
// the second, per 64 and per 32 lanes; the sum of the two results is then
// a + partner's a on the lower side and b + partner's b on the upper side.
__device__ __forceinline__ float keep_half32(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float keep_half16(float a, float b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int kCtrl>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, false));
}

constexpr int kRowMirror = 0x140;       // lane i of 16 reads lane 15 - i
constexpr int kRowHalfMirror = 0x141;   // lane i of 8 reads lane 7 - i
constexpr int kQuadXor2 = 0x4e;         // quad_perm (2, 3, 0, 1)
constexpr int kQuadXor1 = 0xb1;         // quad_perm (1, 0, 3, 2)

// Wave sum of nine per-lane values, transposed: each halving step splits the
// values between the two sides of a lane bit, each side keeping one part
// plus its partner's copy of that part, so a step moves half as many values
// as the one before (5 + 3 + 2 + 1 + 1 + 1 exchanges instead of 9 x 6).
// Lane l ends with the total of value sum9_slot(l) (valid when below 9).
__device__ __forceinline__ float wave_sum9(const float (&g)[9], uint32_t lane)
{
    float a[5];
#pragma unroll
    for (int j = 0; j < 4; j++) a[j] = keep_half32(g[j], g[5 + j]);   // bit 5: 0..4 | 5..8
    a[4] = keep_half32(g[4], 0.0f);
    float b[3];
#pragma unroll
    for (int j = 0; j < 2; j++) b[j] = keep_half16(a[j], a[3 + j]);   // bit 4: 0..2 | 3..4
    b[2] = keep_half16(a[2], 0.0f);
    const bool b3 = (lane >> 3) & 1u, b2 = (lane >> 2) & 1u;
    float c[2];
    c[0] = (b3 ? b[2] : b[0]) + dpp<kRowMirror>(b3 ? b[0] : b[2]);   // bit 3: 0..1 | 2
    c[1] = (b3 ? 0.0f : b[1]) + dpp<kRowMirror>(b3 ? b[1] : 0.0f);
    float d = (b2 ? c[1] : c[0]) + dpp<kRowHalfMirror>(b2 ? c[0] : c[1]);   // bit 2: 0 | 1
    d += dpp<kQuadXor2>(d);
    d += dpp<kQuadXor1>(d);
    return d;
}

// The value whose total lane l holds after wave_sum9 (9 or more: none).
__device__ __forceinline__ uint32_t sum9_slot(uint32_t lane)
{
    const uint32_t b5 = (lane >> 5) & 1u, b4 = (lane >> 4) & 1u, b3 = (lane >> 3) & 1u, b2 = (lane >> 2) & 1u;
    const uint32_t low = 2u * b3 + b2, mid = 3u * b4 + low;
    return (low < 3u && mid < 5u) ? 5u * b5 + mid : 9u;
}

__global__ __launch_bounds__(256) void k_composite_bwd(const FrameParams* __restrict__ fp,
                                                       const uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ sorted,
                                                       const float4* __restrict__ proj,
                                                       const float* __restrict__ final_T,
                                                       const uint32_t* __restrict__ n_contrib,
                                                       const float* __restrict__ dL, float* __restrict__ g2d,
                                                       uint32_t cap)
{
    // the adjoint matches the FP64 oracle within a tolerance, not bit for bit, so products and sums may
    // fuse; the decisions that must equal the compositor's (power, alpha, which pixels blend) come from
    // splat_power's explicit FMAs and plain comparisons, which contraction leaves as they are
#pragma clang fp contract(fast)
    __shared__ float4 s_rec[4][3][64];     // per wave, by batch slot: geo, col, (g, b, -, -)
    __shared__ uint32_t s_a[4][64];        // active index of each slot
    __shared__ uint8_t s_idx[4][64];       // slots that reach the quadrant, in list order

    const int32_t W = fp->cam.width, H = fp->cam.height, TX = fp->TX;
    const uint32_t tile = order[blockIdx.x];
    const uint32_t tx = tile % (uint32_t)TX, ty = tile / (uint32_t)TX;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t qx0 = tx * kTile + (wave & 1u) * 8u, qy0 = ty * kTile + (wave >> 1) * 8u;
    const uint32_t x = qx0 + (lane & 7u), y = qy0 + (lane >> 3);
    const bool inside = (int32_t)x < W && (int32_t)y < H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const uint2 rg = ranges[tile];
    const unsigned long long lt = (1ull << lane) - 1ull;
    float4* const sa = s_rec[wave][0];
    float4* const sb = s_rec[wave][1];
    float4* const sc = s_rec[wave][2];

    const size_t HW = (size_t)W * H, p = (size_t)y * W + x;
    uint32_t last = 0;
    float T = 1.0f, dC0 = 0.0f, dC1 = 0.0f, dC2 = 0.0f;
    if (inside) {
        last = n_contrib[p];
        T = final_T[p];
        dC0 = dL[p];
        dC1 = dL[HW + p];
        dC2 = dL[2 * HW + p];
    }
    const float* bg = fp->cam.bg;
    float D = T * ((dC0 * bg[0] + dC1 * bg[1]) + dC2 * bg[2]);   // dC . (colour behind the current entry)
    const uint32_t slot = sum9_slot(lane);
    const bool adds = (lane & 3u) == 0u && slot < 9u;

    // the quadrant's entries that any pixel blended lie in [0, end)
    uint32_t end = last;
    for (int off = 32; off > 0; off >>= 1) end = max(end, (uint32_t)__shfl_xor(end, off));
    end = min(__builtin_amdgcn_readfirstlane(end), rg.y - rg.x);

    for (uint32_t b0 = end > 0 ? ((end - 1) / 64) * 64 : 0; end > 0;) {
        // stage the batch [b0, b0 + 64) and keep the slots that reach the quadrant
        const uint32_t k = b0 + lane;
        bool hit = false;
        if (k < end) {
            uint32_t a = sorted[rg.x + k];
            a = a < cap ? a : 0u;   // an index outside the active set would be a binning bug
            const float4 r0 = proj[3 * (size_t)a], r1 = proj[3 * (size_t)a + 1], r2 = proj[3 * (size_t)a + 2];
            sa[lane] = r0;
            sb[lane] = r1;
            sc[lane] = make_float4(r2.x, r2.y, 0.0f, 0.0f);
            s_a[wave][lane] = a;
            hit = reaches(box_test(r0, r1, r2), bx0, bx0 + 7.0f, by0, by0 + 7.0f);
        }
        const unsigned long long m = __ballot(hit);
        if (hit) s_idx[wave][__popcll(m & lt)] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // back to front over the kept slots
        for (int jj = (int)__popcll(m) - 1; jj >= 0; jj--) {
            const uint32_t e = s_idx[wave][jj];
            const uint32_t kk = b0 + e;
            // every lane evaluates the entry; those that did not blend it (past their last entry, or alpha
            // below 1/255) keep T and D and give zero gradients through the selects
            const float4 geo = sa[e];
            const float4 col = sb[e];
            const float4 gb = sc[e];
            float dx, dy;
            const float power = splat_power(geo, col, px, py, dx, dy);
            const float G = __expf(power);
            const float og = col.y * G;
            const bool clamped = og > kAlphaMax;
            const float alpha = clamped ? kAlphaMax : og;
            const bool contrib = kk < last && !(power > 0.0f) && alpha >= kAlphaMin;
            const float r = __builtin_amdgcn_rcpf(1.0f - alpha);
            const float Tk = T * r;                   // transmittance before this entry
            const float wgt = alpha * Tk;
            const float cd = (dC0 * col.w + dC1 * gb.x) + dC2 * gb.y;
            const float dalpha = Tk * cd - D * r;
            T = contrib ? Tk : T;
            D = contrib ? D + wgt * cd : D;
            const float wc = contrib ? wgt : 0.0f;
            float g[9];
            g[6] = wc * dC0;
            g[7] = wc * dC1;
            g[8] = wc * dC2;
            g[5] = contrib && !clamped ? dalpha * G : 0.0f;
            const float dpow = g[5] * col.y;
            // power = -A/2 dx^2 - C/2 dy^2 - B dx dy, staged as geo.z = -A/2, geo.w = -B, col.x = -C/2
            g[2] = -0.5f * dx * dx * dpow;
            g[3] = -dx * dy * dpow;
            g[4] = -0.5f * dy * dy * dpow;
            g[0] = (2.0f * geo.z * dx + geo.w * dy) * dpow;
            g[1] = (2.0f * col.x * dy + geo.w * dx) * dpow;
            if (__ballot(contrib) != 0ull) {
                const float sum = wave_sum9(g, lane);
                if (adds && sum != 0.0f) atomicAdd(g2d + (size_t)s_a[wave][e] * kG2 + slot, sum);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (b0 == 0) break;
        b0 -= 64;
    }
}

// Real SH basis to degree 3 (same convention as the projection kernel) and
// its derivatives with respect to the (unnormalised) direction components.
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f;
constexpr float kC2b = 0.31539156525252005f;
constexpr float kC2c = 0.5462742152960396f;
constexpr float kC3a = 0.5900435899266435f;
constexpr float kC3b = 2.890611442640554f;
constexpr float kC3c = 0.4570457994644658f;
constexpr float kC3d = 0.3731763325901154f;
constexpr float kC3e = 1.445305721320277f;

__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float* Y, float (*dY)[3])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kC0;                                   dY[0][0] = 0; dY[0][1] = 0; dY[0][2] = 0;
    Y[1] = -kC1 * y;                              dY[1][0] = 0; dY[1][1] = -kC1; dY[1][2] = 0;
    Y[2] = kC1 * z;                               dY[2][0] = 0; dY[2][1] = 0; dY[2][2] = kC1;
    Y[3] = -kC1 * x;                              dY[3][0] = -kC1; dY[3][1] = 0; dY[3][2] = 0;
    Y[4] = kC2a * x * y;                          dY[4][0] = kC2a * y; dY[4][1] = kC2a * x; dY[4][2] = 0;
    Y[5] = -kC2a * y * z;                         dY[5][0] = 0; dY[5][1] = -kC2a * z; dY[5][2] = -kC2a * y;
    Y[6] = kC2b * (2.0f * zz - xx - yy);          dY[6][0] = -2.0f * kC2b * x; dY[6][1] = -2.0f * kC2b * y;
                                                  dY[6][2] = 4.0f * kC2b * z;
    Y[7] = -kC2a * x * z;                         dY[7][0] = -kC2a * z; dY[7][1] = 0; dY[7][2] = -kC2a * x;
    Y[8] = kC2c * (xx - yy);                      dY[8][0] = 2.0f * kC2c * x; dY[8][1] = -2.0f * kC2c * y; dY[8][2] = 0;
    Y[9] = -kC3a * y * (3.0f * xx - yy);          dY[9][0] = -6.0f * kC3a * x * y;
                                                  dY[9][1] = -3.0f * kC3a * (xx - yy); dY[9][2] = 0;
    Y[10] = kC3b * x * y * z;                     dY[10][0] = kC3b * y * z; dY[10][1] = kC3b * x * z;
                                                  dY[10][2] = kC3b * x * y;
    Y[11] = -kC3c * y * (4.0f * zz - xx - yy);    dY[11][0] = 2.0f * kC3c * x * y;
                                                  dY[11][1] = -kC3c * (4.0f * zz - xx - 3.0f * yy);
                                                  dY[11][2] = -8.0f * kC3c * y * z;
    Y[12] = kC3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
                                                  dY[12][0] = -6.0f * kC3d * x * z; dY[12][1] = -6.0f * kC3d * y * z;
                                                  dY[12][2] = kC3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -kC3c * x * (4.0f * zz - xx - yy);    dY[13][0] = -kC3c * (4.0f * zz - 3.0f * xx - yy);
                                                  dY[13][1] = 2.0f * kC3c * x * y; dY[13][2] = -8.0f * kC3c * x * z;
    Y[14] = kC3e * z * (xx - yy);                 dY[14][0] = 2.0f * kC3e * x * z; dY[14][1] = -2.0f * kC3e * y * z;
                                                  dY[14][2] = kC3e * (xx - yy);
    Y[15] = -kC3a * x * (xx - 3.0f * yy);         dY[15][0] = -3.0f * kC3a * (xx - yy);
                                                  dY[15][1] = 6.0f * kC3a * x * y; dY[15][2] = 0;
}

struct GradsArg {
    lodge_grads g[LODGE_MAX_LEVELS];
};

__global__ __launch_bounds__(256) void k_project_bwd(LevelsArg lv, GradsArg ga, int32_t grad_level,
                                                     const uint32_t* __restrict__ ids, const float* __restrict__ wsel,
                                                     const uint32_t* __restrict__ count, uint32_t cap,
                                                     const FrameParams* __restrict__ fp,
                                                     const uint2* __restrict__ rect, const float* __restrict__ g2d)
{
    // products and sums may fuse here (the adjoint matches the FP64 oracle within a tolerance): the
    // recomputed forward quantities then differ from the projection's by rounding, which only moves a
    // Gaussian exactly on the Jacobian clamp to the other one-sided gradient
#pragma clang fp contract(fast)
    const uint32_t n_act = min(*count, cap);
    const lodge_camera& cam = fp->cam;
    const float s2d = fp->s2d;
    const int compensate = fp->compensate;
    for (uint32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n_act; a += gridDim.x * blockDim.x) {
        const uint2 rc = rect[a];
        if ((rc.y & 0xffffu) <= (rc.x & 0xffffu)) continue;   // culled: empty rectangle
        const float4* const g4 = reinterpret_cast<const float4*>(g2d + (size_t)a * kG2);
        const float4 gq0 = g4[0], gq1 = g4[1], gq2 = g4[2];
        // a Gaussian that no pixel blended (hidden, or below 1/255 everywhere) has a zero 2-D
        // gradient and so a zero gradient for every parameter: nothing to read or add
        if (gq0.x == 0.0f && gq0.y == 0.0f && gq0.z == 0.0f && gq0.w == 0.0f && gq1.x == 0.0f &&
            gq1.y == 0.0f && gq1.z == 0.0f && gq1.w == 0.0f && gq2.x == 0.0f)
            continue;
        const uint32_t gid = ids[a];
        int l = 0;
#pragma unroll
        for (int j = 1; j < LODGE_MAX_LEVELS; j++)
            if (j < lv.L && gid >= lv.lv[j].base) l = j;
        if (grad_level >= 0 && l != grad_level) continue;
        const LevelDev& L = lv.lv[l];
        const lodge_grads& G = ga.g[l];
        const size_t n = L.n;
        const uint32_t i = gid - L.base;
        const float gu = gq0.x, gv = gq0.y, gA = gq0.z, gB = gq0.w, gC = gq1.x, go_eff = gq1.y;
        const float grgb[3] = {gq1.z, gq1.w, gq2.x};

        // ---- forward recomputation (as in the projection kernel)
        const float mx = L.mean[i], my = L.mean[n + i], mz = L.mean[2 * n + i];
        const float s[3] = {L.scale[i], L.scale[n + i], L.scale[2 * n + i]};
        const float qw = L.quat[i], qx = L.quat[n + i], qy = L.quat[2 * n + i], qz = L.quat[3 * n + i];
        const float op = L.opacity[i], w = wsel[a], var = L.var;
        const float* Wc = cam.R;
        const float tx = ((Wc[0] * mx + Wc[1] * my) + Wc[2] * mz) + cam.t[0];
        const float ty = ((Wc[3] * mx + Wc[4] * my) + Wc[5] * mz) + cam.t[1];
        const float tz = ((Wc[6] * mx + Wc[7] * my) + Wc[8] * mz) + cam.t[2];
        const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
        const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
        const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
        const float R[9] = {1.0f - 2.0f * (yy + zz), 2.0f * (xy - wz),        2.0f * (xz + wy),
                            2.0f * (xy + wz),        1.0f - 2.0f * (xx + zz), 2.0f * (yz - wx),
                            2.0f * (xz - wy),        2.0f * (yz + wx),        1.0f - 2.0f * (xx + yy)};
        const float v[3] = {s[0] * s[0] + var, s[1] * s[1] + var, s[2] * s[2] + var};
        float S[9];
        for (int p = 0; p < 3; p++)
            for (int q = p; q < 3; q++) {
                const float e = ((R[3 * p] * v[0]) * R[3 * q] + (R[3 * p + 1] * v[1]) * R[3 * q + 1])
                                + (R[3 * p + 2] * v[2]) * R[3 * q + 2];
                S[3 * p + q] = e;
                S[3 * q + p] = e;
            }
        const float comp3 = sqrtf(((s[0] * s[0] / v[0]) * (s[1] * s[1] / v[1])) * (s[2] * s[2] / v[2]));
        const float ix = tx / tz, iy = ty / tz;
        float rx = ix, ry = iy;
        bool clx = false, cly = false;
        if (rx < -cam.lim_x) { rx = -cam.lim_x; clx = true; }
        if (rx > cam.lim_x) { rx = cam.lim_x; clx = true; }
        if (ry < -cam.lim_y) { ry = -cam.lim_y; cly = true; }
        if (ry > cam.lim_y) { ry = cam.lim_y; cly = true; }
        const float J00 = cam.fx / tz, J02 = -((cam.fx * rx) / tz);
        const float J11 = cam.fy / tz, J12 = -((cam.fy * ry) / tz);
        float M[6];
        for (int j = 0; j < 3; j++) {
            M[j] = J00 * Wc[j] + J02 * Wc[6 + j];
            M[3 + j] = J11 * Wc[3 + j] + J12 * Wc[6 + j];
        }
        float T6[6];
        for (int r = 0; r < 2; r++)
            for (int j = 0; j < 3; j++)
                T6[3 * r + j] = (M[3 * r] * S[j] + M[3 * r + 1] * S[3 + j]) + M[3 * r + 2] * S[6 + j];
        const float a0 = (T6[0] * M[0] + T6[1] * M[1]) + T6[2] * M[2];
        const float b = (T6[0] * M[3] + T6[1] * M[4]) + T6[2] * M[5];
        const float c0 = (T6[3] * M[3] + T6[4] * M[4]) + T6[5] * M[5];
        const float aa = a0 + s2d, cc = c0 + s2d;
        const float det0 = a0 * c0 - b * b;
        const float det = aa * cc - b * b;
        const float comp2 = compensate ? sqrtf((det0 > 0.0f ? det0 : 0.0f) / det) : 1.0f;

        float dmu[3] = {0.0f, 0.0f, 0.0f};

        // ---- colour: rgb = max(0, sum_k sh_k Y_k(dir) + 1/2), dir = (mu - pos) / |mu - pos|
        // Every index below is a compile-time constant (coefficients past the level's
        // degree are zero and never loaded), so the basis stays in registers.
        const float d0 = mx - cam.pos[0], d1 = my - cam.pos[1], d2 = mz - cam.pos[2];
        const float dn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
        const float idn = 1.0f / dn;
        const float ux = d0 * idn, uy = d1 * idn, uz = d2 * idn;
        float Y[kMaxSh], dY[kMaxSh][3];
        sh_basis_grad(ux, uy, uz, Y, dY);
        const int nb = (L.sh_degree + 1) * (L.sh_degree + 1);
        float coef[kMaxSh][3];
#pragma unroll
        for (int k = 0; k < kMaxSh; k++)
#pragma unroll
            for (int ch = 0; ch < 3; ch++) coef[k][ch] = k < nb ? L.sh[((size_t)(k * 3 + ch)) * n + i] : 0.0f;
        // the gradient reaches a channel only where its colour was not clamped at 0
        float m[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < kMaxSh; k++) acc = acc + coef[k][ch] * Y[k];
            m[ch] = acc + 0.5f > 0.0f ? grgb[ch] : 0.0f;
        }
        float ddir[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < kMaxSh; k++) {
            const float wk = (m[0] * coef[k][0] + m[1] * coef[k][1]) + m[2] * coef[k][2];
            ddir[0] += wk * dY[k][0];
            ddir[1] += wk * dY[k][1];
            ddir[2] += wk * dY[k][2];
        }
        if (G.sh) {
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                if (m[ch] == 0.0f) continue;
#pragma unroll
                for (int k = 0; k < kMaxSh; k++)
                    if (k < nb) G.sh[((size_t)(k * 3 + ch)) * n + i] += m[ch] * Y[k];
            }
        }
        const float dot = ddir[0] * ux + ddir[1] * uy + ddir[2] * uz;
        dmu[0] += (ddir[0] - ux * dot) * idn;
        dmu[1] += (ddir[1] - uy * dot) * idn;
        dmu[2] += (ddir[2] - uz * dot) * idn;

        // ---- opacity: o_eff = o w comp3 comp2
        if (G.opacity) G.opacity[i] += go_eff * w * comp3 * comp2;
        const float dcomp3 = go_eff * op * w * comp2;
        const float dcomp2 = go_eff * op * w * comp3;

        // ---- conic (A, B, C) = (c, -b, a) / det, a = a0 + s2d, c = c0 + s2d
        const float idet = 1.0f / det, idet2 = idet * idet;
        float ga_ = (gA * (-(cc * cc)) + gB * (b * cc) + gC * (-(b * b))) * idet2;
        float gc_ = (gA * (-(b * b)) + gB * (b * aa) + gC * (-(aa * aa))) * idet2;
        float gb_ = (gA * (2.0f * b * cc) + gB * (-(aa * cc + b * b)) + gC * (2.0f * aa * b)) * idet2;
        if (compensate && det0 > 0.0f) {
            const float ddet0 = 0.5f * dcomp2 * idet / comp2;
            const float ddet = -0.5f * dcomp2 * comp2 * idet;
            ga_ += ddet0 * c0 + ddet * cc;
            gc_ += ddet0 * a0 + ddet * aa;
            gb_ += -2.0f * b * (ddet0 + ddet);
        }
        // ---- Sigma' = M Sigma M^T
        const float Gp[4] = {ga_, 0.5f * gb_, 0.5f * gb_, gc_};
        float dS[9];
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                float acc = 0.0f;
                for (int p = 0; p < 2; p++)
                    for (int q = 0; q < 2; q++) acc += M[3 * p + r] * Gp[2 * p + q] * M[3 * q + c];
                dS[3 * r + c] = acc;
            }
        float dM[6];
        for (int p = 0; p < 2; p++)
            for (int c = 0; c < 3; c++) {
                float acc = 0.0f;
                for (int q = 0; q < 2; q++)
                    for (int k = 0; k < 3; k++) acc += 2.0f * Gp[2 * p + q] * M[3 * q + k] * S[3 * k + c];
                dM[3 * p + c] = acc;
            }
        // ---- M = J W
        float dJ00 = 0.0f, dJ02 = 0.0f, dJ11 = 0.0f, dJ12 = 0.0f;
        for (int c = 0; c < 3; c++) {
            dJ00 += dM[c] * Wc[c];
            dJ02 += dM[c] * Wc[6 + c];
            dJ11 += dM[3 + c] * Wc[3 + c];
            dJ12 += dM[3 + c] * Wc[6 + c];
        }
        const float itz = 1.0f / tz, itz2 = itz * itz, itz3 = itz2 * itz;
        const float fx2 = cam.fx * itz2, fy2 = cam.fy * itz2;   // f / tz^2
        float dtx = 0.0f, dty = 0.0f, dtz = 0.0f;
        dtz += dJ00 * (-fx2) + dJ11 * (-fy2);
        if (clx) dtz += dJ02 * (rx * fx2);
        else { dtx += dJ02 * (-fx2); dtz += dJ02 * (2.0f * cam.fx * tx * itz3); }
        if (cly) dtz += dJ12 * (ry * fy2);
        else { dty += dJ12 * (-fy2); dtz += dJ12 * (2.0f * cam.fy * ty * itz3); }
        dtx += gu * cam.fx * itz;
        dtz += gu * (-tx * fx2);
        dty += gv * cam.fy * itz;
        dtz += gv * (-ty * fy2);
        for (int j = 0; j < 3; j++) dmu[j] += Wc[j] * dtx + Wc[3 + j] * dty + Wc[6 + j] * dtz;

        // ---- Sigma = R diag(v) R^T, v_j = s_j^2 + var, comp3 = sqrt(prod s_j^2 / v_j)
        float dR[9];
        float ds[3];
        for (int j = 0; j < 3; j++) {
            float acc = 0.0f;
            for (int p = 0; p < 3; p++)
                for (int q = 0; q < 3; q++) acc += R[3 * p + j] * dS[3 * p + q] * R[3 * q + j];
            ds[j] = acc * 2.0f * s[j] + dcomp3 * comp3 * var / (s[j] * v[j]);
        }
        for (int p = 0; p < 3; p++)
            for (int j = 0; j < 3; j++) {
                float acc = 0.0f;
                for (int q = 0; q < 3; q++) acc += dS[3 * p + q] * R[3 * q + j];
                dR[3 * p + j] = 2.0f * acc * v[j];
            }
        // ---- R(q), q = (w, x, y, z) as given
        const float dqw = dR[1] * (-2.0f * qz) + dR[2] * (2.0f * qy) + dR[3] * (2.0f * qz) + dR[5] * (-2.0f * qx) +
                          dR[6] * (-2.0f * qy) + dR[7] * (2.0f * qx);
        const float dqx = dR[1] * (2.0f * qy) + dR[2] * (2.0f * qz) + dR[3] * (2.0f * qy) + dR[4] * (-4.0f * qx) +
                          dR[5] * (-2.0f * qw) + dR[6] * (2.0f * qz) + dR[7] * (2.0f * qw) + dR[8] * (-4.0f * qx);
        const float dqy = dR[0] * (-4.0f * qy) + dR[1] * (2.0f * qx) + dR[2] * (2.0f * qw) + dR[3] * (2.0f * qx) +
                          dR[5] * (2.0f * qz) + dR[6] * (-2.0f * qw) + dR[7] * (2.0f * qz) + dR[8] * (-4.0f * qy);
        const float dqz = dR[0] * (-4.0f * qz) + dR[1] * (-2.0f * qw) + dR[2] * (2.0f * qx) + dR[3] * (2.0f * qw) +
                          dR[4] * (-4.0f * qz) + dR[5] * (2.0f * qy) + dR[6] * (2.0f * qx) + dR[7] * (2.0f * qy);

        if (G.mean) {
            G.mean[i] += dmu[0];
            G.mean[n + i] += dmu[1];
            G.mean[2 * n + i] += dmu[2];
        }
        if (G.scale) {
            G.scale[i] += ds[0];
            G.scale[n + i] += ds[1];
            G.scale[2 * n + i] += ds[2];
        }
        if (G.quat) {
            G.quat[i] += dqw;
            G.quat[n + i] += dqx;
            G.quat[2 * n + i] += dqy;
            G.quat[3 * n + i] += dqz;
        }
    }
}

}  // namespace

hipError_t launch_backward(const LevelsArg& lv, const lodge_selection& sel, const Views& v, const float* final_T,
                           const uint32_t* n_contrib, const float* dL_dimage, int32_t grad_level,
                           const lodge_grads* grads, hipStream_t st, void* const* events)
{
    auto mark = [&](int k) -> hipError_t {
        return events ? hipEventRecord(static_cast<hipEvent_t>(events[k]), st) : hipSuccess;
    };
    GradsArg ga{};
    for (int l = 0; l < lv.L; l++) ga.g[l] = grads[l];
    uint32_t blocks = std::min<uint32_t>(2048, std::max<uint32_t>(1, (v.max_active * (uint32_t)kG2 + 255) / 256));
    k_bwd_setup<<<blocks, 256, 0, st>>>(v.g2d, sel.count, sel.cap);
    hipError_t e = mark(0);
    if (e != hipSuccess) return e;
    k_composite_bwd<<<v.lay.T, 256, 0, st>>>(v.params, v.ranges, v.order, v.sorted, v.proj, final_T, n_contrib,
                                             dL_dimage, v.g2d, v.max_active);
    if ((e = mark(1)) != hipSuccess) return e;
    blocks = std::min<uint32_t>(4096, std::max<uint32_t>(1, (v.max_active + 255) / 256));
    k_project_bwd<<<blocks, 256, 0, st>>>(lv, ga, grad_level, sel.ids, sel.w, sel.count, sel.cap, v.params, v.rect,
                                          v.g2d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return mark(2);
}

}  // namespace lodge
