// Projection of the active Gaussians (LODGE Sec. 3 "Preliminaries: 3D
// Gaussian Splatting": EWA splatting of mean and covariance; Eq. 3: the
// level's 3-D smoothing filter with its opacity factor; supplementary
// "Details on training the full representation": the renderer's 2-D
// screen-space filter; Eq. 4: the chunk weight modulates opacity).
//
// Each wave takes chunks of 64 consecutive actives (grid-stride over the
// chunks), one per lane.  Geometry first: the mean, selection id and weight
// are read; Gaussians behind the near plane stop there, the others read
// scale, rotation and opacity.  Each active writes its depth, tile rectangle
// and tile count (0 when culled), and each chunk writes its tile total (the
// first level of the instance-offset scan).  A visible Gaussian joins the
// wave's LDS queue with its view direction and the geometry of its
// compositing record (centre, conic, opacity, the power below which alpha
// cannot reach 1/255, the half-extents of the ellipse where it can).  Colour
// is evaluated from the queue 64 at a time, so the 48 SH loads and the basis
// run with every lane busy rather than on the few visible lanes of each
// chunk, and each record is then written whole, once (not its geometry
// first and its colour into the same lines later).
// The front/visible counters are reduced per block and added once.
//
// Built with -ffp-contract=off: the rectangle and depth (which decide tile
// membership and sort keys) are evaluated op for op as the oracle defines
// them.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

// Real SH basis to degree 3 with the sign convention of include/lodge.h's
// renderer: k1 = -c1 y, k2 = c1 z, k3 = -c1 x, k4 = c2a xy, k5 = -c2a yz,
// k6 = c2b (2z^2 - x^2 - y^2), k7 = -c2a xz, k8 = c2c (x^2 - y^2),
// k9 = -c3a y(3x^2 - y^2), k10 = c3b xyz, k11 = -c3c y(4z^2 - x^2 - y^2),
// k12 = c3d z(2z^2 - 3x^2 - 3y^2), k13 = -c3c x(4z^2 - x^2 - y^2),
// k14 = c3e z(x^2 - y^2), k15 = -c3a x(x^2 - 3y^2).
constexpr float kC0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kC1 = 0.4886025119029199f;    // sqrt(3 / (4 pi))
constexpr float kC2a = 1.0925484305920792f;   // sqrt(15 / (4 pi))
constexpr float kC2b = 0.31539156525252005f;  // sqrt(5 / (16 pi))
constexpr float kC2c = 0.5462742152960396f;   // sqrt(15 / (16 pi))
constexpr float kC3a = 0.5900435899266435f;   // sqrt(35 / (32 pi))
constexpr float kC3b = 2.890611442640554f;    // sqrt(105 / (4 pi))
constexpr float kC3c = 0.4570457994644658f;   // sqrt(21 / (32 pi))
constexpr float kC3d = 0.3731763325901154f;   // sqrt(7 / (16 pi))
constexpr float kC3e = 1.445305721320277f;    // sqrt(105 / (16 pi))

__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y)
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = kC0;
    Y[1] = -(kC1 * y);
    Y[2] = kC1 * z;
    Y[3] = -(kC1 * x);
    Y[4] = kC2a * (x * y);
    Y[5] = -(kC2a * (y * z));
    Y[6] = kC2b * ((2.0f * zz - xx) - yy);
    Y[7] = -(kC2a * (x * z));
    Y[8] = kC2c * (xx - yy);
    Y[9] = -(kC3a * (y * (3.0f * xx - yy)));
    Y[10] = kC3b * ((x * y) * z);
    Y[11] = -(kC3c * (y * ((4.0f * zz - xx) - yy)));
    Y[12] = kC3d * (z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
    Y[13] = -(kC3c * (x * ((4.0f * zz - xx) - yy)));
    Y[14] = kC3e * (z * (xx - yy));
    Y[15] = -(kC3a * (x * (xx - 3.0f * yy)));
}

// A pointer every active lane holds the same value of, moved to scalar registers.
__device__ __forceinline__ const float* uniform_ptr(const float* p)
{
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const float*>(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float ld(const float* plane, uint32_t off) { return ld_plane(plane, off); }

__device__ __forceinline__ int level_index(const LevelsArg& lv, uint32_t g)
{
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && g >= lv.lv[j].base) l = j;
    return l;
}

constexpr int kQueue = 128;   // per-wave colour queue: < 64 left over + one chunk of 64
constexpr int kQRows = 12;    // per queued Gaussian: view direction (3), then its record's geometry (9)

// A float4 pointer every active lane holds the same value of, in scalar registers.
__device__ __forceinline__ const float4* uniform_ptr4(const float4* p)
{
    return reinterpret_cast<const float4*>(uniform_ptr(reinterpret_cast<const float*>(p)));
}

// Colour of up to 64 queued Gaussians, one per lane (lanes >= cnt idle):
// degree-3 real SH at the view direction, + 0.5, clamped at 0; each lane
// then writes its Gaussian's whole record, the queued geometry with the
// colour.  kPacked: the coefficients come from the level's packed copy (one
// contiguous run per Gaussian) instead of its planes.
template <bool kPacked>
__device__ __forceinline__ void colour_batch(const LevelsArg& lv, const LevelDev* s_lv, const uint32_t* qa,
                                             const uint32_t* qg,
                                             const float (*qd)[kQueue], uint32_t cnt, float4* __restrict__ proj)
{
    const uint32_t lane = threadIdx.x & 63;
    const bool mine = lane < cnt;
    const uint32_t a = mine ? qa[lane] : 0u;
    const uint32_t g = mine ? qg[lane] : 0u;
    const float dx = mine ? qd[0][lane] : 0.0f, dy = mine ? qd[1][lane] : 0.0f, dz = mine ? qd[2][lane] : 0.0f;
    const int lvl = level_index(lv, g);
    bool todo = mine;
    while (true) {
        const unsigned long long pend = __ballot(todo);
        if (pend == 0ull) break;
        const int l0 = __builtin_amdgcn_readlane(lvl, __ffsll((long long)pend) - 1);
        if (todo && lvl == l0) {
            todo = false;
            const LevelDev& Lv = s_lv[l0];
            const int sh_degree = __builtin_amdgcn_readfirstlane(Lv.sh_degree);
            const int nb = (sh_degree + 1) * (sh_degree + 1);
            float coef[kMaxSh][3];
            if constexpr (kPacked) {
                // the Gaussian's run of stride4 words; words past it are never read
                const PackDev& P = lv.pk[l0];
                const uint32_t stride4 = __builtin_amdgcn_readfirstlane(P.sh_stride4);
                const float4* __restrict__ h =
                    uniform_ptr4(P.psh) + (size_t)stride4 * (g - __builtin_amdgcn_readfirstlane(Lv.base));
                float c[4 * kMaxSh * 3 / 4];
#pragma unroll
                for (int j = 0; j < kMaxSh * 3 / 4; j++) {
                    const float4 w = (uint32_t)j < stride4 ? h[j] : make_float4(0.f, 0.f, 0.f, 0.f);
                    c[4 * j] = w.x;
                    c[4 * j + 1] = w.y;
                    c[4 * j + 2] = w.z;
                    c[4 * j + 3] = w.w;
                }
#pragma unroll
                for (int k = 0; k < kMaxSh; k++)
#pragma unroll
                    for (int ch = 0; ch < 3; ch++) coef[k][ch] = k < nb ? c[3 * k + ch] : 0.0f;
            } else {
                const float* __restrict__ shp = uniform_ptr(Lv.sh);
                const size_t n = __builtin_amdgcn_readfirstlane(Lv.n);
                const uint32_t off = (g - __builtin_amdgcn_readfirstlane(Lv.base)) * 4u;
                // all (d+1)^2 x 3 coefficients are loaded before the first use; planes past
                // the level's degree are clamped in bounds and contribute an exact zero
#pragma unroll
                for (int k = 0; k < kMaxSh; k++)
#pragma unroll
                    for (int ch = 0; ch < 3; ch++)
                        coef[k][ch] = ld(shp + (size_t)((k < nb ? k : nb - 1) * 3 + ch) * n, off);
            }
            float Y[kMaxSh];
            sh_basis(dx, dy, dz, Y);
            float rgb[3];
#pragma unroll
            for (int ch = 0; ch < 3; ch++) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < kMaxSh; k++) acc = acc + (k < nb ? coef[k][ch] : 0.0f) * Y[k];
                acc = acc + 0.5f;
                rgb[ch] = acc > 0.0f ? acc : 0.0f;
            }
            // the whole record at once: the geometry the projection queued, then the colour
            const uint32_t k = lane;
            proj[3 * (size_t)a] = make_float4(qd[3][k], qd[4][k], qd[5][k], qd[6][k]);
            proj[3 * (size_t)a + 1] = make_float4(qd[7][k], qd[8][k], qd[9][k], rgb[0]);
            proj[3 * (size_t)a + 2] = make_float4(rgb[1], rgb[2], qd[10][k], qd[11][k]);
        }
    }
}

// kPacked: scale, rotation, opacity and SH come from the levels' packed copy.
template <bool kPacked>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_project(LevelsArg lv, const uint32_t* __restrict__ ids,
                                                 const float* __restrict__ wsel, const uint32_t* __restrict__ count,
                                                 uint32_t cap, const FrameParams* __restrict__ fp, FrameInfo* info,
                                                 float4* __restrict__ proj, float* __restrict__ depth,
                                                 uint2* __restrict__ rect, uint32_t* __restrict__ vtiles,
                                                 uint32_t* __restrict__ chunk_sum, uint32_t* __restrict__ chunk_vis)
{
    __shared__ uint32_t s_cnt[2][4];
    __shared__ uint32_t s_qa[4][kQueue], s_qg[4][kQueue];
    __shared__ float s_qd[4][kQRows][kQueue];
    // the level table in LDS: a level picked at run time is then an LDS read,
    // not a memory round trip on every chunk and colour batch
    __shared__ LevelDev s_lv[LODGE_MAX_LEVELS];
    if (threadIdx.x < LODGE_MAX_LEVELS) s_lv[threadIdx.x] = lv.lv[threadIdx.x];
    __syncthreads();
    const uint32_t n_act = min(*count, cap);
    const lodge_camera& cam = fp->cam;
    const float s2d = fp->s2d;
    const int compensate = fp->compensate;
    const int32_t TX = fp->TX, TY = fp->TY;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t* const qa = s_qa[wave];
    uint32_t* const qg = s_qg[wave];
    float (*const qd)[kQueue] = s_qd[wave];
    uint32_t n_front = 0, n_vis = 0;
    uint32_t qn = 0;   // wave-uniform queue length

    const uint32_t nchunks = (n_act + kProjChunk - 1) / kProjChunk;
    const uint32_t waves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t c = blockIdx.x * (blockDim.x >> 6) + wave; c < nchunks; c += waves) {
        const uint32_t a = c * kProjChunk + lane;
        bool visible = false, front = false;
        uint32_t ntiles = 0;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        float dep = 0.0f, d0n = 0.0f, d1n = 0.0f, d2n = 0.0f;
        int32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0;
        const uint32_t g = a < n_act ? __builtin_nontemporal_load(ids + a) : 0u;
        const int lvl = level_index(lv, g);
        bool todo = a < n_act;
        // one pass per level present in the wave (almost always one): the
        // level's fields are then wave-uniform and live in scalar registers
        while (true) {
          const unsigned long long pend = __ballot(todo);
          if (pend == 0ull) break;
          const int l0 = __builtin_amdgcn_readlane(lvl, __ffsll((long long)pend) - 1);
          if (todo && lvl == l0) {
            todo = false;
            const LevelDev& Lv = s_lv[l0];
            const float* __restrict__ mean = uniform_ptr(Lv.mean);
            const float* __restrict__ scale = uniform_ptr(Lv.scale);
            const float* __restrict__ quat = uniform_ptr(Lv.quat);
            const float* __restrict__ opac = uniform_ptr(Lv.opacity);
            const size_t n = __builtin_amdgcn_readfirstlane(Lv.n);
            const float var = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(Lv.var)));
            // byte offset inside a plane (levels hold fewer than 2^30 Gaussians)
            const uint32_t off = (g - __builtin_amdgcn_readfirstlane(Lv.base)) * 4u;
            const float mx = ld(mean, off), my = ld(mean + n, off), mz = ld(mean + 2 * n, off);
            const float* W = cam.R;
            const float tx = ((W[0] * mx + W[1] * my) + W[2] * mz) + cam.t[0];
            const float ty = ((W[3] * mx + W[4] * my) + W[5] * mz) + cam.t[1];
            const float tz = ((W[6] * mx + W[7] * my) + W[8] * mz) + cam.t[2];
            if (tz > cam.znear) {
                front = true;
                float s0, s1, s2, qw, qx, qy, qz, op_p;
                if constexpr (kPacked) {
                    const float4* __restrict__ pg =
                        uniform_ptr4(lv.pk[l0].pgeo) + 2 * (size_t)(g - __builtin_amdgcn_readfirstlane(Lv.base));
                    const float4 ga = pg[0], gb = pg[1];
                    s0 = ga.x; s1 = ga.y; s2 = ga.z; op_p = ga.w;
                    qw = gb.x; qx = gb.y; qy = gb.z; qz = gb.w;
                } else {
                    s0 = ld(scale, off); s1 = ld(scale + n, off); s2 = ld(scale + 2 * n, off);
                    qw = ld(quat, off); qx = ld(quat + n, off); qy = ld(quat + 2 * n, off); qz = ld(quat + 3 * n, off);
                    op_p = 0.0f;
                }
                // rotation of the quaternion (w, x, y, z) as given
                const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
                const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
                const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
                const float R[9] = {1.0f - 2.0f * (yy + zz), 2.0f * (xy - wz),        2.0f * (xz + wy),
                                    2.0f * (xy + wz),        1.0f - 2.0f * (xx + zz), 2.0f * (yz - wx),
                                    2.0f * (xz - wy),        2.0f * (yz + wx),        1.0f - 2.0f * (xx + yy)};
                // Eq. 3: Sigma + var I, and sqrt(|Sigma| / |Sigma + var I|)
                const float v0 = s0 * s0 + var, v1 = s1 * s1 + var, v2 = s2 * s2 + var;
                float S[9];
#pragma unroll
                for (int p = 0; p < 3; p++)
#pragma unroll
                    for (int q = p; q < 3; q++) {
                        const float e = ((R[3 * p] * v0) * R[3 * q] + (R[3 * p + 1] * v1) * R[3 * q + 1])
                                        + (R[3 * p + 2] * v2) * R[3 * q + 2];
                        S[3 * p + q] = e;
                        S[3 * q + p] = e;
                    }
                const float comp3 = sqrtf(((s0 * s0 / v0) * (s1 * s1 / v1)) * (s2 * s2 / v2));
                // perspective Jacobian at the clamped mean
                const float ix = tx / tz, iy = ty / tz;
                const float u = cam.fx * ix + cam.cx;
                const float v = cam.fy * iy + cam.cy;
                float rx = ix, ry = iy;
                if (rx < -cam.lim_x) rx = -cam.lim_x;
                if (rx > cam.lim_x) rx = cam.lim_x;
                if (ry < -cam.lim_y) ry = -cam.lim_y;
                if (ry > cam.lim_y) ry = cam.lim_y;
                const float J00 = cam.fx / tz, J02 = -((cam.fx * rx) / tz);
                const float J11 = cam.fy / tz, J12 = -((cam.fy * ry) / tz);
                float M[6];
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    M[j] = J00 * W[j] + J02 * W[6 + j];
                    M[3 + j] = J11 * W[3 + j] + J12 * W[6 + j];
                }
                float T[6];
#pragma unroll
                for (int r = 0; r < 2; r++)
#pragma unroll
                    for (int j = 0; j < 3; j++)
                        T[3 * r + j] = (M[3 * r] * S[j] + M[3 * r + 1] * S[3 + j]) + M[3 * r + 2] * S[6 + j];
                const float a0 = (T[0] * M[0] + T[1] * M[1]) + T[2] * M[2];
                const float b = (T[0] * M[3] + T[1] * M[4]) + T[2] * M[5];
                const float c0 = (T[3] * M[3] + T[4] * M[4]) + T[5] * M[5];
                // 2-D filter
                const float aa = a0 + s2d, cc = c0 + s2d;
                const float det0 = a0 * c0 - b * b;
                const float det = aa * cc - b * b;
                if (det > 0.0f) {
                    const float comp2 = compensate ? sqrtf((det0 > 0.0f ? det0 : 0.0f) / det) : 1.0f;
                    const float A = cc / det, B = -(b / det), C = aa / det;
                    const float mid = 0.5f * (aa + cc);
                    const float disc = mid * mid - det;
                    const float lam = mid + sqrtf(disc > 0.0f ? disc : 0.0f);
                    const float rad = ceilf(3.0f * sqrtf(lam));
                    float fx0 = floorf((u - rad) / 16.0f), fx1 = floorf((u + rad) / 16.0f) + 1.0f;
                    float fy0 = floorf((v - rad) / 16.0f), fy1 = floorf((v + rad) / 16.0f) + 1.0f;
                    const float hx = (float)(TX + 1), hy = (float)(TY + 1);
                    fx0 = fx0 < -1.0f ? -1.0f : (fx0 > hx ? hx : fx0);
                    fx1 = fx1 < -1.0f ? -1.0f : (fx1 > hx ? hx : fx1);
                    fy0 = fy0 < -1.0f ? -1.0f : (fy0 > hy ? hy : fy0);
                    fy1 = fy1 < -1.0f ? -1.0f : (fy1 > hy ? hy : fy1);
                    x0 = max((int32_t)fx0, 0);
                    y0 = max((int32_t)fy0, 0);
                    x1 = min((int32_t)fx1, TX);
                    y1 = min((int32_t)fy1, TY);
                    if (x0 < x1 && y0 < y1) {
                        visible = true;
                        ntiles = (uint32_t)((x1 - x0) * (y1 - y0));
                        // view direction camera -> mean, for the colour pass
                        const float d0 = mx - cam.pos[0], d1 = my - cam.pos[1], d2 = mz - cam.pos[2];
                        const float dn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
                        d0n = d0 / dn;
                        d1n = d1 / dn;
                        d2n = d2 / dn;
                        float op;
                        if constexpr (kPacked) op = op_p;
                        else op = ld(opac, off);
                        const float o_eff = ((op * __builtin_nontemporal_load(wsel + a)) * comp3) * comp2;
                        // compositing aids: below power thr alpha cannot reach 1/255 (margin 1e-3);
                        // (ex, ey) half-extents of the ellipse where it can: d^T conic d <= -2 thr
                        const float thr = o_eff > 0.0f ? -logf(255.0f * o_eff) - 1e-3f : INFINITY;
                        const float rho = -2.0f * thr;
                        const float ex = rho > 0.0f ? sqrtf(rho * aa) : -1.0f;
                        const float ey = rho > 0.0f ? sqrtf(rho * cc) : -1.0f;
                        // the record in the form the compositor reads it: the conic
                        // pre-scaled to the power's coefficients (exact scalings)
                        r0 = make_float4(u, v, -0.5f * A, -B);
                        r1 = make_float4(-0.5f * C, o_eff, thr, 0.0f);
                        r2 = make_float4(0.0f, 0.0f, ex, ey);
                        dep = tz;
                    }
                }
            }
          }
        }
        if (a < n_act) {
            depth[a] = dep;
            // culled: the canonical empty rect (the clamped bounds may be -1 and must not be packed)
            rect[a] = visible ? make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16))
                              : make_uint2(0u, 0u);
            vtiles[a] = ntiles;
            n_front += front ? 1u : 0u;
            n_vis += visible ? 1u : 0u;
        }
        // the chunk's tile total and its actives with a tile: first level
        // of the instance scan and of their compaction
        uint32_t csum = ntiles;
        for (int o = 32; o > 0; o >>= 1) csum += __shfl_xor(csum, o);
        const uint32_t cvis = (uint32_t)__popcll(__ballot(ntiles > 0u));
        if (lane == 0) {
            chunk_sum[c] = csum;
            chunk_vis[c] = cvis;
        }
        // queue the visible ones for colour
        const unsigned long long m = __ballot(visible);
        if (visible) {
            const uint32_t p = qn + (uint32_t)__popcll(m & lt);
            qa[p] = a;
            qg[p] = g;
            qd[0][p] = d0n;
            qd[1][p] = d1n;
            qd[2][p] = d2n;
            qd[3][p] = r0.x;
            qd[4][p] = r0.y;
            qd[5][p] = r0.z;
            qd[6][p] = r0.w;
            qd[7][p] = r1.x;
            qd[8][p] = r1.y;
            qd[9][p] = r1.z;
            qd[10][p] = r2.z;
            qd[11][p] = r2.w;
        }
        qn += (uint32_t)__popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (qn >= 64) {
            colour_batch<kPacked>(lv, s_lv, qa, qg, qd, 64, proj);
            // move the left-over entries to the front of the queue
            const uint32_t rem = qn - 64;
            uint32_t ta = 0, tg = 0;
            float tq[kQRows];
#pragma unroll
            for (int q = 0; q < kQRows; q++) tq[q] = 0.0f;
            if (lane < rem) {
                ta = qa[64 + lane];
                tg = qg[64 + lane];
#pragma unroll
                for (int q = 0; q < kQRows; q++) tq[q] = qd[q][64 + lane];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane < rem) {
                qa[lane] = ta;
                qg[lane] = tg;
#pragma unroll
                for (int q = 0; q < kQRows; q++) qd[q][lane] = tq[q];
            }
            qn = rem;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    if (qn > 0) colour_batch<kPacked>(lv, s_lv, qa, qg, qd, qn, proj);
    // counters: wave sums, block sum, one atomic per block
    for (int o = 32; o > 0; o >>= 1) {
        n_front += __shfl_xor(n_front, o);
        n_vis += __shfl_xor(n_vis, o);
    }
    if (lane == 0) { s_cnt[0][wave] = n_front; s_cnt[1][wave] = n_vis; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t f = s_cnt[0][0] + s_cnt[0][1] + s_cnt[0][2] + s_cnt[0][3];
        const uint32_t v = s_cnt[1][0] + s_cnt[1][1] + s_cnt[1][2] + s_cnt[1][3];
        if (f) atomicAdd(&info->n_front, f);
        if (v) atomicAdd(&info->n_visible, v);
    }
}

}  // namespace

hipError_t launch_project(const LevelsArg& lv, const lodge_selection& sel, const Views& v, hipStream_t st)
{
    // persistent waves: exactly as many blocks as the device holds at once, so
    // every wave's queue spans many chunks and no second partial round is left
    static thread_local int dev_cached = -1;
    static thread_local uint32_t resident[2] = {0, 0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != dev_cached) {
        int per_cu[2] = {0, 0}, cus = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[0], k_project<false>, 256, 0)) != hipSuccess)
            return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[1], k_project<true>, 256, 0)) != hipSuccess)
            return e;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        resident[0] = (uint32_t)std::max(1, per_cu[0] * cus);
        resident[1] = (uint32_t)std::max(1, per_cu[1] * cus);
        dev_cached = dev;
    }
    uint32_t blocks = (v.max_active + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > resident[lv.packed ? 1 : 0]) blocks = resident[lv.packed ? 1 : 0];
    if (lv.packed)
        k_project<true><<<blocks, 256, 0, st>>>(lv, sel.ids, sel.w, sel.count, sel.cap, v.params, v.info, v.proj,
                                                v.depth, v.rect, v.vtiles, v.chunk_sum, v.chunk_vis);
    else
        k_project<false><<<blocks, 256, 0, st>>>(lv, sel.ids, sel.w, sel.count, sel.cap, v.params, v.info, v.proj,
                                                 v.depth, v.rect, v.vtiles, v.chunk_sum, v.chunk_vis);
    return hipGetLastError();
}

}  // namespace lodge
