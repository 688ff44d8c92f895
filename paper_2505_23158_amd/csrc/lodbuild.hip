// Kernels of the LOD-level construction loop (LODGE supplementary "LOD
// structure optimization steps"; Sec. 3 "Building LOD representation"):
// the per-level fine-tuning's loss gradient and optimiser step, and the
// compaction of a level after importance pruning.
//
//   k_l1_grad     dL/dimage of the mean L1 loss: scale * sign(image - target)
//                 (sign(0) = 0), and optionally the loss itself (block sums,
//                 one atomic per block).
//   k_adam        one Adam step on a parameter array: m = b1 m + (1 - b1) g,
//                 v = b2 v + (1 - b2) g^2, p -= lr (m / c1) / (sqrt(v / c2) + eps)
//                 with the bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
//                 given by the host.
//   k_keep_count / k_keep_scan / k_keep_emit
//                 indices i (ascending) of the items with score[i] >= thr:
//                 per-block counts, one-block scan, per-block ballot
//                 compaction at the block's offset.
//   k_gather      out[p][j] = in[p][idx[j]] for P planes (a level's
//                 parameters and optimiser moments after pruning).
//   k_ssim_rows / k_blur / k_ssim_map / k_ssim_grad
//                 the D-SSIM term of the loss and its gradient: separable
//                 window filtering of x, y, x^2, y^2, x y, the SSIM map and
//                 g times its derivatives w.r.t. the filtered statistics,
//                 the same filtering of those (the window is symmetric, so
//                 it is its own adjoint), and the gradient
//                 -(w * d_mu + 2 x (w * d_xx) + y (w * d_xy)).
//
// Built with -ffp-contract=off like the rest of the library.
#include <algorithm>
#include <cmath>

#include "lodge_internal.hpp"

namespace lodge {

namespace {

constexpr int kKeepBlock = 256;
constexpr int kKeepItems = 16;
constexpr int kKeepTile = kKeepBlock * kKeepItems;

__global__ __launch_bounds__(256) void k_l1_grad(uint64_t n, const float* __restrict__ image,
                                                 const float* __restrict__ target, float scale,
                                                 float* __restrict__ grad, float* __restrict__ loss)
{
    __shared__ float s_part[4];
    float acc = 0.0f;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float d = image[i] - target[i];
        grad[i] = d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
        acc += fabsf(d);
    }
    if (!loss) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) * scale);
}

__global__ __launch_bounds__(256) void k_adam(uint64_t n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
        m[i] = mi;
        v[i] = vi;
        p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ __launch_bounds__(kKeepBlock) void k_keep_count(uint32_t n, const float* __restrict__ score, float thr,
                                                           uint32_t* __restrict__ cnt)
{
    __shared__ uint32_t s_w[kKeepBlock / 64];
    const uint32_t i0 = blockIdx.x * (uint32_t)kKeepTile;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kKeepItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kKeepBlock + threadIdx.x;
        c += (i < n && score[i] >= thr) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

// one block of 1024 threads: exclusive scan of nb counts in place, total to *total
__global__ __launch_bounds__(1024) void k_keep_scan(uint32_t nb, uint32_t* __restrict__ cnt, uint32_t* __restrict__ total)
{
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + tid;
        const uint32_t x = i < nb ? cnt[i] : 0u;
        uint32_t inc = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o);
            if ((int)lane >= o) inc += u;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        uint32_t before = 0, sum = 0;
        for (uint32_t k = 0; k < 16; k++) {
            before += k < wave ? s_w[k] : 0u;
            sum += s_w[k];
        }
        const uint32_t carry = s_carry;
        if (i < nb) cnt[i] = carry + before + inc - x;
        __syncthreads();
        if (tid == 0) s_carry = carry + sum;
        __syncthreads();
    }
    if (tid == 0) *total = s_carry;
}

__global__ __launch_bounds__(kKeepBlock) void k_keep_emit(uint32_t n, const float* __restrict__ score, float thr,
                                                          const uint32_t* __restrict__ off, uint32_t* __restrict__ idx)
{
    __shared__ uint32_t s_c[kKeepItems * 4];
    const uint32_t i0 = blockIdx.x * (uint32_t)kKeepTile;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool k[kKeepItems];
#pragma unroll
    for (int r = 0; r < kKeepItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kKeepBlock + threadIdx.x;
        k[r] = i < n && score[i] >= thr;
        const unsigned long long m = __ballot(k[r]);
        if (lane == 0) s_c[r * 4 + wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t x = s_c[lane];   // kKeepItems * 4 == 64 entries
        uint32_t inc = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o);
            if ((int)lane >= o) inc += u;
        }
        s_c[lane] = inc - x;
    }
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t base = off[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kKeepItems; r++) {
        const unsigned long long m = __ballot(k[r]);
        if (k[r]) idx[base + s_c[r * 4 + wave] + (uint32_t)__popcll(m & lt)] = i0 + (uint32_t)r * kKeepBlock + threadIdx.x;
    }
}
static_assert(kKeepItems * 4 == 64, "one scan wave");

__global__ __launch_bounds__(256) void k_gather(uint32_t planes, uint32_t n_in, uint32_t n_out,
                                                const float* __restrict__ in, const uint32_t* __restrict__ idx,
                                                const uint32_t* __restrict__ count, float* __restrict__ out)
{
    const uint32_t m = min(*count, n_out);
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const uint32_t s = idx[j];
        if (s >= n_in) continue;
        for (uint32_t p = 0; p < planes; p++) out[(size_t)p * n_out + j] = in[(size_t)p * n_in + s];
    }
}

// ---- the D-SSIM term: SSIM (Wang et al.) with an 11 x 11 Gaussian window of
// sigma 1.5, separable, zero padding outside the image ('same' size).
constexpr int kWin = 11;
constexpr float kC1 = 0.0001f;   // (0.01)^2
constexpr float kC2 = 0.0009f;   // (0.03)^2
struct Window {
    float w[kWin];
};

// Horizontal pass over the five local-statistics inputs of each pixel:
// x, y, x^2, y^2, x y (maps [5][C][H][W]).
__global__ __launch_bounds__(256) void k_ssim_rows(uint32_t C, uint32_t H, uint32_t W, const float* __restrict__ x,
                                                   const float* __restrict__ y, float* __restrict__ out, Window win)
{
    const uint64_t N = (uint64_t)C * H * W;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)(p % W);
        float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < kWin; k++) {
            const int jj = (int)j + k - kWin / 2;
            if (jj < 0 || jj >= (int)W) continue;
            const uint64_t q = p - j + (uint32_t)jj;
            const float a = x[q], b = y[q], w = win.w[k];
            s[0] += w * a;
            s[1] += w * b;
            s[2] += w * (a * a);
            s[3] += w * (b * b);
            s[4] += w * (a * b);
        }
#pragma unroll
        for (int m = 0; m < 5; m++) out[(uint64_t)m * N + p] = s[m];
    }
}

// Generic separable pass over P maps [P][C][H][W]: along rows (vertical = 0)
// or along columns (vertical = 1).
__global__ __launch_bounds__(256) void k_blur(uint32_t P, uint32_t C, uint32_t H, uint32_t W, int32_t vertical,
                                              const float* __restrict__ in, float* __restrict__ out, Window win)
{
    const uint64_t N = (uint64_t)C * H * W;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (uint64_t)P * N;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = t % N;
        const uint32_t j = (uint32_t)(p % W), i = (uint32_t)((p / W) % H);
        const uint32_t pos = vertical ? i : j, len = vertical ? H : W;
        const uint64_t step = vertical ? W : 1;
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; k++) {
            const int q = (int)pos + k - kWin / 2;
            if (q < 0 || q >= (int)len) continue;
            s += win.w[k] * in[t - (uint64_t)pos * step + (uint64_t)q * step];
        }
        out[t] = s;
    }
}

// Per pixel, from the filtered statistics (mu_x, mu_y, E_xx, E_yy, E_xy):
// the SSIM value m and g times its derivatives w.r.t. mu_x, E_xx, E_xy.
__global__ __launch_bounds__(256) void k_ssim_map(uint64_t N, const float* __restrict__ st, float g,
                                                  float* __restrict__ d, float* __restrict__ loss, float weight)
{
    __shared__ float s_part[4];
    float acc = 0.0f;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x) {
        const float mx = st[p], my = st[N + p], exx = st[2 * N + p], eyy = st[3 * N + p], exy = st[4 * N + p];
        const float a1 = 2.0f * mx * my + kC1;
        const float a2 = 2.0f * (exy - mx * my) + kC2;
        const float b1 = mx * mx + my * my + kC1;
        const float b2 = (exx - mx * mx) + (eyy - my * my) + kC2;
        const float den = b1 * b2;
        const float m = (a1 * a2) / den;
        d[p] = g * ((2.0f * my * a2 - 2.0f * my * a1) / den - m * (2.0f * mx) / b1 + m * (2.0f * mx) / b2);
        d[N + p] = g * (-m / b2);
        d[2 * N + p] = g * (2.0f * a1 / den);
        acc += m;
    }
    if (!loss) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    // weight (1 - mean m): block 0 also adds the constant term
    if (threadIdx.x == 0)
        atomicAdd(loss, (blockIdx.x == 0 ? weight : 0.0f) - weight * ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) * g);
}

// grad += weight * -(w * d0 + 2 x (w * d1) + y (w * d2))  (bd: the filtered derivative maps)
__global__ __launch_bounds__(256) void k_ssim_grad(uint64_t N, const float* __restrict__ x,
                                                   const float* __restrict__ y, const float* __restrict__ bd,
                                                   float weight, float* __restrict__ grad)
{
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x)
        grad[p] = grad[p] - weight * ((bd[p] + 2.0f * x[p] * bd[N + p]) + y[p] * bd[2 * N + p]);
}

uint32_t grid_for(uint64_t n) { return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(1, (n + 255) / 256), 8192); }

}  // namespace

}  // namespace lodge

using namespace lodge;

extern "C" {

lodge_status lodge_l1_grad(int64_t n, const float* image, const float* target, float scale, float* grad, float* loss,
                           void* stream)
{
    if (n < 0) return fail(LODGE_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return LODGE_OK;
    if (!image || !target || !grad) return fail(LODGE_ERR_INVALID_ARG, "l1_grad: NULL buffer");
    if (!std::isfinite(scale)) return fail(LODGE_ERR_INVALID_ARG, "l1_grad: scale must be finite");
    k_l1_grad<<<grid_for((uint64_t)n), 256, 0, static_cast<hipStream_t>(stream)>>>((uint64_t)n, image, target, scale,
                                                                                   grad, loss);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_l1_grad");
}

lodge_status lodge_adam(int64_t n, float* param, const float* grad, float* m, float* v, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* stream)
{
    if (n < 0) return fail(LODGE_ERR_INVALID_ARG, "n < 0");
    if (step < 1) return fail(LODGE_ERR_INVALID_ARG, "adam: step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f) || !std::isfinite(lr))
        return fail(LODGE_ERR_INVALID_ARG, "adam: need 0 <= beta < 1, eps >= 0 and a finite lr");
    if (n == 0) return LODGE_OK;
    if (!param || !grad || !m || !v) return fail(LODGE_ERR_INVALID_ARG, "adam: NULL buffer");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    k_adam<<<grid_for((uint64_t)n), 256, 0, static_cast<hipStream_t>(stream)>>>((uint64_t)n, param, grad, m, v, lr,
                                                                                beta1, beta2, eps, c1, c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_adam");
}

lodge_status lodge_keep_scratch_size(int64_t n, size_t* bytes)
{
    if (n < 0 || n >= (int64_t)1 << 32 || !bytes) return fail(LODGE_ERR_INVALID_ARG, "keep: n out of range or bytes NULL");
    *bytes = 4 * (size_t)(((uint64_t)n + kKeepTile - 1) / kKeepTile + 1);
    return LODGE_OK;
}

lodge_status lodge_keep_indices(int64_t n, const float* score, float threshold, uint32_t* idx, uint32_t* count,
                                void* scratch, size_t scratch_bytes, void* stream)
{
    size_t need = 0;
    lodge_status s = lodge_keep_scratch_size(n, &need);
    if (s != LODGE_OK) return s;
    if (!count || (!scratch && need > 0) || scratch_bytes < need || (n > 0 && (!score || !idx)))
        return fail(LODGE_ERR_INVALID_ARG, "keep: NULL buffer or scratch too small");
    if (!std::isfinite(threshold)) return fail(LODGE_ERR_INVALID_ARG, "keep: threshold must be finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nb = (uint32_t)(((uint64_t)n + kKeepTile - 1) / kKeepTile);
    uint32_t* cnt = static_cast<uint32_t*>(scratch);
    if (nb > 0) k_keep_count<<<nb, kKeepBlock, 0, st>>>((uint32_t)n, score, threshold, cnt);
    k_keep_scan<<<1, 1024, 0, st>>>(nb, cnt, count);
    if (nb > 0) k_keep_emit<<<nb, kKeepBlock, 0, st>>>((uint32_t)n, score, threshold, cnt, idx);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_keep_indices");
}

lodge_status lodge_gather_planes(int32_t planes, int64_t n_in, int64_t n_out, const float* in, const uint32_t* idx,
                                 const uint32_t* count, float* out, void* stream)
{
    if (planes < 0 || n_in < 0 || n_out < 0 || n_in >= (int64_t)1 << 32 || n_out >= (int64_t)1 << 32)
        return fail(LODGE_ERR_INVALID_ARG, "gather: sizes out of range");
    if (planes == 0 || n_out == 0) return LODGE_OK;
    if (!in || !idx || !count || !out) return fail(LODGE_ERR_INVALID_ARG, "gather: NULL buffer");
    k_gather<<<grid_for((uint64_t)n_out), 256, 0, static_cast<hipStream_t>(stream)>>>(
        (uint32_t)planes, (uint32_t)n_in, (uint32_t)n_out, in, idx, count, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_gather_planes");
}

lodge_status lodge_dssim_scratch_size(int32_t width, int32_t height, int32_t channels, size_t* bytes)
{
    if (width <= 0 || height <= 0 || channels <= 0 || !bytes) return fail(LODGE_ERR_INVALID_ARG, "dssim: bad size");
    *bytes = 10 * sizeof(float) * (size_t)width * (size_t)height * (size_t)channels;
    return LODGE_OK;
}

lodge_status lodge_dssim_grad(int32_t width, int32_t height, int32_t channels, const float* image, const float* target,
                              float weight, float* grad, float* loss, void* scratch, size_t scratch_bytes,
                              void* stream)
{
    size_t need = 0;
    lodge_status s = lodge_dssim_scratch_size(width, height, channels, &need);
    if (s != LODGE_OK) return s;
    if (!image || !target || !grad || !scratch || scratch_bytes < need)
        return fail(LODGE_ERR_INVALID_ARG, "dssim: NULL buffer or scratch too small");
    if (!std::isfinite(weight)) return fail(LODGE_ERR_INVALID_ARG, "dssim: weight must be finite");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Window win;
    {
        double w[kWin], sum = 0.0;
        for (int k = 0; k < kWin; k++) {
            const double x = (double)(k - kWin / 2);
            w[k] = std::exp(-(x * x) / (2.0 * 1.5 * 1.5));
            sum += w[k];
        }
        for (int k = 0; k < kWin; k++) win.w[k] = (float)(w[k] / sum);
    }
    const uint32_t C = (uint32_t)channels, H = (uint32_t)height, W = (uint32_t)width;
    const uint64_t N = (uint64_t)C * H * W;
    float* a = static_cast<float*>(scratch);   // 5 maps
    float* b = a + 5 * N;                      // 5 maps
    k_ssim_rows<<<grid_for(N), 256, 0, st>>>(C, H, W, image, target, a, win);
    k_blur<<<grid_for(5 * N), 256, 0, st>>>(5, C, H, W, 1, a, b, win);
    k_ssim_map<<<grid_for(N), 256, 0, st>>>(N, b, (float)(1.0 / (double)N), a, loss, weight);
    k_blur<<<grid_for(3 * N), 256, 0, st>>>(3, C, H, W, 0, a, b, win);
    k_blur<<<grid_for(3 * N), 256, 0, st>>>(3, C, H, W, 1, b, a, win);
    k_ssim_grad<<<grid_for(N), 256, 0, st>>>(N, image, target, a, weight, grad);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LODGE_OK : hip_fail(e, "lodge_dssim_grad");
}

}  // extern "C"
