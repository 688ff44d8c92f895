// 3DGS parameter activation and its adjoint, for the differentiable form:
// scale = exp(log_scale), quat = q / |q|, opacity = sigmoid(logit).
// Coalesced plane-wise passes, one thread per Gaussian.
#include "lodge_internal.hpp"

namespace lodge {

namespace {

__global__ void k_activate(int64_t n, const float* __restrict__ ls, const float* __restrict__ qr,
                           const float* __restrict__ ol, float* __restrict__ s, float* __restrict__ q,
                           float* __restrict__ o)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int j = 0; j < 3; j++) s[j * n + i] = expf(ls[j * n + i]);
        const float w = qr[i], x = qr[n + i], y = qr[2 * n + i], z = qr[3 * n + i];
        const float nrm = sqrtf(((w * w + x * x) + y * y) + z * z);
        const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
        q[i] = w * inv;
        q[n + i] = x * inv;
        q[2 * n + i] = y * inv;
        q[3 * n + i] = z * inv;
        o[i] = 1.0f / (1.0f + expf(-ol[i]));
    }
}

__global__ void k_activate_bwd(int64_t n, const float* __restrict__ qr, const float* __restrict__ s,
                               const float* __restrict__ o, const float* __restrict__ gs,
                               const float* __restrict__ gq, const float* __restrict__ go, float* __restrict__ gls,
                               float* __restrict__ gqr, float* __restrict__ gol)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (gs && gls)
            for (int j = 0; j < 3; j++) gls[j * n + i] += gs[j * n + i] * s[j * n + i];
        if (gq && gqr) {
            const float r[4] = {qr[i], qr[n + i], qr[2 * n + i], qr[3 * n + i]};
            const float nrm = sqrtf(((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]) + r[3] * r[3]);
            if (nrm > 0.0f) {
                const float inv = 1.0f / nrm;
                const float u[4] = {r[0] * inv, r[1] * inv, r[2] * inv, r[3] * inv};
                const float g[4] = {gq[i], gq[n + i], gq[2 * n + i], gq[3 * n + i]};
                const float dot = ((u[0] * g[0] + u[1] * g[1]) + u[2] * g[2]) + u[3] * g[3];
                for (int j = 0; j < 4; j++) gqr[j * n + i] += (g[j] - u[j] * dot) * inv;
            }
        }
        if (go && gol) gol[i] += go[i] * o[i] * (1.0f - o[i]);
    }
}

}  // namespace

hipError_t launch_activate(int64_t n, const float* ls, const float* qr, const float* ol, float* s, float* q, float* o,
                           hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
    k_activate<<<(uint32_t)blocks, 256, 0, st>>>(n, ls, qr, ol, s, q, o);
    return hipGetLastError();
}

hipError_t launch_activate_backward(int64_t n, const float* qr, const float* s, const float* o, const float* gs,
                                    const float* gq, const float* go, float* gls, float* gqr, float* gol,
                                    hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
    k_activate_bwd<<<(uint32_t)blocks, 256, 0, st>>>(n, qr, s, o, gs, gq, go, gls, gqr, gol);
    return hipGetLastError();
}

}  // namespace lodge
