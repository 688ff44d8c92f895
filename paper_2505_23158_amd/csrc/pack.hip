// The packed copy of a scene's levels (lodge_scene_pack): a layout change
// only, none of the method's arithmetic.  The projection reads, for every
// Gaussian in front of the camera, its scale, rotation and opacity, and for
// every visible one its 3 (d+1)^2 SH coefficients.  In the caller's
// structure of arrays these are 8 + 48 separate planes, so each Gaussian's
// reads land in 56 different regions of memory; packed, they are two
// 16-byte words and one contiguous run of 16-byte words per Gaussian.
// The means stay in their planes: the selection streams them, and the
// projection needs them before it knows whether the rest is needed.
#include <algorithm>

#include "lodge_internal.hpp"

namespace lodge {

namespace {

__global__ __launch_bounds__(256) void k_pack(LevelDev L, PackDev P)
{
    const uint32_t n = L.n;
    const int nb = (L.sh_degree + 1) * (L.sh_degree + 1);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float4* const g = const_cast<float4*>(P.pgeo) + 2 * (size_t)i;
        g[0] = make_float4(L.scale[i], L.scale[n + i], L.scale[2 * (size_t)n + i], L.opacity[i]);
        g[1] = make_float4(L.quat[i], L.quat[n + i], L.quat[2 * (size_t)n + i], L.quat[3 * (size_t)n + i]);
        float4* const h = const_cast<float4*>(P.psh) + (size_t)P.sh_stride4 * i;
        for (uint32_t j = 0; j < P.sh_stride4; j++) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int c = 4 * (int)j + e;   // coefficient index k * 3 + channel
                v[e] = c < 3 * nb ? L.sh[(size_t)c * n + i] : 0.0f;
            }
            h[j] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

}  // namespace

hipError_t launch_pack(const LevelsArg& lv, hipStream_t st)
{
    for (int l = 0; l < lv.L; l++) {
        const LevelDev& L = lv.lv[l];
        if (L.n == 0) continue;
        const uint32_t blocks = std::min<uint32_t>((L.n + 255) / 256, 8192);
        k_pack<<<blocks, 256, 0, st>>>(L, lv.pk[l]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lodge
