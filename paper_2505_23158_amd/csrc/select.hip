// Active-set selection (LODGE Sec. 3, Eq. 2 with the per-chunk offset
// thresholds of "Reducing memory with chunk-based rendering", and the
// two-chunk opacity weights of Eq. 4).
//
// k_select_setup  one wave finds the two nearest chunk centres and t, and
//                 turns the switch distances into squared FP32 bounds
//                 (k_zero64 clears the look-back flags before it).
// k_select        one pass over every Gaussian of every level (each block
//                 inside one level, so its parameters and bounds are
//                 uniform): coalesced loads of the three mean planes,
//                 membership on squared FP32 distances, wave ballots + an
//                 LDS scan for the block offsets, and a decoupled look-back
//                 across blocks so the output stays in ascending global id
//                 without a second pass.
//
// Bit-exactness: this file is built with -ffp-contract=off, so each
// +, -, *, / and sqrt below is one IEEE-rounded FP32 operation, evaluated
// in the order written (the order the oracle uses as the definition).
#include "lodge_internal.hpp"

namespace lodge {

namespace {

__device__ __forceinline__ float dist2(float px, float py, float pz, const float* q)
{
    const float dx = px - q[0], dy = py - q[1], dz = pz - q[2];
    return (dx * dx + dy * dy) + dz * dz;
}

// lexicographic (d, k) minimum across the wave
__device__ __forceinline__ void wave_argmin(float& d, int& k)
{
    for (int off = 32; off > 0; off >>= 1) {
        const float od = __shfl_xor(d, off);
        const int ok = __shfl_xor(k, off);
        if (od < d || (od == d && ok < k)) { d = od; k = ok; }
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ void k_zero64(unsigned long long* p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// One wave.  (The chunk table is a by-value kernel argument indexed with
// lane-dependent subscripts, which the compiler stages through private
// memory; keeping this kernel to 64 lanes keeps that copy negligible.)
__global__ __launch_bounds__(64) void k_select_setup(ChunksArg ch, LevelsArg lv, int32_t mode, FrameParams* fp,
                                                     FrameInfo* info)
{
    const int lane = threadIdx.x;
    const float px = fp->cam.pos[0], py = fp->cam.pos[1], pz = fp->cam.pos[2];
    int f = -1, o = -1;
    float t = 1.0f;
    if (mode == LODGE_SELECT_CHUNKED) {
        float d = INFINITY;
        int k = 0x7fffffff;
        for (int c = lane; c < ch.K; c += 64) {
            const float dc = dist2(px, py, pz, ch.c[c]);
            if (dc < d || (dc == d && c < k)) { d = dc; k = c; }
        }
        wave_argmin(d, k);
        f = k;
        if (ch.K > 1) {
            float d2 = INFINITY;
            int k2 = 0x7fffffff;
            for (int c = lane; c < ch.K; c += 64) {
                if (c == f) continue;
                const float dc = dist2(px, py, pz, ch.c[c]);
                if (dc < d2 || (dc == d2 && c < k2)) { d2 = dc; k2 = c; }
            }
            wave_argmin(d2, k2);
            o = k2;
            // Eq. 4: t_bar = ((c - m_o) . (m_f - m_o)) / |m_f - m_o|^2
            const float g0 = ch.c[f][0] - ch.c[o][0], g1 = ch.c[f][1] - ch.c[o][1], g2 = ch.c[f][2] - ch.c[o][2];
            const float e0 = px - ch.c[o][0], e1 = py - ch.c[o][1], e2 = pz - ch.c[o][2];
            const float num = (e0 * g0 + e1 * g1) + e2 * g2;
            const float den = (g0 * g0 + g1 * g1) + g2 * g2;
            float tb = num / den;
            if (ch.band > 0.0f) tb = 0.5f + (tb - 0.5f) * (sqrtf(den) / ch.band);
            t = tb < 0.0f ? 0.0f : tb;
            t = t > 1.0f ? 1.0f : t;
        }
    }
    if (lane != 0) return;
    fp->mode = mode;
    fp->f = f;
    fp->o = o;
    fp->t = t;
    fp->w_o = 1.0f - t;
    const float zero3[3] = {0.0f, 0.0f, 0.0f};
    const float* cf = zero3;
    const float* co = zero3;
    float rf = 0.0f, ro = 0.0f;
    if (mode == LODGE_SELECT_LOD_CAMERA) cf = fp->cam.pos;
    if (mode == LODGE_SELECT_CHUNKED) {
        cf = ch.c[f];
        rf = ch.r[f];
        if (o >= 0) { co = ch.c[o]; ro = ch.r[o]; }
    }
    for (int j = 0; j < 3; j++) { fp->cf[j] = cf[j]; fp->co[j] = co[j]; }
    // squared bounds: lo(0) = 0, lo(l) = (d_l + r)^2, hi(l) = lo(l+1), hi(L-1) = inf
    for (int l = 0; l < lv.L; l++) {
        float s;
        s = (l == 0) ? 0.0f : lv.d[l - 1] + rf;
        fp->lo_f[l] = (l == 0) ? 0.0f : s * s;
        s = (l == lv.L - 1) ? 0.0f : lv.d[l] + rf;
        fp->hi_f[l] = (l == lv.L - 1) ? INFINITY : s * s;
        s = (l == 0) ? 0.0f : lv.d[l - 1] + ro;
        fp->lo_o[l] = (l == 0) ? 0.0f : s * s;
        s = (l == lv.L - 1) ? 0.0f : lv.d[l] + ro;
        fp->hi_o[l] = (l == lv.L - 1) ? INFINITY : s * s;
    }
    info->n_selected = 0;
    info->overflow = 0;
    info->sel_ticket = 0;
    info->f = f;
    info->o = o;
    info->t = t;
}

// Decoupled look-back by one wave: returns the exclusive prefix of `tile`.
// Flag word = status << 32 | value; status 1 = block aggregate, 2 = inclusive.
__device__ uint32_t lookback(unsigned long long* flags, int32_t tile, uint32_t lane)
{
    uint32_t prefix = 0;
    int32_t pred = tile - 1;
    while (true) {
        const int32_t idx = pred - (int32_t)lane;
        unsigned long long v = 2ull << 32;
        if (idx >= 0) v = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t st = (uint32_t)(v >> 32);
        if (__ballot(st == 0u) != 0ull) continue;          // a predecessor has not published yet
        const unsigned long long inc = __ballot(st == 2u);
        uint32_t val = (uint32_t)v;
        if (inc != 0ull) {
            const int first = __ffsll((long long)inc) - 1;
            if ((int)lane > first) val = 0;
            prefix += wave_sum(val);
            break;
        }
        prefix += wave_sum(val);
        pred -= 64;
    }
    return prefix;
}

__global__ __launch_bounds__(kSelBlock) void k_select(LevelsArg lv, const FrameParams* fp, FrameInfo* info,
                                                      unsigned long long* flags, uint32_t ntiles, uint32_t* ids,
                                                      float* w, uint32_t cap, uint32_t* count_out)
{
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_cnt[kSelItems * 4];
    __shared__ uint32_t s_excl;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(&info->sel_ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) return;

    // every block lies inside one level: level parameters and bounds are block-uniform
    int l = 0;
#pragma unroll
    for (int j = 1; j < LODGE_MAX_LEVELS; j++)
        if (j < lv.L && tile >= lv.first_block[j]) l = j;
    const LevelDev& L = lv.lv[l];
    const uint32_t n = L.n;
    const uint32_t i0 = (tile - lv.first_block[l]) * (uint32_t)kSelTile;
    const int32_t mode = fp->mode;
    const bool all = mode == LODGE_SELECT_ALL;
    const bool two = (mode == LODGE_SELECT_CHUNKED) && (fp->o >= 0);
    const float cf[3] = {fp->cf[0], fp->cf[1], fp->cf[2]};
    const float co[3] = {fp->co[0], fp->co[1], fp->co[2]};
    const float lof = fp->lo_f[l], hif = fp->hi_f[l], loo = fp->lo_o[l], hio = fp->hi_o[l];

    // all loads first (48 in flight per thread), then the tests
    float mx[kSelItems], my[kSelItems], mz[kSelItems];
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kSelBlock + tid;
        mx[r] = my[r] = mz[r] = 0.0f;
        if (i < n && !all) {
            mx[r] = L.mean[i];
            my[r] = L.mean[(size_t)n + i];
            mz[r] = L.mean[2 * (size_t)n + i];
        }
    }
    uint32_t bits = 0;   // 2 bits per item: in_f, in_o
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t i = i0 + (uint32_t)r * kSelBlock + tid;
        uint32_t s = 0;
        if (i < n) {
            if (all) {
                s = 1;
            } else {
                const float df = dist2(mx[r], my[r], mz[r], cf);
                if (lof <= df && df < hif) s |= 1u;
                if (two) {
                    const float dq = dist2(mx[r], my[r], mz[r], co);
                    if (loo <= dq && dq < hio) s |= 2u;
                }
            }
        }
        bits |= s << (2 * r);
        const unsigned long long m = __ballot(s != 0u);
        if (lane == 0) s_cnt[r * 4 + wave] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t v = s_cnt[lane];
        uint32_t inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(inc, off);
            if ((int)lane >= off) inc += o;
        }
        const uint32_t block_total = __shfl(inc, 63);
        s_cnt[lane] = inc - v;
        uint32_t prefix = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&flags[0], (2ull << 32) | block_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&flags[tile], (1ull << 32) | block_total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            prefix = lookback(flags, (int32_t)tile, lane);
            if (lane == 0)
                __hip_atomic_store(&flags[tile], (2ull << 32) | (prefix + block_total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_excl = prefix;
            if (tile == ntiles - 1) {
                const uint32_t n = prefix + block_total;
                *count_out = n;
                info->n_selected = n;
                if (n > cap) atomicOr(&info->overflow, kOvfSelect);
            }
        }
    }
    __syncthreads();
    const uint32_t excl = s_excl;
    const float t = fp->t, w_o = fp->w_o;
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < kSelItems; r++) {
        const uint32_t s = (bits >> (2 * r)) & 3u;
        const unsigned long long m = __ballot(s != 0u);
        if (s != 0u) {
            const uint32_t pos = excl + s_cnt[r * 4 + wave] + (uint32_t)__popcll(m & lt);
            if (pos < cap) {
                ids[pos] = L.base + i0 + (uint32_t)r * kSelBlock + tid;
                w[pos] = (s == 3u) ? 1.0f : (s == 1u ? t : w_o);
            }
        }
    }
}

}  // namespace

hipError_t launch_select_setup(const LevelsArg& lv, const ChunksArg& ch, int32_t mode, const Views& v, hipStream_t st)
{
    const uint32_t n = std::max<uint32_t>(lv.sel_blocks, 1);   // an empty scene still runs one block (count 0)
    uint32_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    k_zero64<<<blocks, 256, 0, st>>>(v.sel_flags, n);
    k_select_setup<<<1, 64, 0, st>>>(ch, lv, mode, v.params, v.info);
    return hipGetLastError();
}

hipError_t launch_select(const LevelsArg& lv, const Views& v, const lodge_selection& sel, hipStream_t st)
{
    const uint32_t ntiles = std::max<uint32_t>(lv.sel_blocks, 1);
    k_select<<<ntiles, kSelBlock, 0, st>>>(lv, v.params, v.info, v.sel_flags, ntiles, sel.ids, sel.w, sel.cap,
                                           sel.count);
    return hipGetLastError();
}

}  // namespace lodge
