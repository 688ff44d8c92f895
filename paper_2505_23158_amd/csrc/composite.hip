// Front-to-back alpha compositing (LODGE Sec. 3 "Preliminaries", Eq. 1:
// alpha = o G(p), G = exp(-1/2 (p - mu')^T Sigma'^-1 (p - mu'))).
//
// Each 16 x 16 tile is split into four 8 x 8 quadrants and every quadrant is
// one wave that works on its own: the waves of a block share no data and
// never wait for each other, so a quadrant that reaches full opacity stops
// at once.  Blocks take tiles longest-list first.  Inside a wave, each group
// of 16 lanes is a 4 x 4 sub-quadrant with a list of its own.
//
// A wave walks its tile's sorted run in batches of 64, the gathers of the
// next batch in flight while the current one is composited.  Each lane
// takes one splat of the batch, stores its record in the wave's LDS slice
// and tests where its alpha can reach 1/255: against the quadrant, a
// bounding-box test on that ellipse (half-extents ex, ey from the
// projection) and then the exact minimum of the conic quadratic form over
// the quadrant's box of pixel centres; against each sub-quadrant, the
// bounding box.  Ballots compact the survivors, in list order, into one
// slot list per sub-quadrant, the shorter ones padded with a slot every
// pixel skips; the wave then runs as many steps as the longest list, each
// lane following its own, predicated, with the next entry read one step
// ahead.  Per (pixel, splat): power = -1/2
// (A dx^2 + C dy^2) - B dx dy; alpha = min(0.99, o exp(power)); skip if
// power > 0 or alpha < 1/255 (as is every power below the splat's threshold
// ln(1/(255 o)) - 1e-3, which the culling uses); stop (without blending)
// once T (1 - alpha) < 1e-4; else C += rgb alpha T, T *= 1 - alpha.  A splat
// dropped for a sub-quadrant changes no decision: the tests keep every
// splat that any of its pixels would not skip, with a margin above the
// rounding of both computations.
//
// Per-wave pair counters go to one slot each (no atomics); the host sums
// them when the frame info is read.
#include "lodge_internal.hpp"
#include "splat.hpp"

namespace lodge {

namespace {

// Records of one wave: three thirds of 65 float4 (65 = 64 batch slots + the
// sentinel), each third one float4 of the projected record in its stored
// form: [0] u, v, -A/2, -B; [1] -C/2, o, threshold, r; [2] g, b, ex, ey.
constexpr uint32_t kSlots = 65;
constexpr uint32_t kWaveRec = 3 * kSlots;
constexpr uint32_t kThird = kSlots * sizeof(float4);   // bytes between the thirds
constexpr uint32_t kListLen = 68;

// kScore: the importance variant.  Instead of the image it max-accumulates
// each blended entry's weight alpha T into score[ids[a]] (float bits,
// non-negative, so unsigned order is float order): per batch, every lane
// takes an LDS max on its entry's slot; after the walk each slot's maximum
// over the wave's pixels goes out with one global atomic max.
template <bool kScore>
__global__ __launch_bounds__(256) void k_composite(const FrameParams* __restrict__ fp,
                                                   const uint2* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ sorted,
                                                   const float4* __restrict__ proj, float* __restrict__ image,
                                                   float* __restrict__ final_T, uint32_t* __restrict__ n_contrib,
                                                   uint4* __restrict__ wstats, uint32_t cap,
                                                   const uint32_t* __restrict__ sel_ids, uint32_t* __restrict__ score)
{
    // Slot 64 of every wave is a sentinel every pixel skips (threshold
    // +inf): it pads the shorter sub-quadrant lists to the longest.  The
    // lists hold LDS byte offsets (from s_rec) of the first third of a slot.
    __shared__ float4 s_rec[4 * kWaveRec];
    // per wave and sub-quadrant; 4 entries past the 64 a batch can fill,
    // always the sentinel, for the reads one trip ahead
    __shared__ uint32_t s_idx[4][4][kListLen];
    // importance variant: per wave and batch slot, the largest weight (float bits)
    __shared__ uint32_t s_wmax[kScore ? 4 : 1][kScore ? kSlots : 1];

    const int32_t W = fp->cam.width, H = fp->cam.height, TX = fp->TX;
    const uint32_t tile = order[blockIdx.x];
    const uint32_t tx = tile % (uint32_t)TX, ty = tile / (uint32_t)TX;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t sub = lane >> 4;
    const uint32_t qx0 = tx * kTile + (wave & 1u) * 8u, qy0 = ty * kTile + (wave >> 1) * 8u;
    const uint32_t x = qx0 + (sub & 1u) * 4u + (lane & 3u), y = qy0 + (sub >> 1) * 4u + ((lane >> 2) & 3u);
    const bool inside = (int32_t)x < W && (int32_t)y < H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float bx0 = (float)qx0 + 0.5f, by0 = (float)qy0 + 0.5f;
    const uint2 rg = ranges[tile];
    const uint32_t len = rg.y - rg.x;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t rbase = wave * kWaveRec;   // the wave's first record (float4 index)
    float4* const sa = s_rec + rbase;
    const char* const rec = reinterpret_cast<const char*>(s_rec);
    const uint32_t* const sidx = s_idx[wave][sub];
    const uint32_t own_off = (rbase + lane) * (uint32_t)sizeof(float4);
    const uint32_t sent_off = (rbase + 64u) * (uint32_t)sizeof(float4);
    constexpr uint32_t kNone = 0xffffffffu;

    if (lane == 0) {
        sa[64] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        sa[kSlots + 64] = make_float4(0.0f, 0.0f, INFINITY, 0.0f);
        sa[2 * kSlots + 64] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    // every list position starts as the sentinel, so a read ahead past the
    // end of a list always lands on a record of this wave
#pragma unroll
    for (int g = 0; g < 4; g++) {
        s_idx[wave][g][lane] = sent_off;
        if (lane < kListLen - 64) s_idx[wave][g][64 + lane] = sent_off;
    }

    float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
    uint32_t last = 0, nblend = 0, neval = len;
    // the alpha a splat needs to count: +inf once the pixel is done (stopped, or outside the image)
    float amin = inside ? kAlphaMin : INFINITY;

    // software pipeline: records of batch b in r*, of batch b + 1 in flight,
    // the list index of batch b + 2 in flight
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    if (lane < len) {
        uint32_t a = sorted[rg.x + lane];
        a = a < cap ? a : 0u;   // an index outside the active set would be a binning bug
        r0 = proj[3 * (size_t)a];
        r1 = proj[3 * (size_t)a + 1];
        r2 = proj[3 * (size_t)a + 2];
    }
    uint32_t a_next = 64 + lane < len ? sorted[rg.x + 64 + lane] : 0u;
    // importance variant: the active index of the lane's entry in the current batch
    uint32_t a_cur = 0;
    if (kScore && lane < len) a_cur = sorted[rg.x + lane];

    for (uint32_t b0 = 0; b0 < len; b0 += 64) {
        if (__ballot(amin < INFINITY) == 0ull) break;
        const uint32_t k = b0 + lane;
        const bool cur = k < len;
        const float4 q0 = r0, q1 = r1, q2 = r2;
        const uint32_t a_batch = a_cur;
        if (kScore) a_cur = a_next;
        if (b0 + 64 + lane < len) {
            const uint32_t a = a_next < cap ? a_next : 0u;
            r0 = proj[3 * (size_t)a];
            r1 = proj[3 * (size_t)a + 1];
            r2 = proj[3 * (size_t)a + 2];
        }
        a_next = b0 + 128 + lane < len ? sorted[rg.x + b0 + 128 + lane] : 0u;
        if (kScore) s_wmax[wave][lane] = 0u;

        bool hit[4] = {false, false, false, false};
        if (cur) {
            sa[lane] = q0;
            sa[kSlots + lane] = q1;
            sa[2 * kSlots + lane] = q2;
            const BoxTest bt = box_test(q0, q1, q2);
            // exact test for the quadrant, bounding boxes for its sub-quadrants
            if (reaches(bt, bx0, bx0 + 7.0f, by0, by0 + 7.0f)) {
#pragma unroll
                for (int g = 0; g < 4; g++) {
                    const float sx0 = bx0 + (float)((g & 1) * 4), sy0 = by0 + (float)((g >> 1) * 4);
                    hit[g] = box_overlaps(bt, sx0, sx0 + 3.0f, sy0, sy0 + 3.0f);
                }
            }
        }
        uint32_t cnt[4], n_max = 0;
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const unsigned long long m = __ballot(hit[g]);
            if (hit[g]) s_idx[wave][g][__popcll(m & lt)] = own_off;
            cnt[g] = (uint32_t)__popcll(m);
            n_max = cnt[g] > n_max ? cnt[g] : n_max;
        }
        // pad every sub-quadrant list to the longest with the sentinel slot
#pragma unroll
        for (int g = 0; g < 4; g++)
            if (lane >= cnt[g] && lane < n_max) s_idx[wave][g][lane] = sent_off;
        // the wave's own LDS slice: order its writes before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // walk the lane's sub-quadrant list two entries per trip, predicated
        // rather than branched, each entry's records read one entry ahead
        if (n_max > 0 && __ballot(amin < INFINITY) != 0ull) {
            uint32_t last_off = kNone, stop_off = kNone;
            // one (pixel, splat) pair; off: the splat's record offset
            auto step = [&](const float4& g, const float4& c, const float2& f, uint32_t off) {
                float alpha;
                const bool keep = splat_keep(g, c, px, py, amin, alpha);
                const float Tn = T * (1.0f - alpha);
                const bool stop = keep && Tn < kTStop;
                if (stop) {
                    amin = INFINITY;
                    stop_off = off;
                }
                if (keep && !stop) {
                    const float wgt = alpha * T;
                    if (kScore) atomicMax(&s_wmax[wave][(off / (uint32_t)sizeof(float4)) - rbase], __float_as_uint(wgt));
                    cr = __builtin_fmaf(c.w, wgt, cr);
                    cg = __builtin_fmaf(f.x, wgt, cg);
                    cb = __builtin_fmaf(f.y, wgt, cb);
                    T = Tn;
                    last_off = off;
                    nblend++;
                }
            };
            auto load = [&](uint32_t off, float4& g, float4& c, float2& f) {
                g = *reinterpret_cast<const float4*>(rec + off);
                c = *reinterpret_cast<const float4*>(rec + off + kThird);
                f = *reinterpret_cast<const float2*>(rec + off + 2 * kThird);
            };
            uint32_t eA = sidx[0], eB = sidx[1];
            float4 gA, cA, gB, cB;
            float2 fA, fB;
            load(eA, gA, cA, fA);
            for (uint32_t j = 0; j < n_max; j += 2) {
                if (__ballot(amin < INFINITY) == 0ull) break;
                const uint32_t* const p = sidx + j;   // p[2], p[3] < kListLen: j <= 63
                load(eB, gB, cB, fB);
                const uint32_t eA2 = p[2];
                step(gA, cA, fA, eA);
                if (j + 1 >= n_max) break;
                load(eA2, gA, cA, fA);
                const uint32_t eB2 = p[3];
                step(gB, cB, fB, eB);
                eA = eA2;
                eB = eB2;
            }
            // list offsets back to positions in the tile's run
            if (last_off != kNone) last = b0 + (last_off / (uint32_t)sizeof(float4) - rbase) + 1u;
            if (stop_off != kNone) neval = b0 + (stop_off / (uint32_t)sizeof(float4) - rbase) + 1u;
        }
        // every lane is past its reads before the next batch overwrites the slice
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (kScore && cur) {
            const uint32_t m = s_wmax[wave][lane];
            if (m != 0u) atomicMax(score + sel_ids[a_batch < cap ? a_batch : 0u], m);
        }
    }
    if (kScore) return;
    if (inside) {
        const size_t p = (size_t)y * W + x;
        const size_t HW = (size_t)W * H;
        // outputs, not read again by this frame: streamed past the caches
        __builtin_nontemporal_store(cr + T * fp->cam.bg[0], image + p);
        __builtin_nontemporal_store(cg + T * fp->cam.bg[1], image + HW + p);
        __builtin_nontemporal_store(cb + T * fp->cam.bg[2], image + 2 * HW + p);
        __builtin_nontemporal_store(T, final_T + p);
        __builtin_nontemporal_store(last, n_contrib + p);
    } else {
        neval = 0;
    }
    // per-wave counters, one slot per (tile, quadrant)
    unsigned long long ev = neval;
    uint32_t bl = nblend;
    const uint32_t stopped = (uint32_t)__popcll(__ballot(inside && !(amin < INFINITY)));
    for (int off = 32; off > 0; off >>= 1) {
        ev += __shfl_xor(ev, off);
        bl += __shfl_xor(bl, off);
    }
    if (lane == 0) wstats[4 * tile + wave] = make_uint4((uint32_t)ev, (uint32_t)(ev >> 32), bl, stopped);
}

}  // namespace

hipError_t launch_composite(const Views& v, float* image, float* final_T, uint32_t* n_contrib, hipStream_t st)
{
    k_composite<false><<<v.lay.T, 256, 0, st>>>(v.params, v.ranges, v.order, v.sorted, v.proj, image, final_T,
                                                n_contrib, v.wstats, v.max_active, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_importance(const Views& v, const uint32_t* sel_ids, float* score, hipStream_t st)
{
    k_composite<true><<<v.lay.T, 256, 0, st>>>(v.params, v.ranges, v.order, v.sorted, v.proj, nullptr, nullptr,
                                               nullptr, v.wstats, v.max_active, sel_ids,
                                               reinterpret_cast<uint32_t*>(score));
    return hipGetLastError();
}

}  // namespace lodge
