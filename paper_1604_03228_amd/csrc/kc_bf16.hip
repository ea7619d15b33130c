// kc_bf16.hip -- Gonzalez steps over BF16 points with exact FP32 rescoring.
//
// Per point i the stream keeps s_i, the min over steps of the canonical FP32
// squared distance computed from the BF16 coordinates x~_i (exactly
// representable in FP32) to the center's exact FP32 coordinates.  With
//   e_i   = |x~_i - x_i|           (per point, rounded up)
//   gamma = gamma_{d+2}            (canonical FP32 distance error)
// the canonical FP32 min-distance m_i of the FP32 path (the value the FP32
// stream would hold) lies in [lo(s_i), hi(s_i)] with
//   lo(s) = (1-gamma) max(0, sqrt(s/(1+gamma)) - e_i)^2
//   hi(s) = (1+gamma) (sqrt(s/(1-gamma)) + e_i)^2
// (triangle inequality for the BF16 rounding, gamma for the FP32 sums; both
// bounds are monotone in s, so they survive the min over steps).  A step:
//   k_gon_step_bf16   updates s_i, reduces the largest lower bound into the
//                     step's partial slots (L_t is their max) and lists every
//                     point whose upper bound reaches its own tile's largest
//                     lower bound -- a superset of the candidates, since a
//                     tile's bound never exceeds L_t;
//   k_bf16_rescore    keeps the listed points with hi_i >= L_t and computes
//                     their exact canonical FP32 min-distance with one wave
//                     each, over the centers chosen since the point was last
//                     rescored (cached per point), then offers the packed key
//                     to the step's argmax slots.
// The farthest point of the FP32 path (lowest index on ties) always has
// hi >= m >= L_t, so the argmax over candidates is exactly the FP32 path's.
#include "kc_host.h"

#define KC_BF_PTS 8   // points per lane: one 16-byte load per coordinate row
#define KC_BF_TILE (KC_BLOCK * KC_BF_PTS)

__device__ __forceinline__ float kc_bf_lo(float s, float e, float g)
{
    // every rounding is covered by the 16u margins folded into g by the host
    const float a = s * (1.f - g);
    float r = __builtin_sqrtf(a) * (1.f - 1e-6f) - e;
    r = r > 0.f ? r : 0.f;
    return r * r * (1.f - g);
}
__device__ __forceinline__ float kc_bf_hi(float s, float e, float g)
{
    const float a = s * (1.f + g);
    const float r = __builtin_sqrtf(a) * (1.f + 1e-6f) + e;
    return r * r * (1.f + g);
}

__device__ __forceinline__ float kc_bf_dec(uint32_t w, int hi)
{
    return __uint_as_float(hi ? (w & 0xFFFF0000u) : (w << 16));
}

// largest-lower-bound partial maxima: lpart[(key * KC_PARTS + slot) * 32]
// (u32 bits of a non-negative float, one 128-byte line per slot)
__device__ __forceinline__ uint32_t* kc_lpart(uint32_t* lpart, uint64_t key, uint32_t slot)
{
    return lpart + (key * KC_PARTS + slot) * 32;
}
__device__ __forceinline__ float kc_lpart_max(const uint32_t* lpart, uint64_t key)
{
    uint32_t v = 0;
    for (uint32_t s = 0; s < KC_PARTS; ++s) {
        const uint32_t x = __hip_atomic_load(lpart + (key * KC_PARTS + s) * 32,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = x > v ? x : v;
    }
    return __uint_as_float(v);
}

template <int D>
__global__ __launch_bounds__(KC_BLOCK) void k_gon_step_bf16(
    const uint16_t* __restrict__ xb, const float* __restrict__ xs, uint64_t stride, int d_rt,
    const float* __restrict__ ex, float* __restrict__ mind, u64* __restrict__ part,
    uint32_t* __restrict__ lpart, float* __restrict__ ccoord, const KcSeg* __restrict__ segs,
    const uint32_t* __restrict__ blk_seg, const uint32_t* __restrict__ blk_start, int t,
    float g, u64* __restrict__ list, float* __restrict__ list_hi,
    uint32_t* __restrict__ listcnt, uint32_t region)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ float red[KC_BLOCK / 64];
    __shared__ float sL;
    __shared__ uint32_t scount, sbase;
    const uint32_t b = blockIdx.x;
    const uint32_t sidx = blk_seg[b];
    const KcSeg sg = segs[sidx];
    if ((uint32_t)t >= sg.ksteps) return;
    const uint32_t loc = blk_start[b] + threadIdx.x * KC_BF_PTS;
    const uint64_t col = sg.base + loc;
    const bool live = loc < sg.len;

    float4 m0 = make_float4(0.f, 0.f, 0.f, 0.f), m1 = m0, e0 = m0, e1 = m0;
    if (live) {
        m0 = *(const float4*)(mind + col);
        m1 = *(const float4*)(mind + col + 4);
        e0 = *(const float4*)(ex + col);
        e1 = *(const float4*)(ex + col + 4);
    }
    uint32_t c;
    if (t == 0) {
        c = sg.first;
    } else {
        const int lane = threadIdx.x & 63;
        u64 pv = 0;
        if (lane < KC_PARTS)
            pv = __hip_atomic_load(kc_part_slot(part, sg.keyoff + t - 1, lane),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pv = kc_wave_max64(pv);
        if ((pv >> 32) == 0) return;   // radius reached 0: segment finished
        c = __builtin_amdgcn_readfirstlane(kc_key_idx(pv));
    }
    const float* xc = xs + sg.base + c;
    if (blk_start[b] == 0) {
        for (int j = threadIdx.x; j < d; j += KC_BLOCK)
            ccoord[(uint64_t)(sg.keyoff + t) * d + j] = xc[(uint64_t)j * stride];
    }
    float s[KC_BF_PTS];
#pragma unroll
    for (int q = 0; q < KC_BF_PTS; ++q) s[q] = 0.f;
    if (live) {
        constexpr int CH = 2;   // coordinate rows per pass: few VGPRs, many waves
#pragma unroll 1
        for (int j0 = 0; j0 < d; j0 += CH) {
            uint4 w4[CH];
            float cc[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (j0 + u < d) {
                    w4[u] = *(const uint4*)(xb + (uint64_t)(j0 + u) * stride + col);
                    cc[u] = xc[(uint64_t)(j0 + u) * stride];
                }
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (j0 + u < d) {
                    const uint32_t w[4] = {w4[u].x, w4[u].y, w4[u].z, w4[u].w};
#pragma unroll
                    for (int q = 0; q < KC_BF_PTS; ++q)
                        s[q] = kc_d32_step(s[q], kc_bf_dec(w[q >> 1], q & 1), cc[u]);
                }
        }
    }
    float lo = 0.f;
    float hq[KC_BF_PTS];
#pragma unroll
    for (int q = 0; q < KC_BF_PTS; ++q) hq[q] = -1.f;
    if (live) {
        float mm[KC_BF_PTS] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
        const float ee[KC_BF_PTS] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
        for (int q = 0; q < KC_BF_PTS; ++q) {
            mm[q] = fminf(mm[q], s[q]);
            if (loc + q < sg.len) {
                lo = fmaxf(lo, kc_bf_lo(mm[q], ee[q], g));
                hq[q] = kc_bf_hi(mm[q], ee[q], g);
            }
        }
        *(float4*)(mind + col) = make_float4(mm[0], mm[1], mm[2], mm[3]);
        *(float4*)(mind + col + 4) = make_float4(mm[4], mm[5], mm[6], mm[7]);
    }
    for (int off = 32; off >= 1; off >>= 1) lo = fmaxf(lo, __shfl_xor(lo, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lo;
    if (threadIdx.x == 0) scount = 0;
    __syncthreads();
    const uint32_t slot = b % KC_PARTS;
    if (threadIdx.x == 0) {
        float L = red[0];
        for (int w = 1; w < KC_BLOCK / 64; ++w) L = fmaxf(L, red[w]);
        sL = L;
        uint32_t* p = kc_lpart(lpart, sg.keyoff + t, slot);
        const uint32_t lb = __float_as_uint(L);
        if (lb > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_fetch_max(p, lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // list the tile's points that can reach the tile's own largest lower
    // bound (a lower bound of L_t, so the list is a superset of the step's
    // candidates; the rescoring kernel applies L_t itself)
    const float Lb = sL;
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < KC_BF_PTS; ++q) mine += hq[q] >= Lb;
    const uint32_t off = mine ? atomicAdd(&scount, mine) : 0u;
    __syncthreads();
    // one of KC_PARTS list regions (each on its own counter line), so tiles do
    // not serialise on one address; region `slot` holds at most the points of
    // the tiles b with b mod KC_PARTS == slot
    if (threadIdx.x == 0)
        sbase = scount ? slot * region + atomicAdd(&listcnt[((uint64_t)t * KC_PARTS + slot) * 32],
                                                   scount)
                       : 0u;
    __syncthreads();
    if (mine) {
        uint32_t w = sbase + off;
#pragma unroll
        for (int q = 0; q < KC_BF_PTS; ++q)
            if (hq[q] >= Lb) {
                list[w] = ((u64)sidx << 32) | (loc + q);
                list_hi[w] = hq[q];
                ++w;
            }
    }
}

// Rescoring of step t.  Every block first computes L_t of each segment (the
// max over its partial slots) into LDS.  Then each wave takes 64 listed
// points at a time, one per lane, keeps those with hi >= L_t of their segment
// and rescores the kept ones one after another with the whole wave: lanes
// over the centers chosen since the point was last rescored (exm/exupto
// cache it), canonical FP32, then the packed key goes to the step's argmax
// slots.  nresc[t] counts the rescored points.
#define KC_RESC_SEGS 1024   // segments whose L_t fits the LDS table
#define KC_RESC_LT_SEGS 8   // above this many segments L_t comes from k_bf16_lt

// L_t of every segment for step t (the max over its partial slots), one
// thread per segment, so that the rescoring blocks of a run with many
// segments read one word per listed point instead of every segment's slots.
__global__ void k_bf16_lt(const uint32_t* __restrict__ lpart, const KcSeg* __restrict__ segs,
                          int nseg, int t, float* __restrict__ Lt)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const KcSeg sg = segs[s];
    uint32_t v = 0;
    if ((uint32_t)t < sg.ksteps)
        for (uint32_t p = 0; p < KC_PARTS; ++p) {
            const uint32_t x = lpart[((uint64_t)(sg.keyoff + t) * KC_PARTS + p) * 32];
            v = x > v ? x : v;
        }
    Lt[s] = __uint_as_float(v);
}

template <int D>
__global__ __launch_bounds__(256) void k_bf16_rescore(
    const u64* __restrict__ list, const float* __restrict__ list_hi,
    const uint32_t* __restrict__ listcnt, uint32_t region, const uint32_t* __restrict__ lpart,
    const float* __restrict__ xs, uint64_t stride, int d, const float* __restrict__ ccoord,
    const KcSeg* __restrict__ segs, int nseg, float* __restrict__ exm,
    uint32_t* __restrict__ exupto, u64* __restrict__ part, uint32_t* __restrict__ nresc, int t,
    const float* __restrict__ Lt)
{
    __shared__ float sL[KC_RESC_SEGS];
    __shared__ uint32_t sinc[KC_PARTS];
    __shared__ float sx[4 * KC_MAXD];   // one coordinate row per wave
    const int lane = threadIdx.x & 63;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    // L_t per segment (the step's partial slots are final: written by the
    // step kernel that ran before this one); KC_PARTS lanes per segment
    const int nsl = Lt ? 0 : (nseg < KC_RESC_SEGS ? nseg : KC_RESC_SEGS);
    for (int s0 = 0; s0 < nsl; s0 += (int)blockDim.x / KC_PARTS) {
        const int s = s0 + (int)threadIdx.x / KC_PARTS, p = threadIdx.x % KC_PARTS;
        uint32_t x = 0;
        if (s < nsl) {
            const KcSeg sg = segs[s];
            if ((uint32_t)t < sg.ksteps)
                x = lpart[((uint64_t)(sg.keyoff + t) * KC_PARTS + p) * 32];
        }
        for (int off = KC_PARTS / 2; off >= 1; off >>= 1) {
            const uint32_t o = __shfl_xor(x, off, 64);
            x = o > x ? o : x;
        }
        if (p == 0 && s < nsl) sL[s] = __uint_as_float(x);
    }
    if (threadIdx.x < 64) {
        // inclusive prefix of the region counts
        uint32_t inc = lane < KC_PARTS ? listcnt[((uint64_t)t * KC_PARTS + lane) * 32] : 0u;
        for (int off = 1; off < KC_PARTS; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off) inc += y;
        }
        if (lane < KC_PARTS) sinc[lane] = inc;
    }
    __syncthreads();
    const uint32_t total = sinc[KC_PARTS - 1];
    // every wave takes an equal share of the list, at most 64 entries at a time,
    // so the rescoring of kept entries spreads over all waves of the grid
    const uint32_t wid = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    uint32_t share = (total + waves - 1) / waves;
    if (share > 64) share = 64;
    if (share == 0) share = 1;
    float* xw = sx + (threadIdx.x >> 6) * KC_MAXD;
    uint32_t done = 0;
    for (uint32_t base = wid * share; base < total; base += waves * share) {
        const uint32_t q = base + lane;
        bool keep = false;
        u64 e = 0;
        if (lane < (int)share && q < total) {
            // flat index -> (region, offset)
            uint32_t rg = 0;
            while (sinc[rg] <= q) ++rg;
            const uint32_t before = rg ? sinc[rg - 1] : 0u;
            const uint64_t qi = (uint64_t)rg * region + (q - before);
            e = list[qi];
            const uint32_t sidx = (uint32_t)(e >> 32);
            float L;
            if (Lt) {
                L = Lt[sidx];
            } else if (sidx < KC_RESC_SEGS) {
                L = sL[sidx];
            } else {
                uint32_t v = 0;
                const KcSeg sg = segs[sidx];
                for (uint32_t p = 0; p < KC_PARTS; ++p) {
                    const uint32_t x = lpart[((uint64_t)(sg.keyoff + t) * KC_PARTS + p) * 32];
                    v = x > v ? x : v;
                }
                L = __uint_as_float(v);
            }
            keep = list_hi[qi] >= L;
        }
        u64 mask = __ballot(keep);
        while (mask) {
            const int j = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            const u64 ej = __shfl(e, j, 64);
            const uint32_t sidx = (uint32_t)(ej >> 32), loc = (uint32_t)ej;
            const KcSeg sg = segs[sidx];
            const uint64_t col = sg.base + loc;
            // the point's coordinates once into this wave's LDS row
            for (int u = lane; u < d; u += 64) xw[u] = xs[(uint64_t)u * stride + col];
            const uint32_t from = exupto[col];
            float best = exm[col];
            __builtin_amdgcn_wave_barrier();
            if (D > 0) {
                // two centers per lane and pass, every coordinate load of
                // both issued before the arithmetic: one memory latency per
                // 128 centers
                for (uint32_t c = from + lane; c <= (uint32_t)t; c += 128) {
                    const bool two = c + 64 <= (uint32_t)t;
                    const float* c0 = ccoord + (uint64_t)(sg.keyoff + c) * D;
                    const float* c1 = two ? c0 + 64 * D : c0;
                    float v0[D > 0 ? D : 1], v1[D > 0 ? D : 1];
#pragma unroll
                    for (int u = 0; u < D; ++u) {
                        v0[u] = c0[u];
                        v1[u] = c1[u];
                    }
                    float a0 = 0.f, a1 = 0.f;
#pragma unroll
                    for (int u = 0; u < D; ++u) {
                        a0 = kc_d32_step(a0, xw[u], v0[u]);
                        a1 = kc_d32_step(a1, xw[u], v1[u]);
                    }
                    best = fminf(best, a0);
                    if (two) best = fminf(best, a1);
                }
            } else {
                for (uint32_t c = from + lane; c <= (uint32_t)t; c += 64) {
                    const float* cj = ccoord + (uint64_t)(sg.keyoff + c) * d;
                    float acc = 0.f;
                    for (int u = 0; u < d; ++u) acc = kc_d32_step(acc, xw[u], cj[u]);
                    best = fminf(best, acc);
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int off = 32; off >= 1; off >>= 1) best = fminf(best, __shfl_xor(best, off, 64));
            if (lane == 0) {
                exm[col] = best;
                exupto[col] = (uint32_t)t + 1;
                kc_part_offer(part, sg.keyoff + t, (base + j) % KC_PARTS, kc_pack(best, loc));
            }
            ++done;
        }
    }
    if (lane == 0 && done) atomicAdd(&nresc[t], done);
}

// Final-radius candidates in BF16 mode: hi_i >= L_last * (1 - band), where
// L_last is the largest lower bound after the last step; the band covers the
// FP32 error between the exact maximiser and the FP32 values.
__global__ void k_bf16_radius_cand(const float* __restrict__ mind, const float* __restrict__ ex,
                                   const uint32_t* __restrict__ lpart,
                                   const KcSeg* __restrict__ segs,
                                   const uint32_t* __restrict__ blk_seg,
                                   const uint32_t* __restrict__ blk_start,
                                   const int64_t* __restrict__ n_chosen, float g, double band,
                                   u64* __restrict__ cand, uint32_t* __restrict__ ncand,
                                   uint32_t cap)
{
    const uint32_t b = blockIdx.x;
    const uint32_t sidx = blk_seg[b];
    const KcSeg sg = segs[sidx];
    const int64_t nch = n_chosen[sidx];
    if (nch <= 0) return;
    const float L = kc_lpart_max(lpart, sg.keyoff + nch - 1);
    const double thr = (double)L * (1.0 - band);
    for (int q = 0; q < KC_BF_PTS; ++q) {
        const uint32_t loc = blk_start[b] + q * KC_BLOCK + threadIdx.x;
        if (loc >= sg.len) continue;
        const uint64_t col = sg.base + loc;
        if ((double)kc_bf_hi(mind[col], ex[col], g) >= thr) {
            const uint32_t slot = atomicAdd(ncand, 1u);
            if (slot < cap) cand[slot] = ((u64)sidx << 32) | loc;
        }
    }
}

#define KC_BF_CASE(DD)                                                                    \
    case DD:                                                                              \
        hipLaunchKernelGGL(k_gon_step_bf16<DD>, dim3(R.nblk), dim3(KC_BLOCK), 0, s, B.xb,  \
                           R.xs, R.stride, R.d, B.ex, R.mind, R.part, B.lpart, R.ccoord,   \
                           R.segs, R.blk_seg, R.blk_start, t, B.g, B.list, B.list_hi,      \
                           B.listcnt, B.region);                                           \
        break;

void kc_enqueue_bf16_steps(const KcGonRun& R, const KcBf16Run& B, hipStream_t s)
{
    for (int t = 0; t < (int)R.kmax; ++t) {
        switch (R.d) {
            KC_BF_CASE(2)
            KC_BF_CASE(8)
            KC_BF_CASE(10)
            KC_BF_CASE(16)
            KC_BF_CASE(32)
            KC_BF_CASE(41)
        default:
            hipLaunchKernelGGL(k_gon_step_bf16<0>, dim3(R.nblk), dim3(KC_BLOCK), 0, s, B.xb,
                               R.xs, R.stride, R.d, B.ex, R.mind, R.part, B.lpart, R.ccoord,
                               R.segs, R.blk_seg, R.blk_start, t, B.g, B.list, B.list_hi,
                               B.listcnt, B.region);
        }
        const float* Lt = nullptr;
        if (R.nseg > KC_RESC_LT_SEGS) {
            hipLaunchKernelGGL(k_bf16_lt, dim3((R.nseg + 255) / 256), dim3(256), 0, s, B.lpart,
                               R.segs, R.nseg, t, B.Lt);
            Lt = B.Lt;
        }
        switch (R.d) {
#define KC_RS_CASE(DD)                                                                        \
    case DD:                                                                                  \
        hipLaunchKernelGGL(k_bf16_rescore<DD>, dim3(B.rescore_blocks), dim3(256), 0, s, B.list, \
                           B.list_hi, B.listcnt, B.region, B.lpart, R.xs, R.stride, R.d,      \
                           R.ccoord, R.segs, R.nseg, B.exm, B.exupto, R.part, B.nresc, t, Lt); \
        break;
            KC_RS_CASE(2)
            KC_RS_CASE(8)
            KC_RS_CASE(10)
            KC_RS_CASE(16)
            KC_RS_CASE(32)
            KC_RS_CASE(41)
#undef KC_RS_CASE
        default:
            hipLaunchKernelGGL(k_bf16_rescore<0>, dim3(B.rescore_blocks), dim3(256), 0, s, B.list,
                               B.list_hi, B.listcnt, B.region, B.lpart, R.xs, R.stride, R.d,
                               R.ccoord, R.segs, R.nseg, B.exm, B.exupto, R.part, B.nresc, t,
                               Lt);
        }
    }
    kc_part_collect(R.part, R.keys, R.keysum, s);
}

void kc_enqueue_bf16_prep(const KcGonRun& R, const KcBf16Run& B, const KcGonHost& H,
                          const std::vector<KcGonJob>& jobs, hipStream_t s)
{
    kc_enqueue_stage(R, H, jobs, s, B.xb, B.ex);
    kc_fill_u32((uint32_t*)R.mind, 0x7F800000u, R.stride, s);   // +inf
    kc_fill_u32((uint32_t*)B.exm, 0x7F800000u, R.stride, s);
    kc_fill_u32(B.exupto, 0u, R.stride, s);
    kc_fill_u64(R.part, 0ull, R.keysum * KC_PARTS * KC_PSTRIDE, s);
    kc_fill_u32(B.lpart, 0u, R.keysum * KC_PARTS * 32, s);
    kc_fill_u32(B.listcnt, 0u, (uint64_t)R.kmax * KC_PARTS * 32, s);
    kc_fill_u32(B.nresc, 0u, R.kmax, s);
}

// Finishing in BF16 mode: centers, trace (FP64, from the centers' exact
// coordinates recorded by the steps) and the exact radius from bound-based
// candidates.
void kc_bf16_finish(const KcGonRun& R, const KcBf16Run& B, int64_t* centers,
                    int64_t* n_chosen, double* trace, double* radius_out,
                    const int64_t* report_base, hipStream_t s)
{
    kc_gon_finish_impl(R, centers, n_chosen, trace, radius_out, report_base, nullptr, false, s,
                       [&](hipStream_t st) {
                           hipLaunchKernelGGL(k_bf16_radius_cand, dim3(R.nblk), dim3(KC_BLOCK),
                                              0, st, R.mind, B.ex, B.lpart, R.segs, R.blk_seg,
                                              R.blk_start, n_chosen, B.g, R.band, R.cand,
                                              R.ncand, R.cand_cap);
                       });
}
