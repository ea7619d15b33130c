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
//   k_gon_step_bf16   update s_i, reduce max lo into per-step partial slots,
//                     record each block's max hi;
//   k_bf16_cand       every point with hi_i >= L_t = max lo becomes a
//                     candidate (blocks whose max hi is below L_t skip);
//   k_bf16_rescore    one wave per candidate computes its exact canonical
//                     FP32 min-distance over the centers chosen since it was
//                     last rescored (cached per point) and offers the packed
//                     key to the step's argmax slots.
// The farthest point of the FP32 path (lowest index on ties) always has
// hi >= L_t, so the argmax over candidates is exactly the FP32 path's choice.
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

// SoA BF16 staging of rows [row0, row0+len) plus the per-point rounding
// radius e_i (FP64, rounded up), indexed like the SoA columns.
__global__ void k_stage_bf16(const float* __restrict__ X, const uint16_t* __restrict__ Xb,
                             int64_t ld, int d, uint64_t row0, uint32_t len,
                             uint16_t* __restrict__ xb, float* __restrict__ ex, uint64_t stride,
                             uint64_t base, uint32_t padded)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    const uint64_t r = row0 + (i < len ? i : 0);
    double ee = 0.0;
    for (int j = 0; j < d; ++j) {
        const uint16_t h = Xb[r * ld + j];
        xb[(uint64_t)j * stride + base + i] = h;
        const double e = (double)__uint_as_float((uint32_t)h << 16) - (double)X[r * ld + j];
        ee += e * e;
    }
    ex[base + i] = (float)(sqrt(ee) * (1.0 + 1e-12)) * (1.f + 1e-6f);
}

void kc_stage_bf16(const float* X, const uint16_t* Xb, int64_t ld, int d, uint64_t row0,
                   uint32_t len, uint16_t* xb, float* ex, uint64_t stride, uint64_t base,
                   hipStream_t s)
{
    const uint32_t padded = kc_pad64(len);
    if (padded == 0) return;
    hipLaunchKernelGGL(k_stage_bf16, dim3((padded + 255) / 256), dim3(256), 0, s, X, Xb, ld, d,
                       row0, len, xb, ex, stride, base, padded);
}

// lo partial maxima: lpart[(key * KC_PARTS + slot) * 32] (u32 bits of a
// non-negative float, one 128-byte line per slot)
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
    uint32_t* __restrict__ lpart, float* __restrict__ blk_hi, float* __restrict__ ccoord,
    const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, int t, float g)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ float red[KC_BLOCK / 64];
    __shared__ float redh[KC_BLOCK / 64];
    const uint32_t b = blockIdx.x;
    const KcSeg sg = segs[blk_seg[b]];
    if ((uint32_t)t >= sg.ksteps) return;
    const uint32_t loc = blk_start[b] + threadIdx.x * KC_BF_PTS;
    const uint64_t col = sg.base + loc;
    const bool live = loc < sg.len;

    uint4 v[D > 0 ? D : 1];
    if (D > 0 && live) {
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = *(const uint4*)(xb + (uint64_t)j * stride + col);
    }
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
    const float* xc = xs + sg.base + c;   // exact FP32 center, uniform
    if (b == 0 || blk_start[b] == 0) {
        // the segment's first block records the center's coordinates
        for (int j = threadIdx.x; j < d; j += KC_BLOCK)
            ccoord[(uint64_t)(sg.keyoff + t) * d + j] = xc[(uint64_t)j * stride];
    }

    float s[KC_BF_PTS];
#pragma unroll
    for (int q = 0; q < KC_BF_PTS; ++q) s[q] = 0.f;
    if (live) {
        if (D > 0) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float cj = xc[(uint64_t)j * stride];
                const uint32_t w[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
                for (int q = 0; q < KC_BF_PTS; ++q)
                    s[q] = kc_d32_step(s[q], kc_bf_dec(w[q >> 1], q & 1), cj);
            }
        } else {
            for (int j = 0; j < d; ++j) {
                const uint4 u = *(const uint4*)(xb + (uint64_t)j * stride + col);
                const float cj = xc[(uint64_t)j * stride];
                const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int q = 0; q < KC_BF_PTS; ++q)
                    s[q] = kc_d32_step(s[q], kc_bf_dec(w[q >> 1], q & 1), cj);
            }
        }
    }
    float lo = 0.f, hi = 0.f;
    if (live) {
        float mm[KC_BF_PTS] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
        const float ee[KC_BF_PTS] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
        for (int q = 0; q < KC_BF_PTS; ++q) {
            mm[q] = fminf(mm[q], s[q]);
            if (loc + q < sg.len) {
                lo = fmaxf(lo, kc_bf_lo(mm[q], ee[q], g));
                hi = fmaxf(hi, kc_bf_hi(mm[q], ee[q], g));
            }
        }
        *(float4*)(mind + col) = make_float4(mm[0], mm[1], mm[2], mm[3]);
        *(float4*)(mind + col + 4) = make_float4(mm[4], mm[5], mm[6], mm[7]);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        lo = fmaxf(lo, __shfl_xor(lo, off, 64));
        hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = lo;
        redh[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float L = red[0], Hh = redh[0];
        for (int w = 1; w < KC_BLOCK / 64; ++w) {
            L = fmaxf(L, red[w]);
            Hh = fmaxf(Hh, redh[w]);
        }
        blk_hi[b] = Hh;
        uint32_t* p = kc_lpart(lpart, sg.keyoff + t, b % KC_PARTS);
        const uint32_t lb = __float_as_uint(L);
        if (lb > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_fetch_max(p, lb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Candidates of step t: hi_i >= L_t.  cand entries are (segment << 32 | loc);
// ncand[t] counts them over all segments (a fresh counter per step, so the
// shared candidate list never needs resetting inside the step loop).
__global__ void k_bf16_cand(const float* __restrict__ mind, const float* __restrict__ ex,
                            const float* __restrict__ blk_hi, const uint32_t* __restrict__ lpart,
                            const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
                            const uint32_t* __restrict__ blk_start, int t, float g,
                            u64* __restrict__ cand, uint32_t* __restrict__ ncand, uint32_t cap,
                            const u64* __restrict__ part)
{
    const uint32_t b = blockIdx.x;
    const uint32_t sidx = blk_seg[b];
    const KcSeg sg = segs[sidx];
    if ((uint32_t)t >= sg.ksteps) return;
    if (t > 0) {
        // a segment that stopped at the previous step has nothing to do
        const int lane = threadIdx.x & 63;
        u64 pv = 0;
        if (lane < KC_PARTS)
            pv = __hip_atomic_load(kc_part_slot((u64*)part, sg.keyoff + t - 1, lane),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pv = kc_wave_max64(pv);
        if ((pv >> 32) == 0) return;
    }
    const float L = kc_lpart_max(lpart, sg.keyoff + t);
    if (blk_hi[b] < L) return;
    for (int q = 0; q < KC_BF_PTS; ++q) {
        const uint32_t loc = blk_start[b] + q * KC_BLOCK + threadIdx.x;
        if (loc >= sg.len) continue;
        const uint64_t col = sg.base + loc;
        if (kc_bf_hi(mind[col], ex[col], g) >= L) {
            const uint32_t slot = atomicAdd(&ncand[t], 1u);
            if (slot < cap) cand[slot] = ((u64)sidx << 32) | loc;
        }
    }
}

// One wave per candidate: exact canonical FP32 min-distance over the centers
// chosen since the point was last rescored (exm/exupto cache it), then its
// packed key is offered to step t's argmax slots of its segment.
__global__ void k_bf16_rescore(const u64* __restrict__ cand,
                               const uint32_t* __restrict__ ncand_total, uint32_t cap,
                               const float* __restrict__ xs, uint64_t stride, int d,
                               const float* __restrict__ ccoord, const KcSeg* __restrict__ segs,
                               float* __restrict__ exm, uint32_t* __restrict__ exupto,
                               u64* __restrict__ part, int t)
{
    const int lane = threadIdx.x & 63;
    uint32_t nc = *ncand_total;
    if (nc > cap) nc = cap;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nc;
         q += waves) {
        const u64 e = cand[q];
        const uint32_t sidx = (uint32_t)(e >> 32), loc = (uint32_t)e;
        const KcSeg sg = segs[sidx];
        const uint64_t col = sg.base + loc;
        const uint32_t from = exupto[col];
        float best = exm[col];
        for (uint32_t j = from + lane; j <= (uint32_t)t; j += 64) {
            const float* cj = ccoord + (uint64_t)(sg.keyoff + j) * d;
            float s = 0.f;
            for (int u = 0; u < d; ++u) s = kc_d32_step(s, xs[(uint64_t)u * stride + col], cj[u]);
            best = fminf(best, s);
        }
        for (int off = 32; off >= 1; off >>= 1) best = fminf(best, __shfl_xor(best, off, 64));
        if (lane == 0) {
            exm[col] = best;
            exupto[col] = (uint32_t)t + 1;
            kc_part_offer(part, sg.keyoff + t, q % KC_PARTS, kc_pack(best, loc));
        }
    }
}

// Candidates and their rescoring in one pass over the step's tiles: a block
// whose largest upper bound is below L_t leaves at once; otherwise it lists
// its candidates in LDS, rescores each with one wave (lanes over the centers
// chosen since the point was last rescored) and offers the block's best key.
__global__ __launch_bounds__(KC_BLOCK) void k_bf16_cand_rescore(
    const float* __restrict__ mind, const float* __restrict__ ex,
    const float* __restrict__ blk_hi, const uint32_t* __restrict__ lpart,
    const float* __restrict__ xs, uint64_t stride, int d, const float* __restrict__ ccoord,
    const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, int t, float g, float* __restrict__ exm,
    uint32_t* __restrict__ exupto, u64* __restrict__ part)
{
    __shared__ uint32_t list[KC_BF_TILE];
    __shared__ uint32_t nlist;
    __shared__ float sL;
    __shared__ u64 red[KC_BLOCK / 64];
    const uint32_t b = blockIdx.x;
    const KcSeg sg = segs[blk_seg[b]];
    if ((uint32_t)t >= sg.ksteps) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (w == 0) {
        u64 pv = 1ull << 32;
        if (t > 0) {   // a segment that stopped at the previous step is done
            pv = 0;
            if (lane < KC_PARTS)
                pv = __hip_atomic_load(kc_part_slot(part, sg.keyoff + t - 1, lane),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            pv = kc_wave_max64(pv);
        }
        uint32_t lv = 0;
        if (lane < KC_PARTS)
            lv = __hip_atomic_load(lpart + ((uint64_t)(sg.keyoff + t) * KC_PARTS + lane) * 32,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int off = 32; off >= 1; off >>= 1) {
            const uint32_t o = __shfl_xor(lv, off, 64);
            lv = o > lv ? o : lv;
        }
        if (lane == 0) {
            // stopped segments and blocks without candidates skip the step
            sL = ((pv >> 32) == 0 || blk_hi[b] < __uint_as_float(lv)) ? -1.f
                                                                     : __uint_as_float(lv);
            nlist = 0;
        }
    }
    __syncthreads();
    const float L = sL;
    if (L < 0.f) return;
    for (int q = 0; q < KC_BF_PTS; ++q) {
        const uint32_t loc = blk_start[b] + q * KC_BLOCK + threadIdx.x;
        if (loc < sg.len) {
            const uint64_t col = sg.base + loc;
            if (kc_bf_hi(mind[col], ex[col], g) >= L) list[atomicAdd(&nlist, 1u)] = loc;
        }
    }
    __syncthreads();
    const uint32_t nl = nlist;
    u64 key = 0;
    for (uint32_t q = w; q < nl; q += KC_BLOCK / 64) {
        const uint32_t loc = list[q];
        const uint64_t col = sg.base + loc;
        const uint32_t from = exupto[col];
        float best = exm[col];
        for (uint32_t j = from + lane; j <= (uint32_t)t; j += 64) {
            const float* cj = ccoord + (uint64_t)(sg.keyoff + j) * d;
            float s = 0.f;
            for (int u = 0; u < d; ++u) s = kc_d32_step(s, xs[(uint64_t)u * stride + col], cj[u]);
            best = fminf(best, s);
        }
        for (int off = 32; off >= 1; off >>= 1) best = fminf(best, __shfl_xor(best, off, 64));
        if (lane == 0) {
            exm[col] = best;
            exupto[col] = (uint32_t)t + 1;
        }
        key = kc_umax64(key, kc_pack(best, loc));
    }
    key = kc_block_max64(key, red);
    if (threadIdx.x == 0 && key) kc_part_offer(part, sg.keyoff + t, b % KC_PARTS, key);
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

#define KC_BF_CASE(DD)                                                                   \
    case DD:                                                                             \
        hipLaunchKernelGGL(k_gon_step_bf16<DD>, dim3(R.nblk), dim3(KC_BLOCK), 0, s, B.xb, \
                           R.xs, R.stride, R.d, B.ex, R.mind, R.part, B.lpart, B.blk_hi,  \
                           R.ccoord, R.segs, R.blk_seg, R.blk_start, t, B.g);             \
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
                               R.xs, R.stride, R.d, B.ex, R.mind, R.part, B.lpart, B.blk_hi,
                               R.ccoord, R.segs, R.blk_seg, R.blk_start, t, B.g);
        }
        hipLaunchKernelGGL(k_bf16_cand_rescore, dim3(R.nblk), dim3(KC_BLOCK), 0, s, R.mind,
                           B.ex, B.blk_hi, B.lpart, R.xs, R.stride, R.d, R.ccoord, R.segs,
                           R.blk_seg, R.blk_start, t, B.g, B.exm, B.exupto, R.part);
    }
    kc_part_collect(R.part, R.keys, R.keysum, s);
}

void kc_enqueue_bf16_prep(const KcGonRun& R, const KcBf16Run& B, const KcGonHost& H,
                          const std::vector<KcGonJob>& jobs, hipStream_t s)
{
    for (size_t q = 0; q < jobs.size(); ++q) {
        kc_stage_soa(jobs[q].X, jobs[q].ld, R.d, jobs[q].row0, jobs[q].len, (float*)R.xs,
                     R.stride, H.segs[q].base, s);
        kc_stage_bf16(jobs[q].X, jobs[q].Xb, jobs[q].ld, R.d, jobs[q].row0, jobs[q].len, B.xb,
                      B.ex, R.stride, H.segs[q].base, s);
    }
    kc_fill_u32((uint32_t*)R.mind, 0x7F800000u, R.stride, s);   // +inf
    kc_fill_u32((uint32_t*)B.exm, 0x7F800000u, R.stride, s);
    kc_fill_u32(B.exupto, 0u, R.stride, s);
    kc_fill_u64(R.part, 0ull, R.keysum * KC_PARTS * KC_PSTRIDE, s);
    kc_fill_u32(B.lpart, 0u, R.keysum * KC_PARTS * 32, s);
    kc_fill_u32(B.ncand, 0u, R.kmax, s);
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
