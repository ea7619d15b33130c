// kc_assign.hip -- nearest-center distances on MFMA with certified results.
//
// k_mindist_mfma computes, for every point x and a set of "centers" c_i,
//     v_i = |c_i|^2 - 2 x.c_i        (the dot products on MFMA)
// and keeps per point the smallest v (with its lowest center index) and the
// second smallest; |x|^2 is added afterwards.  The contraction is
//     C (16 centers x K) * X^T (K x 16 points)  -> 16 x 16 accumulators,
// so every lane ends up holding one point and four centers of each tile, and
// the per-point minimum needs one merge over the four lanes sharing a point.
// FP32 inputs use v_mfma_f32_16x16x4f32 (K = 4 per instruction), BF16 inputs
// v_mfma_f32_16x16x32_bf16 (K = 32), both accumulating in FP32.  Centers are
// staged through LDS in chunks; points stream from the caller's array.
//
// Certification (used by the assignment and by EIM's distance pass): with
//     g = (6d + 32) u,  err = g (|x| + max_i |c_i|)^2
// every exact squared distance lies within err of |x|^2 + v_i (BF16 inputs
// add the rounding radius E = e_x + max e_c in the square-root domain).  A
// point whose second-best lower bound exceeds its best upper bound has a
// certified nearest center; every other point is rescored exactly in FP64.
#include "kc_device.h"
#include "kc_internal.h"

typedef float kc_v4f __attribute__((ext_vector_type(4)));
typedef __bf16 kc_v8bf __attribute__((ext_vector_type(8)));

struct KcBest {
    float m1;
    int a1;
    float m2;
};

__device__ __forceinline__ void kc_best_push(KcBest& b, float v, int idx)
{
    // centers arrive in ascending index order per lane: strict < keeps the
    // lower index on ties, and a tie leaves m2 == m1 (ambiguous)
    if (v < b.m1) {
        b.m2 = b.m1;
        b.m1 = v;
        b.a1 = idx;
    } else {
        b.m2 = fminf(b.m2, v);
    }
}

__device__ __forceinline__ KcBest kc_best_merge(KcBest a, KcBest o)
{
    const bool take_o = (o.m1 < a.m1) || (o.m1 == a.m1 && o.a1 < a.a1);
    KcBest r;
    if (take_o) {
        r.m1 = o.m1;
        r.a1 = o.a1;
        r.m2 = fminf(o.m2, a.m1);
    } else {
        r.m1 = a.m1;
        r.a1 = a.a1;
        r.m2 = fminf(a.m2, o.m1);
    }
    return r;
}

__device__ __forceinline__ KcBest kc_best_xor(KcBest b, int mask)
{
    KcBest o;
    o.m1 = __shfl_xor(b.m1, mask, 64);
    o.a1 = __shfl_xor(b.a1, mask, 64);
    o.m2 = __shfl_xor(b.m2, mask, 64);
    return kc_best_merge(b, o);
}

__device__ __forceinline__ float kc_bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

#define KC_MD_WAVES 4
// Point tiles (16 points each) per wave: four where the B operand is small
// (more independent MFMA chains per center tile, fewer A reads per point),
// two where it would crowd the VGPRs.
__host__ __device__ constexpr int kc_md_pt(bool bf, int ks)
{
    return (!bf && ks <= 8) || (bf && ks <= 2) ? 4 : 2;
}

// BF: BF16 inputs.  KS: MFMA K-steps (K = 4*KS for FP32, 32*KS for BF16).
// LAB: keep the best index and the second-best value (labels need them);
// without it only the smallest value per point is kept (a covering radius or
// a distance to a set needs nothing else), and out_arg / out_m2 are unused.
template <bool BF, int KS, bool LAB>
__global__ __launch_bounds__(KC_MD_WAVES * 64) void k_mindist_mfma(
    const float* __restrict__ X, const uint16_t* __restrict__ Xb, int64_t ld, uint32_t n,
    int d, const float* __restrict__ Cf, const uint16_t* __restrict__ Cb,
    const float* __restrict__ cnorm, uint32_t kpad, uint32_t chunk,
    int32_t* __restrict__ out_arg, float* __restrict__ out_m1, float* __restrict__ out_m2,
    float* __restrict__ out_nx)
{
    constexpr int DP = BF ? KS * 32 : KS * 4;   // padded K
    constexpr int KC_MD_PT = kc_md_pt(BF, KS);
    extern __shared__ __align__(16) unsigned char kc_smem[];
    float* s_norm = (float*)kc_smem;                          // [chunk]
    void* s_c = (void*)(kc_smem + sizeof(float) * chunk);     // [chunk][DP]

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const uint64_t p0 =
        ((uint64_t)blockIdx.x * KC_MD_WAVES + wave) * (16 * KC_MD_PT);

    // B operand (points) for all point tiles and K-steps, kept in registers
    float bf[KC_MD_PT][BF ? 1 : KS];
    kc_v8bf bb[KC_MD_PT][BF ? KS : 1];
    float nxp[KC_MD_PT];
#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        const uint64_t p = p0 + pt * 16 + col;
        const bool ok = p < n;
        nxp[pt] = 0.f;
        if (!BF) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kk = ks * 4 + grp;
                float v = (ok && kk < d) ? X[p * ld + kk] : 0.f;
                bf[pt][BF ? 0 : ks] = v;
                nxp[pt] = __builtin_fmaf(v, v, nxp[pt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kc_v8bf w;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = ks * 32 + grp * 8 + e;
                    const uint16_t h = (ok && kk < d) ? Xb[p * ld + kk] : (uint16_t)0;
                    const float f = kc_bf16_to_f32(h);
                    w[e] = (__bf16)f;
                    nxp[pt] = __builtin_fmaf(f, f, nxp[pt]);
                }
                bb[pt][BF ? ks : 0] = w;
            }
        }
    }

    KcBest best[KC_MD_PT];
#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        best[pt].m1 = __builtin_inff();
        best[pt].m2 = __builtin_inff();
        best[pt].a1 = 0x7FFFFFFF;
    }

    for (uint32_t c0 = 0; c0 < kpad; c0 += chunk) {
        const uint32_t cn = min(chunk, kpad - c0);
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < cn; q += blockDim.x) s_norm[q] = cnorm[c0 + q];
        if (!BF) {
            const float4* src = (const float4*)(Cf + (uint64_t)c0 * DP);
            float4* dst = (float4*)s_c;
            for (uint32_t q = threadIdx.x; q < cn * DP / 4; q += blockDim.x) dst[q] = src[q];
        } else {
            const uint4* src = (const uint4*)(Cb + (uint64_t)c0 * DP);
            uint4* dst = (uint4*)s_c;
            for (uint32_t q = threadIdx.x; q < cn * DP / 8; q += blockDim.x) dst[q] = src[q];
        }
        __syncthreads();

        for (uint32_t ct = 0; ct < cn; ct += 16) {
            // A operand: centers ct + col, K slice of this lane group
            float af[BF ? 1 : KS];
            kc_v8bf ab[BF ? KS : 1];
            if (!BF) {
                const float* cs = (const float*)s_c + (uint64_t)(ct + col) * DP;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) af[BF ? 0 : ks] = cs[ks * 4 + grp];
            } else {
                const uint16_t* cs = (const uint16_t*)s_c + (uint64_t)(ct + col) * DP;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    ab[BF ? ks : 0] = *(const kc_v8bf*)(cs + ks * 32 + grp * 8);
            }
            const float4 nc4 = *(const float4*)(s_norm + ct + grp * 4);
#pragma unroll
            for (int pt = 0; pt < KC_MD_PT; ++pt) {
                kc_v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    if (!BF)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[BF ? 0 : ks],
                                                                   bf[pt][BF ? 0 : ks], acc,
                                                                   0, 0, 0);
                    else
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[BF ? ks : 0],
                                                                      bb[pt][BF ? ks : 0],
                                                                      acc, 0, 0, 0);
                }
                if (LAB) {
                    const int ib = (int)(c0 + ct) + grp * 4;
                    kc_best_push(best[pt], __builtin_fmaf(-2.f, acc[0], nc4.x), ib + 0);
                    kc_best_push(best[pt], __builtin_fmaf(-2.f, acc[1], nc4.y), ib + 1);
                    kc_best_push(best[pt], __builtin_fmaf(-2.f, acc[2], nc4.z), ib + 2);
                    kc_best_push(best[pt], __builtin_fmaf(-2.f, acc[3], nc4.w), ib + 3);
                } else {
                    // padding centers have norm +inf, so they never win
                    float v = fminf(__builtin_fmaf(-2.f, acc[0], nc4.x),
                                    __builtin_fmaf(-2.f, acc[1], nc4.y));
                    v = fminf(v, fminf(__builtin_fmaf(-2.f, acc[2], nc4.z),
                                       __builtin_fmaf(-2.f, acc[3], nc4.w)));
                    best[pt].m1 = fminf(best[pt].m1, v);
                }
            }
        }
    }

#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        KcBest b = best[pt];
        if (LAB) {
            b = kc_best_xor(b, 16);
            b = kc_best_xor(b, 32);
        } else {
            b.m1 = fminf(b.m1, __shfl_xor(b.m1, 16, 64));
            b.m1 = fminf(b.m1, __shfl_xor(b.m1, 32, 64));
        }
        float nx = nxp[pt];
        nx += __shfl_xor(nx, 16, 64);
        nx += __shfl_xor(nx, 32, 64);
        const uint64_t p = p0 + pt * 16 + col;
        if (grp == 0 && p < n) {
            if (LAB) {
                out_arg[p] = b.a1;
                out_m2[p] = b.m2;
            }
            out_m1[p] = b.m1;
            out_nx[p] = nx;
        }
    }
}

// ---------------------------------------------------------------------------
// center staging: compact FP32 / BF16 rows [kpad][DP], norms (+inf padding),
// and the maxima |c| and e_c used by the error bound.

__global__ void k_stage_centers(const float* __restrict__ X, const uint16_t* __restrict__ Xb,
                                int64_t ld, int d, uint32_t n, const int64_t* __restrict__ idx,
                                const uint32_t* __restrict__ idx32, uint32_t k,
                                const int64_t* __restrict__ k_dev, uint32_t kpad, int dp,
                                float* __restrict__ Cf, uint16_t* __restrict__ Cb,
                                float* __restrict__ cnorm, float* __restrict__ cmax,
                                uint32_t* __restrict__ status)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kpad) return;
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    int64_t ri = 0;
    if (i < k) {
        ri = idx ? idx[i] : (int64_t)idx32[i];
        if (ri < 0 || ri >= (int64_t)n) {   // invalid index: report, stay in bounds
            atomicOr(status, 4u);
            ri = 0;
        }
    }
    if (i >= k) {
        for (int j = 0; j < dp; ++j) {
            if (Cf) Cf[(uint64_t)i * dp + j] = 0.f;
            if (Cb) Cb[(uint64_t)i * dp + j] = 0;
        }
        cnorm[i] = __builtin_inff();
        return;
    }
    const uint64_t r = (uint64_t)ri;
    double nn = 0.0, ee = 0.0;
    float nf = 0.f;
    for (int j = 0; j < dp; ++j) {
        const float v = j < d ? X[r * ld + j] : 0.f;
        if (Cf) Cf[(uint64_t)i * dp + j] = v;
        if (Cb) {
            const uint16_t h = j < d ? Xb[r * ld + j] : (uint16_t)0;
            Cb[(uint64_t)i * dp + j] = h;
            const float f = kc_bf16_to_f32(h);
            nf = __builtin_fmaf(f, f, nf);
            const double e = (double)f - (double)v;
            ee += e * e;
        }
        nn += (double)v * (double)v;
    }
    // norm used in v_i: of the values fed to the MFMA
    cnorm[i] = Cb ? nf : (float)nn;
    const float len = Cb ? sqrtf(nf) : (float)sqrt(nn);
    kc_atomic_max_f32_nonneg(&cmax[0], len * (1.f + 1e-6f));
    if (Cb) kc_atomic_max_f32_nonneg(&cmax[1], (float)(sqrt(ee) * (1.0 + 1e-12)) * (1.f + 1e-6f));
}

// Per-point BF16 rounding radius e_x = |bf16(x) - x| (FP64, rounded up).
__global__ void k_bf16_err(const float* __restrict__ X, const uint16_t* __restrict__ Xb,
                           int64_t ld, int d, uint32_t n, float* __restrict__ ex)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double ee = 0.0;
    for (int j = 0; j < d; ++j) {
        const double e = (double)kc_bf16_to_f32(Xb[(uint64_t)p * ld + j]) -
                         (double)X[(uint64_t)p * ld + j];
        ee += e * e;
    }
    ex[p] = (float)(sqrt(ee) * (1.0 + 1e-12)) * (1.f + 1e-6f);
}

// ---------------------------------------------------------------------------
// assignment epilogue: certify, collect ambiguous points, radius lower bound

__device__ __forceinline__ double kc_lo_bound(double v, double err, double E)
{
    double a = v - err;
    if (a < 0.0) a = 0.0;
    double r = sqrt(a) - E;
    if (r < 0.0) r = 0.0;
    return r * r * (1.0 - 1e-12);
}
__device__ __forceinline__ double kc_hi_bound(double v, double err, double E)
{
    const double r = sqrt(v + err) + E;
    return r * r * (1.0 + 1e-12);
}

// Append `val` to list for every lane whose `pred` holds, one atomic per
// wave.  All 64 lanes must call it together.
__device__ __forceinline__ void kc_wave_append(bool pred, uint32_t val, uint32_t* list,
                                               uint32_t* nlist)
{
    const u64 b = __ballot(pred);
    if (b == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(b);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(nlist, (uint32_t)__builtin_popcountll(b));
    base = (uint32_t)__shfl((int)base, leader, 64);
    if (pred) list[base + (uint32_t)__builtin_popcountll(b & ((1ull << lane) - 1ull))] = val;
}

// With labels == NULL only the radius is wanted: an ambiguous point matters
// only if its upper bound reaches the largest lower bound, and
// k_radius_candidates lists exactly those, so ambiguity lists nothing.
__global__ void k_assign_epilogue(uint32_t n, int d, const int32_t* __restrict__ arg,
                                  const float* __restrict__ m1, const float* __restrict__ m2,
                                  const float* __restrict__ nxv, const float* __restrict__ ex,
                                  const float* __restrict__ cmax, int32_t* __restrict__ labels,
                                  float* __restrict__ hi_out, uint32_t* __restrict__ list,
                                  uint32_t* __restrict__ nlist, float* __restrict__ lo_max)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    float lo_f = 0.f;
    bool amb = false;
    if (p < n) {
        const double g = (6.0 * d + 32.0) * 5.9604644775390625e-8;
        const double nx = nxv[p];
        const double xl = sqrt(nx) * (1.0 + 1e-6);
        const double s = xl + (double)cmax[0];
        const double err = g * s * s + 1e-30 * d;
        const double E = ex ? (double)ex[p] + (double)cmax[1] : 0.0;
        const double d1 = nx + (double)m1[p];
        const double hi1 = kc_hi_bound(d1, err, E);
        const double lo1 = kc_lo_bound(d1, err, E);
        if (labels) {
            const double d2 = nx + (double)m2[p];
            const double lo2 = kc_lo_bound(d2, err, E);
            amb = !(lo2 > hi1);
            labels[p] = amb ? -1 : arg[p];
        }
        hi_out[p] = (float)hi1 * (1.f + 1e-6f);
        lo_f = (float)lo1 * (1.f - 1e-6f);
    }
    kc_wave_append(amb, p, list, nlist);
    // block max of the lower bounds, one atomic per block
    __shared__ float red[4];
    float v = lo_f;
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
        // tens of thousands of blocks meet at one word: skip the atomic when
        // the word already holds as much (a stale read is never larger)
        const float cur = __uint_as_float(__hip_atomic_load(
            (const uint32_t*)lo_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (r > cur) kc_atomic_max_f32_nonneg(lo_max, r);
    }
}

// points whose upper bound reaches the largest lower bound may attain the
// covering radius: rescore them too
__global__ void k_radius_candidates(uint32_t n, const float* __restrict__ hi,
                                    const float* __restrict__ lo_max,
                                    uint32_t* __restrict__ list, uint32_t* __restrict__ nlist)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const float L = *lo_max;
    kc_wave_append(p < n && hi[p] >= L, p, list, nlist);
}

// One wave per listed point: exact FP64 nearest center (lowest position on
// ties) over all k centers; label and radius^2 (as bits of a double).
__global__ void k_rescore_f64(const float* __restrict__ X, int64_t ld, int d,
                              const float* __restrict__ Cf, int dp, uint32_t k,
                              const int64_t* __restrict__ k_dev,
                              const uint32_t* __restrict__ list,
                              const uint32_t* __restrict__ nlist, uint32_t cap,
                              int32_t* __restrict__ labels, double* __restrict__ radius2)
{
    const int lane = threadIdx.x & 63;
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    uint32_t nl = *nlist;
    if (nl > cap) nl = cap;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nl; q += waves) {
        const uint64_t p = list[q];
        const float* xp = X + p * ld;
        double best = __builtin_inf();
        int bj = 0x7FFFFFFF;
        for (uint32_t j = lane; j < k; j += 64) {
            const float* cj = Cf + (uint64_t)j * dp;
            double s = 0.0;
            for (int u = 0; u < d; ++u) s = kc_d64_step(s, (double)xp[u], (double)cj[u]);
            if (s < best) {
                best = s;
                bj = (int)j;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oj = __shfl_xor(bj, off, 64);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (lane == 0) {
            if (labels) labels[p] = bj;
            kc_atomic_max_f64_nonneg(radius2, best);
        }
    }
}

// Covering radius only, small d: the canonical FP32 distance to every
// center (one lane per point, coordinates in VGPRs, the centers streamed
// through LDS).  Its relative error is at most g = gamma_{d+2}, so the
// exact min-distance lies in [m / (1 + g), m / (1 - g)] around the smallest
// FP32 value m (widened for rounding and for squares that underflow): far
// tighter than the MFMA bound, whose error scales with the norms, so only
// a handful of points reach the largest lower bound and go to the exact
// FP64 pass.  Writes hi_out[p] and the maximum lower bound into lo_max.
#define KC_RD_MAXD 8
#define KC_RD_CHUNK 1024
template <int D>
__global__ __launch_bounds__(256) void k_radius_direct(const float* __restrict__ X, int64_t ld,
                                                       uint32_t n, const float* __restrict__ Cf,
                                                       int dp, uint32_t k,
                                                       const int64_t* __restrict__ k_dev,
                                                       double g, float* __restrict__ hi_out,
                                                       float* __restrict__ lo_max)
{
    __shared__ float sC[KC_RD_CHUNK * D];
    __shared__ float red[4];
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < n;
    float xc[D];
#pragma unroll
    for (int u = 0; u < D; ++u) xc[u] = live ? X[(uint64_t)p * ld + u] : 0.f;
    float m = __builtin_inff();
    for (uint32_t j0 = 0; j0 < k; j0 += KC_RD_CHUNK) {
        const uint32_t cnt = min((uint32_t)KC_RD_CHUNK, k - j0);
        __syncthreads();
        for (uint32_t e0 = threadIdx.x; e0 < cnt * D; e0 += 8 * blockDim.x) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t e = e0 + q * blockDim.x, r = e / D, u = e - r * D;
                v[q] = e < cnt * D ? Cf[(uint64_t)(j0 + r) * dp + u] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t e = e0 + q * blockDim.x;
                if (e < cnt * D) sC[e] = v[q];
            }
        }
        __syncthreads();
        for (uint32_t r = 0; r < cnt; ++r) {
            float a = 0.f;
#pragma unroll
            for (int u = 0; u < D; ++u) a = kc_d32_step(a, xc[u], sC[r * D + u]);
            m = fminf(m, a);
        }
    }
    float lo_f = 0.f;
    if (live) {
        const double mv = (double)m;
        double l = mv / (1.0 + g) - 1e-37 * D;
        if (l < 0.0) l = 0.0;
        const double u = mv / (1.0 - g) + 1e-37 * D;
        hi_out[p] = (float)u * (1.f + 1e-6f);
        lo_f = (float)l * (1.f - 1e-6f);
    }
    float v = lo_f;
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
        const float cur = __uint_as_float(__hip_atomic_load(
            (const uint32_t*)lo_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (r > cur) kc_atomic_max_f32_nonneg(lo_max, r);
    }
}

__global__ void k_sqrt_out(const double* __restrict__ r2, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = kc_sqrt_rn(*r2);
}

// ---------------------------------------------------------------------------
// host launchers

#define KC_MD_CASES_F32(X) X(1) X(2) X(3) X(4) X(8) X(11) X(16) X(32) X(64)
#define KC_MD_CASES_BF16(X) X(1) X(2) X(4) X(8)

int kc_mindist_ksteps(int d, bool bf)
{
    if (bf) {
        const int ks = (d + 31) / 32;
        if (ks <= 1) return 1;
        if (ks <= 2) return 2;
        if (ks <= 4) return 4;
        return 8;
    }
    const int ks = (d + 3) / 4;
    const int opts[] = {1, 2, 3, 4, 8, 11, 16, 32, 64};
    for (int o : opts)
        if (ks <= o) return o;
    return 64;
}

int kc_mindist_dpad(int d, bool bf)
{
    return bf ? kc_mindist_ksteps(d, true) * 32 : kc_mindist_ksteps(d, false) * 4;
}

// Largest center chunk (multiple of 16) whose LDS copy fits in 64 KiB.
uint32_t kc_mindist_chunk(int d, bool bf, uint32_t kpad)
{
    const uint32_t dp = (uint32_t)kc_mindist_dpad(d, bf);
    const uint32_t per = dp * (bf ? 2 : 4) + 4;
    uint32_t c = (64u * 1024u / per) & ~15u;
    if (c < 16) c = 16;
    return c < kpad ? c : kpad;
}

void kc_mindist(const float* X, const uint16_t* Xb, int64_t ld, uint32_t n, int d,
                const float* Cf, const uint16_t* Cb, const float* cnorm, uint32_t kpad,
                int32_t* arg, float* m1, float* m2, float* nx, hipStream_t s)
{
    const bool lab = arg != nullptr;
    const bool bf = Xb != nullptr;
    const int ks = kc_mindist_ksteps(d, bf);
    const uint32_t chunk = kc_mindist_chunk(d, bf, kpad);
    const int dp = kc_mindist_dpad(d, bf);
    const size_t smem = (size_t)chunk * 4 + (size_t)chunk * dp * (bf ? 2 : 4);
    const uint32_t per_block = KC_MD_WAVES * 16 * kc_md_pt(bf, ks);
    const dim3 grid((n + per_block - 1) / per_block), block(KC_MD_WAVES * 64);
    if (!bf) {
        switch (ks) {
#define KC_CASE(K)                                                                       \
    case K:                                                                              \
        if (lab)                                                                         \
            hipLaunchKernelGGL((k_mindist_mfma<false, K, true>), grid, block, smem, s, X, \
                               Xb, ld, n, d, Cf, Cb, cnorm, kpad, chunk, arg, m1, m2, nx); \
        else                                                                             \
            hipLaunchKernelGGL((k_mindist_mfma<false, K, false>), grid, block, smem, s, X, \
                               Xb, ld, n, d, Cf, Cb, cnorm, kpad, chunk, arg, m1, m2, nx); \
        break;
            KC_MD_CASES_F32(KC_CASE)
#undef KC_CASE
        }
    } else {
        switch (ks) {
#define KC_CASE(K)                                                                       \
    case K:                                                                              \
        if (lab)                                                                         \
            hipLaunchKernelGGL((k_mindist_mfma<true, K, true>), grid, block, smem, s, X,  \
                               Xb, ld, n, d, Cf, Cb, cnorm, kpad, chunk, arg, m1, m2, nx); \
        else                                                                             \
            hipLaunchKernelGGL((k_mindist_mfma<true, K, false>), grid, block, smem, s, X, \
                               Xb, ld, n, d, Cf, Cb, cnorm, kpad, chunk, arg, m1, m2, nx); \
        break;
            KC_MD_CASES_BF16(KC_CASE)
#undef KC_CASE
        }
    }
}

void kc_stage_centers(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n,
                      const int64_t* idx, const uint32_t* idx32, uint32_t k,
                      const int64_t* k_dev, uint32_t kpad, int dp, float* Cf, uint16_t* Cb,
                      float* cnorm, float* cmax, uint32_t* status, hipStream_t s)
{
    kc_fill_u32((uint32_t*)cmax, 0u, 2, s);
    hipLaunchKernelGGL(k_stage_centers, dim3((kpad + 255) / 256), dim3(256), 0, s, X, Xb, ld, d,
                       n, idx, idx32, k, k_dev, kpad, dp, Cf, Cb, cnorm, cmax, status);
}

void kc_bf16_err(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n, float* ex,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_bf16_err, dim3((n + 255) / 256), dim3(256), 0, s, X, Xb, ld, d, n, ex);
}

bool kc_radius_direct(uint32_t n, int d, const float* X, int64_t ld, const float* Cf, int dp,
                      uint32_t k, const int64_t* k_dev, float* hi, uint32_t* list,
                      uint32_t* nlist, float* lo_max, double* radius2, double* radius_out,
                      hipStream_t s)
{
    if (d < 1 || d > KC_RD_MAXD) return false;
    const double u32 = 5.9604644775390625e-8, m = d + 2;
    const double g = m * u32 / (1.0 - m * u32);
    kc_fill_u32(nlist, 0u, 1, s);
    kc_fill_u32((uint32_t*)lo_max, 0u, 1, s);
    kc_fill_u64((u64*)radius2, 0ull, 1, s);
    const dim3 gr((n + 255) / 256);
    switch (d) {
#define KC_RD_CASE(DD)                                                                      \
    case DD:                                                                                \
        hipLaunchKernelGGL(k_radius_direct<DD>, gr, dim3(256), 0, s, X, ld, n, Cf, dp, k,    \
                           k_dev, g, hi, lo_max);                                           \
        break;
        KC_RD_CASE(1)
        KC_RD_CASE(2)
        KC_RD_CASE(3)
        KC_RD_CASE(4)
        KC_RD_CASE(5)
        KC_RD_CASE(6)
        KC_RD_CASE(7)
        KC_RD_CASE(8)
#undef KC_RD_CASE
    }
    hipLaunchKernelGGL(k_radius_candidates, gr, dim3(256), 0, s, n, hi, lo_max, list, nlist);
    hipLaunchKernelGGL(k_rescore_f64, dim3(2048), dim3(256), 0, s, X, ld, d, Cf, dp, k, k_dev,
                       list, nlist, 2 * n, nullptr, radius2);
    hipLaunchKernelGGL(k_sqrt_out, dim3(1), dim3(64), 0, s, radius2, radius_out);
    return true;
}

void kc_assign_finish(uint32_t n, int d, const float* X, int64_t ld, const float* Cf, int dp,
                      uint32_t k, const int64_t* k_dev, const int32_t* arg, const float* m1,
                      const float* m2, const float* nx, const float* ex, const float* cmax,
                      int32_t* labels, float* hi, uint32_t* list, uint32_t* nlist,
                      float* lo_max, double* radius2, double* radius_out, hipStream_t s)
{
    kc_fill_u32(nlist, 0u, 1, s);
    kc_fill_u32((uint32_t*)lo_max, 0u, 1, s);
    kc_fill_u64((u64*)radius2, 0ull, 1, s);
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(k_assign_epilogue, g, dim3(256), 0, s, n, d, arg, m1, m2, nx, ex, cmax,
                       labels, hi, list, nlist, lo_max);
    hipLaunchKernelGGL(k_radius_candidates, g, dim3(256), 0, s, n, hi, lo_max, list, nlist);
    hipLaunchKernelGGL(k_rescore_f64, dim3(2048), dim3(256), 0, s, X, ld, d, Cf, dp, k, k_dev,
                       list, nlist, 2 * n, labels, radius2);
    hipLaunchKernelGGL(k_sqrt_out, dim3(1), dim3(64), 0, s, radius2, radius_out);
}
