// kc_eim.hip -- the EIM sampling pass (Algorithm 2 with Select, Algorithm 3,
// and the Section 4.1 changes) on gfx950, followed by Gonzalez on the sample.
//
// Per iteration (host-driven, one synchronisation to size the next one):
//   k_eim_draw        Philox4x64-10 Bernoulli draws for every x in R: into
//                     S with probability p_S, into H with probability p_H
//                     (one counter-based block per point and iteration);
//   compaction        stable scans split R into dS (new samples), H and the
//                     points that stay candidates (not sampled);
//   k_eim_dist_h      exact FP64 d(h,S)^2 for h in H (split over S, min via
//                     64-bit atomics on the bits of non-negative doubles);
//   k_eim_select      tau = the min(r,|H|)-th largest d(h,S)^2 (rank count);
//   distance pass     d(x,dS)^2 for the remaining x on MFMA; per point the
//                     certified interval [lo, hi] of d(x,S)^2 is narrowed by
//                     a running min over the iterations;
//   k_eim_decide      keep x iff d(x,S)^2 > tau: decided by the interval when
//                     it does not contain tau, otherwise in exact FP64 over
//                     all of S (k_eim_exact).
// Every draw and decision is per point, so the result is independent of how
// the paper's mappers partition R.
#include <math.h>
#include <string.h>

#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "kc_host.h"

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// products with the published multipliers; the key advances by the published
// Weyl constants between rounds.

__device__ __forceinline__ void kc_philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// flags: bit 0 = drawn into S, bit 1 = drawn into H
__global__ void k_eim_draw(const uint32_t* __restrict__ R, uint32_t nr, uint64_t seed, int it,
                           double pS, double pH, uint8_t* __restrict__ fS,
                           uint8_t* __restrict__ fH, uint8_t* __restrict__ fKeep)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nr) return;
    uint64_t c[4] = {(uint64_t)R[j], (uint64_t)it, 0ull, 0ull};
    kc_philox4x64_10(c, seed, 0ull);
    const double uS = (double)(c[0] >> 11) * 0x1.0p-53;
    const double uH = (double)(c[1] >> 11) * 0x1.0p-53;
    const bool s = uS < pS;
    fS[j] = s;
    fH[j] = uH < pH;
    fKeep[j] = !s;   // sampled points always leave R
}

// ---------------------------------------------------------------------------
// stable compaction: out[rank] = in[i] (or i) for every flagged i, in order

#define KC_CMP_ITEMS 1024   // items per block (256 threads x 4)

__global__ void k_cmp_count(const uint8_t* __restrict__ f, uint32_t n,
                            uint32_t* __restrict__ blk_cnt)
{
    __shared__ uint32_t red[4];
    const uint32_t base = blockIdx.x * KC_CMP_ITEMS;
    uint32_t c = 0;
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        if (i < n) c += f[i] != 0;
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// one block: exclusive scan of nb block counts; total -> *count
__global__ void k_cmp_scan(uint32_t* __restrict__ blk, uint32_t nb, uint32_t* __restrict__ count)
{
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[16];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? blk[i] : 0u;
        // inclusive scan within the wave
        uint32_t x = v;
        const int lane = threadIdx.x & 63;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[threadIdx.x >> 6] = x;
        __syncthreads();
        uint32_t wpre = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wpre += wsum[w];
        const uint32_t excl = carry + wpre + x - v;
        __syncthreads();
        if (i < nb) blk[i] = excl;
        if (threadIdx.x == blockDim.x - 1) carry = excl + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

__global__ void k_cmp_scatter(const uint8_t* __restrict__ f, const uint32_t* __restrict__ in,
                              uint32_t n, const uint32_t* __restrict__ blk_off,
                              uint32_t* __restrict__ out)
{
    __shared__ uint32_t wcnt[16];
    const uint32_t base = blockIdx.x * KC_CMP_ITEMS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t run = blk_off[blockIdx.x];
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        const bool on = i < n && f[i] != 0;
        const u64 mask = __ballot(on);
        const uint32_t before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[w] = __popcll(mask);
        __syncthreads();
        uint32_t wpre = 0;
        for (int v = 0; v < w; ++v) wpre += wcnt[v];
        if (on) out[run + wpre + before] = in ? in[i] : i;
        uint32_t tot = 0;
        for (int v = 0; v < 4; ++v) tot += wcnt[v];
        __syncthreads();
        run += tot;
    }
}

struct KcCompact {
    uint32_t* blk = nullptr;   // [nblocks]
    uint32_t nb_cap = 0;
};

static void kc_compact(const KcCompact& C, const uint8_t* f, const uint32_t* in, uint32_t n,
                       uint32_t* out, uint32_t* count, hipStream_t s)
{
    if (n == 0) {
        kc_fill_u32(count, 0u, 1, s);
        return;
    }
    const uint32_t nb = (n + KC_CMP_ITEMS - 1) / KC_CMP_ITEMS;
    hipLaunchKernelGGL(k_cmp_count, dim3(nb), dim3(256), 0, s, f, n, C.blk);
    hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(1024), 0, s, C.blk, nb, count);
    hipLaunchKernelGGL(k_cmp_scatter, dim3(nb), dim3(256), 0, s, f, in, n, C.blk, out);
}

// ---------------------------------------------------------------------------
// Select (Algorithm 3): d(h,S)^2 for h in H exactly, then tau

// grid.x covers H, grid.y splits S; one wave per (h, slice)
__global__ void k_eim_dist_h(const float* __restrict__ X, int64_t ld, int d,
                             const uint32_t* __restrict__ H, uint32_t nh,
                             const uint32_t* __restrict__ S, uint32_t ns,
                             double* __restrict__ dH)
{
    const uint32_t h = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (h >= nh) return;
    const float* xh = X + (uint64_t)H[h] * ld;
    const uint32_t per = (ns + gridDim.y - 1) / gridDim.y;
    const uint32_t s0 = blockIdx.y * per, s1 = min(ns, s0 + per);
    double best = __builtin_inf();
    for (uint32_t q = s0 + lane; q < s1; q += 64) {
        const float* xs = X + (uint64_t)S[q] * ld;
        double a = 0.0;
        for (int u = 0; u < d; ++u) a = kc_d64_step(a, (double)xh[u], (double)xs[u]);
        best = fmin(best, a);
    }
    best = kc_wave_min_f64(best);
    if (lane == 0 && best < __builtin_inf())
        atomicMin((u64*)&dH[h], (u64)__double_as_longlong(best));
}

// tau = the r-th largest of dH[0..nh) (rank by counting; ties share a value)
__global__ void k_eim_select(const double* __restrict__ dH, uint32_t nh, uint32_t r,
                             double* __restrict__ tau)
{
    for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) {
        const double v = dH[i];
        uint32_t greater = 0, equal = 0;
        for (uint32_t j = 0; j < nh; ++j) {
            greater += dH[j] > v;
            equal += dH[j] == v;
        }
        if (greater < r && r <= greater + equal) *tau = v;   // all writers agree
    }
}

// ---------------------------------------------------------------------------
// distance pass bounds and the keep decision

// XR[j][*] = X[R[j]][*] for the candidates (compact AoS, row stride d)
__global__ void k_gather_rows(const float* __restrict__ X, int64_t ld, int d,
                              const uint32_t* __restrict__ idx, uint32_t n,
                              float* __restrict__ out)
{
    const uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (q >= (uint64_t)n * d) return;
    const uint64_t j = q / d, u = q % d;
    out[q] = X[(uint64_t)idx[j] * ld + u];
}

// Sort keys of this iteration's samples for the MFMA pass: the FP32 squared
// norm of the translated coordinates (its bits order as unsigned integers),
// with the sample's index.  Centers ordered by norm make the pass's
// per-chunk bounds nearly per-center ones.
__global__ void k_sample_norm_keys(const float* __restrict__ X, int64_t ld, int d,
                                   const uint32_t* __restrict__ idx, uint32_t cnt,
                                   const float* __restrict__ mu, uint32_t* __restrict__ key,
                                   uint32_t* __restrict__ val)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const uint32_t r = idx[i];
    float s = 0.f;
    for (int j = 0; j < d; ++j) {
        const float t = X[(uint64_t)r * ld + j] - mu[j];
        s = __builtin_fmaf(t, t, s);
    }
    key[i] = __float_as_uint(s);
    val[i] = r;
}

// Narrow [lo, hi] of d(x,S)^2 with this iteration's new samples (certified
// bounds of the MFMA pass, per pair; see kc_md_bounds).
__global__ void k_eim_bounds(uint32_t nc, int d, const uint32_t* __restrict__ cand, KcMinOut O,
                             KcCenters C, float* __restrict__ lo, float* __restrict__ hi)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc) return;
    const uint32_t x = cand[j];
    const KcMdBounds B = kc_md_bounds(O, j, nullptr, C, d, false);
    lo[x] = fminf(lo[x], (float)B.lo_min * (1.f - 1e-6f));
    hi[x] = fminf(hi[x], (float)B.hi * (1.f + 1e-6f));
}

// dst[r * d + j] = X[S[r] * ld + j] (converted to T) for r < cnt, j < d, by
// the whole block: sixteen elements per thread and pass, the sample indices
// first and then the coordinates, each group in flight together (an element
// at a time would wait out two dependent memory latencies per element).
template <typename T>
__device__ __forceinline__ void kc_stage_samples(T* dst, const float* __restrict__ X, int64_t ld,
                                                 int d, const uint32_t* __restrict__ S,
                                                 uint32_t cnt)
{
    constexpr int V = 16;
    const uint32_t tot = cnt * (uint32_t)d;
    for (uint32_t e0 = threadIdx.x; e0 < tot; e0 += V * blockDim.x) {
        uint32_t r[V], idx[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t e = e0 + v * blockDim.x;
            r[v] = e < tot ? e / (uint32_t)d : 0u;
            idx[v] = e < tot ? S[r[v]] : 0u;
        }
        float val[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t e = e0 + v * blockDim.x;
            val[v] = e < tot ? X[(uint64_t)idx[v] * ld + (e - r[v] * (uint32_t)d)] : 0.f;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t e = e0 + v * blockDim.x;
            if (e < tot) dst[e] = (T)val[v];
        }
    }
}

// For small d the canonical FP32 distance (one lane per pair, ascending
// coordinates, relative error at most g = gamma_{d+2}) certifies far more
// tightly than MFMA's |x|^2 + |c|^2 - 2x.c, whose error scales with the
// norms: a block takes 256 candidates (one per lane, coordinates in VGPRs)
// and streams this iteration's samples through LDS.  The interval of
// d(x,S)^2 narrows to [m / (1 + g), m / (1 - g)] around the smallest FP32
// value m, widened for rounding and for squares that underflow.
#define KC_EIM_DIRECT_MAXD 8
#define KC_EIM_DIRECT_CHUNK 1024
template <int D>
__global__ __launch_bounds__(256) void k_eim_direct(const float* __restrict__ X, int64_t ld,
                                                    const uint32_t* __restrict__ cand,
                                                    uint32_t nc, const uint32_t* __restrict__ dS,
                                                    uint32_t nds, double g,
                                                    float* __restrict__ lo,
                                                    float* __restrict__ hi)
{
    __shared__ float sS[KC_EIM_DIRECT_CHUNK * D];
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = j < nc;
    const uint32_t x = live ? cand[j] : 0u;
    float xc[D];
#pragma unroll
    for (int u = 0; u < D; ++u) xc[u] = live ? X[(uint64_t)x * ld + u] : 0.f;
    float m = __builtin_inff();
    for (uint32_t i0 = 0; i0 < nds; i0 += KC_EIM_DIRECT_CHUNK) {
        const uint32_t cnt = min((uint32_t)KC_EIM_DIRECT_CHUNK, nds - i0);
        __syncthreads();
        kc_stage_samples(sS, X, ld, D, dS + i0, cnt);
        __syncthreads();
        for (uint32_t r = 0; r < cnt; ++r) {
            const float a = kc_d32_dist<D>(xc, sS + r * D);
            m = fminf(m, a);
        }
    }
    if (live) {
        const double mv = (double)m;
        double l = mv / (1.0 + g) - 1e-37 * D;
        if (l < 0.0) l = 0.0;
        const double uu = mv / (1.0 - g) + 1e-37 * D;
        lo[x] = fminf(lo[x], (float)l * (1.f - 1e-6f));
        hi[x] = fminf(hi[x], (float)uu * (1.f + 1e-6f));
    }
}

// keep iff d(x,S)^2 > tau; interval decides, else the exact pass does
__global__ void k_eim_decide(uint32_t nc, const uint32_t* __restrict__ cand,
                             const float* __restrict__ lo, const float* __restrict__ hi,
                             const double* __restrict__ tau, uint8_t* __restrict__ keep,
                             uint32_t* __restrict__ unsure, uint32_t* __restrict__ nunsure)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nc) return;
    const uint32_t x = cand[j];
    const double t = *tau;
    if ((double)lo[x] > t) {
        keep[j] = 1;
    } else if ((double)hi[x] <= t) {
        keep[j] = 0;
    } else {
        keep[j] = 0;
        unsure[atomicAdd(nunsure, 1u)] = j;
    }
}

// exact FP64 d(x,S)^2 for an undecided candidate: one block per candidate
__global__ void k_eim_exact(const float* __restrict__ X, int64_t ld, int d,
                            const uint32_t* __restrict__ cand,
                            const uint32_t* __restrict__ unsure,
                            const uint32_t* __restrict__ nunsure,
                            const uint32_t* __restrict__ S, uint32_t ns,
                            const double* __restrict__ tau, uint8_t* __restrict__ keep,
                            float* __restrict__ lo, float* __restrict__ hi)
{
    __shared__ double red[16];
    const uint32_t nu = *nunsure;
    for (uint32_t q = blockIdx.x; q < nu; q += gridDim.x) {
        const uint32_t j = unsure[q];
        const uint32_t x = cand[j];
        const float* xp = X + (uint64_t)x * ld;
        double best = __builtin_inf();
        for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x) {
            const float* sp = X + (uint64_t)S[i] * ld;
            double a = 0.0;
            for (int u = 0; u < d; ++u) a = kc_d64_step(a, (double)xp[u], (double)sp[u]);
            best = fmin(best, a);
        }
        best = kc_wave_min_f64(best);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = red[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = fmin(b, red[w]);
            keep[j] = b > *tau;
            // the exact value is its own interval from now on
            lo[x] = (float)b * (1.f - 1e-6f);
            hi[x] = (float)b * (1.f + 1e-6f);
        }
        __syncthreads();
    }
}

// The same exact pass, tiled and split: block (x, y) takes undecided
// candidates 64x .. 64x+63 (their coordinates in LDS) and slice y of S, which
// it streams through LDS in chunks of FP64 rows, so each sample row is read
// once per 64 candidates instead of once per candidate, and small candidate
// counts still spread over the whole chip.  Wave w of the block scores
// samples w, w+4, ... of a chunk against the 64 candidates (one per lane;
// the sample row is a broadcast read); the arithmetic is kc_d64_step's, so
// every value is the one the per-candidate kernel computes.  Each block's
// minimum goes into exm[q] by an atomic minimum on the bits (non-negative
// doubles order as integers); k_eim_exact_finish then decides.  For
// d <= KC_EXT_MAXD.
#define KC_EXT_MAXD 64
#define KC_EXT_LDS (32 * 1024)   // bytes for the sample chunk
__global__ __launch_bounds__(256) void k_eim_exact_split(
    const float* __restrict__ X, int64_t ld, int d, const uint32_t* __restrict__ cand,
    const uint32_t* __restrict__ unsure, uint32_t nu, const uint32_t* __restrict__ S,
    uint32_t ns, double* __restrict__ exm)
{
    __shared__ float sC[64 * (KC_EXT_MAXD + 1)];           // candidates, row pitch d | 1
    __shared__ double sS[KC_EXT_LDS / sizeof(double)];      // sample chunk, row pitch d
    __shared__ double sB[4][64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t pitch = (uint32_t)d | 1u;
    const uint32_t chunk = (uint32_t)(KC_EXT_LDS / sizeof(double)) / (uint32_t)d;
    const uint32_t q0 = blockIdx.x * 64u;
    if (q0 >= nu) return;
    const uint32_t nq = min(64u, nu - q0);
    const uint32_t per = (ns + gridDim.y - 1) / gridDim.y;
    const uint32_t s0 = min(ns, blockIdx.y * per), s1 = min(ns, s0 + per);
    for (uint32_t e = threadIdx.x; e < nq * (uint32_t)d; e += blockDim.x) {
        const uint32_t c = e / (uint32_t)d, j = e - c * (uint32_t)d;
        sC[c * pitch + j] = X[(uint64_t)cand[unsure[q0 + c]] * ld + j];
    }
    double best = __builtin_inf();
    for (uint32_t i0 = s0; i0 < s1; i0 += chunk) {
        const uint32_t nsc = min(chunk, s1 - i0);
        __syncthreads();
        kc_stage_samples(sS, X, ld, d, S + i0, nsc);
        __syncthreads();
        if (lane < nq) {
            const float* xc = sC + lane * pitch;
            for (uint32_t r = wave; r < nsc; r += 4) {
                const double* sr = sS + r * d;
                double a = 0.0;
                for (int u = 0; u < d; ++u) a = kc_d64_step(a, (double)xc[u], sr[u]);
                best = fmin(best, a);
            }
        }
    }
    sB[wave][lane] = best;
    __syncthreads();
    if (threadIdx.x < nq) {
        const double b = fmin(fmin(sB[0][lane], sB[1][lane]), fmin(sB[2][lane], sB[3][lane]));
        if (b < __builtin_inf()) atomicMin((u64*)&exm[q0 + lane], (u64)__double_as_longlong(b));
    }
}

// The same split pass for a dimension known at compile time: each lane
// holds its candidate's coordinates as doubles in VGPRs, so a pair costs a
// broadcast LDS read and three FP64 operations per coordinate (no per-pair
// conversion or candidate read); the values are kc_d64_step's, as above.
template <int D>
__global__ __launch_bounds__(256) void k_eim_exact_split_d(
    const float* __restrict__ X, int64_t ld, const uint32_t* __restrict__ cand,
    const uint32_t* __restrict__ unsure, uint32_t nu, const uint32_t* __restrict__ S,
    uint32_t ns, double* __restrict__ exm)
{
    constexpr uint32_t CH = (uint32_t)(KC_EXT_LDS / sizeof(double)) / D;   // samples per chunk
    __shared__ double sS[CH * D];
    __shared__ double sB[4][64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t q0 = blockIdx.x * 64u;
    if (q0 >= nu) return;
    const uint32_t nq = min(64u, nu - q0);
    const uint32_t per = (ns + gridDim.y - 1) / gridDim.y;
    const uint32_t s0 = min(ns, blockIdx.y * per), s1 = min(ns, s0 + per);
    const bool live = lane < nq;
    const uint32_t x = live ? cand[unsure[q0 + lane]] : 0u;
    double xd[D];
#pragma unroll
    for (int u = 0; u < D; ++u) xd[u] = (double)(live ? X[(uint64_t)x * ld + u] : 0.f);
    double best = __builtin_inf();
    for (uint32_t i0 = s0; i0 < s1; i0 += CH) {
        const uint32_t nsc = min(CH, s1 - i0);
        __syncthreads();
        kc_stage_samples(sS, X, ld, D, S + i0, nsc);
        __syncthreads();
        for (uint32_t r = wave; r < nsc; r += 4) {
            const double* sr = sS + r * D;
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < D; ++u) a = kc_d64_step(a, xd[u], sr[u]);
            best = fmin(best, a);
        }
    }
    sB[wave][lane] = best;
    __syncthreads();
    if (threadIdx.x < nq) {
        const double b = fmin(fmin(sB[0][lane], sB[1][lane]), fmin(sB[2][lane], sB[3][lane]));
        if (b < __builtin_inf()) atomicMin((u64*)&exm[q0 + lane], (u64)__double_as_longlong(b));
    }
}

// keep iff the exact d(x,S)^2 > tau; the exact value is its own interval// keep iff the exact d(x,S)^2 > tau; the exact value is its own interval
// from now on
__global__ void k_eim_exact_finish(const uint32_t* __restrict__ cand,
                                   const uint32_t* __restrict__ unsure, uint32_t nu,
                                   const double* __restrict__ exm,
                                   const double* __restrict__ tau, uint8_t* __restrict__ keep,
                                   float* __restrict__ lo, float* __restrict__ hi)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nu) return;
    const double b = exm[q];
    const uint32_t j = unsure[q];
    const uint32_t x = cand[j];
    keep[j] = b > *tau;
    lo[x] = (float)b * (1.f - 1e-6f);
    hi[x] = (float)b * (1.f + 1e-6f);
}

// Refinement of the candidates an MFMA pass left undecided, before any
// FP64: the canonical FP32 d(x,S)^2 over all of S (relative error at most
// g = gamma_{d+2}, as in the direct pass), laid out like the split exact
// pass -- blocks of 64 candidates times slices of S, partial minima by an
// atomic min on the bits (non-negative floats order as integers).
template <int D>
__global__ __launch_bounds__(256) void k_eim_refine_split(
    const float* __restrict__ X, int64_t ld, int d_rt, const uint32_t* __restrict__ cand,
    const uint32_t* __restrict__ unsure, uint32_t nu, const uint32_t* __restrict__ S,
    uint32_t ns, uint32_t* __restrict__ rmin)
{
    const int d = D > 0 ? D : d_rt;
    constexpr uint32_t LDSF = KC_EXT_LDS / sizeof(float);
    __shared__ float sS[LDSF];
    __shared__ float sB[4][64];
    const uint32_t CH = LDSF / (uint32_t)d;   // samples per chunk
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t q0 = blockIdx.x * 64u;
    if (q0 >= nu) return;
    const uint32_t nq = min(64u, nu - q0);
    const uint32_t per = (ns + gridDim.y - 1) / gridDim.y;
    const uint32_t s0 = min(ns, blockIdx.y * per), s1 = min(ns, s0 + per);
    const bool live = lane < nq;
    const uint32_t x = live ? cand[unsure[q0 + lane]] : 0u;
    const float* xp = X + (uint64_t)x * ld;
    float xr[D > 0 ? D : 1];
    if constexpr (D > 0) {
#pragma unroll
        for (int u = 0; u < D; ++u) xr[u] = live ? xp[u] : 0.f;
    }
    float best = __builtin_inff();
    for (uint32_t i0 = s0; i0 < s1; i0 += CH) {
        const uint32_t nsc = min(CH, s1 - i0);
        __syncthreads();
        kc_stage_samples(sS, X, ld, d, S + i0, nsc);
        __syncthreads();
        if (live) {
            for (uint32_t r = wave; r < nsc; r += 4) {
                const float* sr = sS + r * (uint32_t)d;
                float a = 0.f;
                if constexpr (D > 0) {
                    a = kc_d32_dist<D>(xr, sr);
                } else {
                    for (int u = 0; u < d; ++u) a = kc_d32_step(a, xp[u], sr[u]);
                }
                best = fminf(best, a);
            }
        }
    }
    sB[wave][lane] = best;
    __syncthreads();
    if (threadIdx.x < nq) {
        const float b = fminf(fminf(sB[0][lane], sB[1][lane]), fminf(sB[2][lane], sB[3][lane]));
        atomicMin(&rmin[q0 + lane], __float_as_uint(b));
    }
}

// The refined interval [m / (1 + g), m / (1 - g)] (widened as in the direct
// pass) bounds d(x,S)^2 over all of S, so it replaces the MFMA one; keep /
// remove where it decides, else the candidate joins the FP64 list.
__global__ void k_eim_refine_finish(const uint32_t* __restrict__ cand,
                                    const uint32_t* __restrict__ unsure, uint32_t nu,
                                    const uint32_t* __restrict__ rmin, double g, int d,
                                    const double* __restrict__ tau, uint8_t* __restrict__ keep,
                                    float* __restrict__ lo, float* __restrict__ hi,
                                    uint32_t* __restrict__ unsure2, uint32_t* __restrict__ n2)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nu) return;
    const uint32_t j = unsure[q];
    const uint32_t x = cand[j];
    const double mv = (double)__uint_as_float(rmin[q]);
    double l = mv / (1.0 + g) - 1e-37 * d;
    if (l < 0.0) l = 0.0;
    const double u = mv / (1.0 - g) + 1e-37 * d;
    const float lf = (float)l * (1.f - 1e-6f), uf = (float)u * (1.f + 1e-6f);
    lo[x] = lf;
    hi[x] = uf;
    const double t = *tau;
    if ((double)lf > t) {
        keep[j] = 1;
    } else {
        keep[j] = 0;
        if (!((double)uf <= t)) unsure2[atomicAdd(n2, 1u)] = j;
    }
}

__global__ void k_mark(const uint32_t* __restrict__ idx, uint32_t n, uint8_t* __restrict__ f)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) f[idx[j]] = 1;
}

__global__ void k_iota(uint32_t* __restrict__ p, uint32_t n)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = j;
}

__global__ void k_u32_to_i64(const uint32_t* __restrict__ a, uint32_t n, int64_t* __restrict__ b)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) b[j] = a[j];
}

__global__ void k_gather_soa32(const float* __restrict__ X, int64_t ld, int d,
                               const uint32_t* __restrict__ idx, uint32_t n, uint32_t padded,
                               float* __restrict__ xs, uint64_t stride)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    const uint64_t r = idx[i < n ? i : 0];
    for (int j = 0; j < d; ++j) xs[(uint64_t)j * stride + i] = X[r * ld + j];
}

// ---------------------------------------------------------------------------
// host driver

static inline dim3 g1(uint64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

static int kc_read_u32(kc_handle* h, const uint32_t* dev, uint32_t* out, hipStream_t s)
{
    if (hipMemcpyAsync(out, dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        hipError_t e = hipGetLastError();
        return h->fail(KC_EHIP, "readback: %s", hipGetErrorString(e));
    }
    return KC_OK;
}

extern "C" int kcenter_eim(kc_handle* h, const kc_points* pts, int64_t k,
                           const kc_eim_params* prm, int64_t* centers, int64_t* n_centers,
                           double* radius, int64_t* sample, int64_t* n_sample,
                           kc_eim_iter* iters, int32_t* n_iters, void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, true);
    if (rc) return rc;
    if (!prm) return h->fail(KC_EINVAL, "params NULL");
    if (!(prm->eps > 0.0 && prm->eps < 1.0)) return h->fail(KC_EINVAL, "eps must be in (0,1)");
    if (!(prm->phi > 0.0)) return h->fail(KC_EINVAL, "phi must be > 0");
    if (prm->max_iters < 1) return h->fail(KC_EINVAL, "max_iters must be >= 1");
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k out of range");
    if (!centers || !n_centers || !radius) return h->fail(KC_EINVAL, "outputs NULL");
    return kc_eim_run(h, pts, k, prm, centers, n_centers, radius, sample, n_sample, iters,
                      n_iters, (hipStream_t)stream, nullptr, nullptr);
}

int kc_eim_run(kc_handle* h, const kc_points* pts, int64_t k, const kc_eim_params* prm,
               int64_t* centers, int64_t* n_centers, double* radius, int64_t* sample,
               int64_t* n_sample, kc_eim_iter* iters, int32_t* n_iters, hipStream_t s,
               uint32_t* c_keep, uint32_t* nc_keep)
{
    int rc = KC_OK;
    const uint32_t n = (uint32_t)pts->n;
    const int d = pts->d;
    const float* X = pts->f32;
    const int64_t ld = pts->ld;

    // constants of Algorithm 2 and Select, in FP64 on the host (natural log)
    const double L = log((double)n);
    const double ne = pow((double)n, prm->eps);
    const double A_S = 9.0 * (double)k * ne * L;
    const double A_H = 4.0 * ne * L;
    const double thr = (4.0 / prm->eps) * (double)k * ne * L;
    int64_t rsel = (int64_t)ceil(prm->phi * L);
    if (rsel < 1) rsel = 1;

    uint32_t* R = (uint32_t*)h->ws("e.R", 4ull * n);
    uint32_t* R2 = (uint32_t*)h->ws("e.R2", 4ull * n);
    uint32_t* S = (uint32_t*)h->ws("e.S", 4ull * n);
    uint32_t* H = (uint32_t*)h->ws("e.H", 4ull * n);
    uint32_t* cand = (uint32_t*)h->ws("e.cand", 4ull * n);
    uint8_t* fS = (uint8_t*)h->ws("e.fS", n);
    uint8_t* fH = (uint8_t*)h->ws("e.fH", n);
    uint8_t* fK = (uint8_t*)h->ws("e.fK", n);
    uint8_t* keep = (uint8_t*)h->ws("e.keep", n);
    float* lo = (float*)h->ws("e.lo", 4ull * n);
    float* hi = (float*)h->ws("e.hi", 4ull * n);
    double* dH = (double*)h->ws("e.dH", 8ull * n);
    double* tau = (double*)h->ws("e.tau", 16);
    uint32_t* cnt = (uint32_t*)h->ws("e.cnt", 64);   // [0] dS [1] H [2] cand [3] R [4] FP64 [5] refined-undecided
    uint32_t* unsure = (uint32_t*)h->ws("e.uns", 4ull * n);
    double* exm = (double*)h->ws("e.exm", 8ull * n);   // exact minima of the undecided
    KcCompact C;
    C.nb_cap = (n + KC_CMP_ITEMS - 1) / KC_CMP_ITEMS + 1;
    C.blk = (uint32_t*)h->ws("e.blk", 4ull * C.nb_cap);
    if (!R || !R2 || !S || !H || !cand || !fS || !fH || !fK || !keep || !lo || !hi || !dH ||
        !tau || !cnt || !unsure || !exm || !C.blk)
        return h->fail(KC_ENOMEM, "workspace allocation failed");

    // local origin of the points for the MFMA distance passes (every d: the
    // MFMA variants can run at d <= 8 too): their error bound scales with
    // the norms, measured from it
    float* mu = (float*)h->ws("e.mu", 4ull * d);
    if (!mu) return h->fail(KC_ENOMEM, "workspace allocation failed");
    kc_local_origin(X, ld, d, n, mu, s);
    h->eim_exact = 0;
    h->eim_refined = 0;
    hipLaunchKernelGGL(k_iota, g1(n), dim3(256), 0, s, R, n);
    kc_fill_u32((uint32_t*)lo, 0x7F800000u, n, s);
    kc_fill_u32((uint32_t*)hi, 0x7F800000u, n, s);
    uint32_t nr = n, ns = 0;
    int it = 0;
    while ((double)nr > thr) {
        if (it >= prm->max_iters) {
            if (n_iters) *n_iters = it;
            return h->fail(KC_ENOCONV, "R still has %u points after %d iterations", nr, it);
        }
        double pS = A_S / (double)nr;
        if (pS > 1.0) pS = 1.0;
        double pH = A_H / (double)nr;
        if (pH > 1.0) pH = 1.0;
        hipLaunchKernelGGL(k_eim_draw, g1(nr), dim3(256), 0, s, R, nr, prm->seed, it, pS, pH,
                           fS, fH, fK);
        kc_compact(C, fS, R, nr, S + ns, cnt + 0, s);
        kc_compact(C, fH, R, nr, H, cnt + 1, s);
        kc_compact(C, fK, R, nr, cand, cnt + 2, s);
        uint32_t hc[3];
        if (hipMemcpyAsync(hc, cnt, 12, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return h->fail(KC_EHIP, "readback failed");
        const uint32_t nds = hc[0], nh = hc[1], nc = hc[2];
        ns += nds;
        double tau_h = -INFINITY;
        uint32_t new_nr = nr;
        if (ns > 0) {
            // Select: tau over H (exact FP64 against all of S)
            if (nh > 0) {
                kc_fill_u64((u64*)dH, 0x7FF0000000000000ull, nh, s);   // +inf
                if (d <= KC_EXT_MAXD) {
                    // the exact pass's tiling: 64 points of H per block, held
                    // as doubles, S streamed through LDS in slices (the same
                    // FP64 arithmetic, so the same values)
                    uint32_t* iota = (uint32_t*)h->ws("e.iota", 4ull * nh);
                    if (!iota) return h->fail(KC_ENOMEM, "workspace allocation failed");
                    hipLaunchKernelGGL(k_iota, g1(nh), dim3(256), 0, s, iota, nh);
                    const uint32_t gx = (nh + 63) / 64;
                    const uint32_t gy = std::max<uint32_t>(
                        1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
                    switch (d) {
#define KC_EXH_CASE(DD)                                                                        \
    case DD:                                                                                   \
        hipLaunchKernelGGL(k_eim_exact_split_d<DD>, dim3(gx, gy), dim3(256), 0, s, X, ld, H,     \
                           iota, nh, S, ns, dH);                                               \
        break;
                        KC_EXH_CASE(10)
                        KC_EXH_CASE(16)
                        KC_EXH_CASE(32)
#undef KC_EXH_CASE
                    default:
                        hipLaunchKernelGGL(k_eim_exact_split, dim3(gx, gy), dim3(256), 0, s, X,
                                           ld, d, H, iota, nh, S, ns, dH);
                    }
                } else {
                    const uint32_t splits =
                        std::max<uint32_t>(1, std::min<uint32_t>(64, ns / 4096));
                    hipLaunchKernelGGL(k_eim_dist_h, dim3((nh + 3) / 4, splits), dim3(256), 0, s,
                                       X, ld, d, H, nh, S, ns, dH);
                }
                const uint32_t rr = (uint32_t)std::min<int64_t>(rsel, nh);
                hipLaunchKernelGGL(k_eim_select, dim3(1), dim3(1024), 0, s, dH, nh, rr, tau);
            } else {
                kc_fill_u64((u64*)tau, 0xFFF0000000000000ull, 1, s);   // -inf
            }
            // Distance pass of the candidates against this iteration's
            // samples, then the keep / remove decisions: variant 0 computes
            // canonical FP32 distances on the VALU (d <= 8), 1 the FP32 MFMA,
            // 2 to 5 split BF16 MFMAs (option mfma_split): 4 or 8 waves per
            // block with 64 KiB of staged samples, then 8 or 4 waves with 32
            // KiB; all MFMA ones on the points translated to the local
            // origin.  All decide exactly alike; the
            // autotuner measures them once per shape bucket (with the
            // intervals restored before each of its runs).
            uint32_t refined_it = 0;
            auto pass = [&](int var) -> int {
                refined_it = 0;
                if (nds > 0 && nc > 0 && var == 0) {
                    const double u32 = 5.9604644775390625e-8, m = d + 2;
                    const double g = m * u32 / (1.0 - m * u32);
                    hipEvent_t ev = h->span_begin(s);
                    switch (d) {
#define KC_DIR_CASE(DD)                                                                     \
    case DD:                                                                                \
        hipLaunchKernelGGL(k_eim_direct<DD>, g1(nc), dim3(256), 0, s, X, ld, cand, nc,      \
                           S + ns - nds, nds, g, lo, hi);                                   \
        break;
                        KC_DIR_CASE(1)
                        KC_DIR_CASE(2)
                        KC_DIR_CASE(3)
                        KC_DIR_CASE(4)
                        KC_DIR_CASE(5)
                        KC_DIR_CASE(6)
                        KC_DIR_CASE(7)
                        KC_DIR_CASE(8)
#undef KC_DIR_CASE
                    }
                    h->span_end("eim_dist", ev, 1, s);
                } else if (nds > 0 && nc > 0) {
                    const bool split = var >= 2;
                    const uint32_t kpad = (nds + 15u) & ~15u;
                    const int dp =
                        split ? kc_mindist_dpad_split(d, kpad) : kc_mindist_dpad(d, false);
                    const bool packed = split && kc_split_use_packed(d, kpad);
                    float* XR = (float*)h->ws("e.XR", 4ull * nc * d);
                    KcCenters Cs;
                    Cs.kpad = kpad;
                    Cs.dp = dp;
                    Cs.Cf = (float*)h->ws("e.cf", 4ull * kpad * dp);
                    Cs.cn = (float*)h->ws("e.cn", 4ull * kpad);
                    Cs.cnl = (float*)h->ws("e.cnl", 4ull * kpad);
                    Cs.clen = (float*)h->ws("e.clen", 4ull * kpad);
                    Cs.cmax = (float*)h->ws("e.cmax", 16);
                    Cs.mu = mu;
                    if (split) {
                        Cs.Cb = (uint16_t*)h->ws("e.cbh", 2ull * kpad * dp);
                        if (packed)
                            Cs.pk = true;
                        else
                            Cs.Cbl = (uint16_t*)h->ws("e.cbl", 2ull * kpad * dp);
                    } else {
                        Cs.Ct = (float*)h->ws("e.ct", 4ull * kpad * dp);
                    }
                    KcMinOut O;
                    O.arg = (int32_t*)h->ws("e.arg", 4ull * nc);
                    O.m1 = (float*)h->ws("e.m1", 4ull * nc);
                    O.lo2 = (float*)h->ws("e.m2", 4ull * nc);
                    O.nx = (float*)h->ws("e.nx", 4ull * nc);
                    // the new samples in ascending order of norm, then staged
                    uint32_t* kin = (uint32_t*)h->ws("e.skey", 4ull * nds);
                    uint32_t* kout = (uint32_t*)h->ws("e.skey2", 4ull * nds);
                    uint32_t* vin = (uint32_t*)h->ws("e.sval", 4ull * nds);
                    uint32_t* vout = (uint32_t*)h->ws("e.sval2", 4ull * nds);
                    size_t tbytes = 0;
                    hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, kin, kout, vin, vout,
                                                       (int)nds, 0, 32, s);
                    void* tmp = h->ws("e.sorttmp", tbytes);
                    if (!XR || !Cs.Cf || (!split && !Cs.Ct) ||
                        (split && (!Cs.Cb || (!packed && !Cs.Cbl))) ||
                        !Cs.cn || !Cs.cnl || !Cs.clen || !Cs.cmax || !O.arg || !O.m1 || !O.lo2 ||
                        !O.nx || !kin || !kout || !vin || !vout || !tmp)
                        return h->fail(KC_ENOMEM, "workspace allocation failed");
                    hipLaunchKernelGGL(k_gather_rows, g1((uint64_t)nc * d), dim3(256), 0, s, X,
                                       ld, d, cand, nc, XR);
                    hipLaunchKernelGGL(k_sample_norm_keys, g1(nds), dim3(256), 0, s, X, ld, d,
                                       S + ns - nds, nds, mu, kin, vin);
                    if (hipcub::DeviceRadixSort::SortPairs(tmp, tbytes, kin, kout, vin, vout,
                                                           (int)nds, 0, 32, s) != hipSuccess) {
                        (void)hipGetLastError();
                        return h->fail(KC_EHIP, "sample sort failed");
                    }
                    kc_stage_centers(X, nullptr, ld, d, n, nullptr, vout, nds, nullptr, Cs,
                                     h->status_word, s);
                    hipEvent_t ev = h->span_begin(s);
                    // d(x, S) needs the smallest distance's bounds only
                    kc_mindist(XR, nullptr, nullptr, d, nc, d, Cs, O, false, s,
                               (var == 3 || var == 4) ? 8 : 4, var >= 4 ? 32 : 64);
                    h->span_end("eim_dist", ev, 1, s);
                    hipLaunchKernelGGL(k_eim_bounds, g1(nc), dim3(256), 0, s, nc, d, cand, O,
                                       Cs, lo, hi);
                }
                // keep / remove
                kc_fill_u32(cnt + 4, 0u, 1, s);
                hipLaunchKernelGGL(k_eim_decide, g1(nc), dim3(256), 0, s, nc, cand, lo, hi, tau,
                                   keep, unsure, cnt + 4);
                if (d <= KC_EXT_MAXD) {
                    // the undecided count sizes the split pass: candidate
                    // groups of 64 times slices of S, about 2048 blocks in all
                    uint32_t nu = 0;
                    int rc3 = kc_read_u32(h, cnt + 4, &nu, s);
                    if (rc3) return rc3;
                    const uint32_t* uns = unsure;
                    if (var > 0 && nu > 0 && (uint64_t)nu * ns >= (1ull << 22)) {
                        // the MFMA pass's undecided: canonical FP32 first
                        refined_it = nu;   // the last run's count stands
                        uint32_t* rmin = (uint32_t*)h->ws("e.rmin", 4ull * nu);
                        uint32_t* uns2 = (uint32_t*)h->ws("e.uns2", 4ull * nu);
                        if (!rmin || !uns2) return h->fail(KC_ENOMEM, "workspace allocation failed");
                        const uint32_t gx = (nu + 63) / 64;
                        const uint32_t gy = std::max<uint32_t>(
                            1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
                        kc_fill_u32(rmin, 0x7F800000u, nu, s);   // +inf
                        kc_fill_u32(cnt + 5, 0u, 1, s);
                        switch (d) {
#define KC_RFS_CASE(DD)                                                                        \
    case DD:                                                                                   \
        hipLaunchKernelGGL(k_eim_refine_split<DD>, dim3(gx, gy), dim3(256), 0, s, X, ld, d,     \
                           cand, unsure, nu, S, ns, rmin);                                     \
        break;
                            KC_RFS_CASE(2)
                            KC_RFS_CASE(3)
                            KC_RFS_CASE(8)
                            KC_RFS_CASE(10)
                            KC_RFS_CASE(16)
                            KC_RFS_CASE(32)
#undef KC_RFS_CASE
                        default:
                            hipLaunchKernelGGL(k_eim_refine_split<0>, dim3(gx, gy), dim3(256), 0,
                                               s, X, ld, d, cand, unsure, nu, S, ns, rmin);
                        }
                        const double u32 = 5.9604644775390625e-8, m = d + 2;
                        hipLaunchKernelGGL(k_eim_refine_finish, g1(nu), dim3(256), 0, s, cand,
                                           unsure, nu, rmin, m * u32 / (1.0 - m * u32), d, tau,
                                           keep, lo, hi, uns2, cnt + 5);
                        // the FP64 pass takes what is still undecided
                        hipMemcpyAsync(cnt + 4, cnt + 5, 4, hipMemcpyDeviceToDevice, s);
                        rc3 = kc_read_u32(h, cnt + 5, &nu, s);
                        if (rc3) return rc3;
                        uns = uns2;
                    }
                    if (nu > 0) {
                        const uint32_t gx = (nu + 63) / 64;
                        const uint32_t gy = std::max<uint32_t>(
                            1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
                        kc_fill_u64((u64*)exm, 0x7FF0000000000000ull, nu, s);   // +inf
                        switch (d) {
#define KC_EXS_CASE(DD)                                                                       \
    case DD:                                                                                  \
        hipLaunchKernelGGL(k_eim_exact_split_d<DD>, dim3(gx, gy), dim3(256), 0, s, X, ld, cand, \
                           uns, nu, S, ns, exm);                                              \
        break;
                            KC_EXS_CASE(10)
                            KC_EXS_CASE(16)
                            KC_EXS_CASE(32)
#undef KC_EXS_CASE
                        default:
                            hipLaunchKernelGGL(k_eim_exact_split, dim3(gx, gy), dim3(256), 0, s,
                                               X, ld, d, cand, uns, nu, S, ns, exm);
                        }
                        hipLaunchKernelGGL(k_eim_exact_finish, g1(nu), dim3(256), 0, s, cand,
                                           uns, nu, exm, tau, keep, lo, hi);
                    }
                } else {
                    hipLaunchKernelGGL(k_eim_exact, dim3(2048), dim3(256), 0, s, X, ld, d, cand,
                                       unsure, cnt + 4, S, ns, tau, keep, lo, hi);
                }
                const hipError_t e = hipGetLastError();
                return e == hipSuccess ? KC_OK
                                       : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
            };
            const bool feas[6] = {d <= KC_EIM_DIRECT_MAXD, true, h->mfma_split,
                                  h->mfma_split, h->mfma_split, h->mfma_split};
            char tkey[96];
            snprintf(tkey, sizeof tkey, "eim/%d/%d/%d", d, (int)floor(2.0 * log2((double)nc + 1)),
                     (int)floor(2.0 * log2((double)nds + 1)));
            const bool tuning = h->autotune && nds > 0 && nc > 0 && !h->tuned.count(tkey);
            if (tuning) {   // the intervals every measured run starts from
                float* lo0 = (float*)h->ws("e.lo0", 4ull * n);
                float* hi0 = (float*)h->ws("e.hi0", 4ull * n);
                if (!lo0 || !hi0) return h->fail(KC_ENOMEM, "workspace allocation failed");
                hipMemcpyAsync(lo0, lo, 4ull * n, hipMemcpyDeviceToDevice, s);
                hipMemcpyAsync(hi0, hi, 4ull * n, hipMemcpyDeviceToDevice, s);
                rc = h->tune(tkey, 6, feas, s, [&](int var) {
                    hipMemcpyAsync(lo, lo0, 4ull * n, hipMemcpyDeviceToDevice, s);
                    hipMemcpyAsync(hi, hi0, 4ull * n, hipMemcpyDeviceToDevice, s);
                    return pass(var);
                });
            } else if (nds > 0 && nc > 0) {
                rc = h->tune(tkey, 6, feas, s, pass);
            } else {
                rc = pass(1);
            }
            if (rc) return rc;
            h->eim_refined += refined_it;
            kc_compact(C, keep, cand, nc, R2, cnt + 3, s);
            std::swap(R, R2);
            uint32_t rc2[2];
            if (hipMemcpyAsync(rc2, cnt + 3, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&tau_h, tau, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return h->fail(KC_EHIP, "readback failed");
            new_nr = rc2[0];
            h->eim_exact += rc2[1];
        }
        if (iters) {
            kc_eim_iter& rec = iters[it];
            rec.r_size = nr;
            rec.ds_size = nds;
            rec.h_size = nh;
            rec.s_size = ns;
            rec.tau = tau_h;
            rec.p_s = pS;
            rec.p_h = pH;
        }
        nr = new_nr;
        ++it;
    }
    if (n_iters) *n_iters = it;

    // C = S u R, ascending: mark and compact the index range
    uint8_t* mark = fS;
    uint32_t* Cidx = H;
    hipMemsetAsync(mark, 0, n, s);
    if (ns) hipLaunchKernelGGL(k_mark, g1(ns), dim3(256), 0, s, S, ns, mark);
    if (nr) hipLaunchKernelGGL(k_mark, g1(nr), dim3(256), 0, s, R, nr, mark);
    kc_compact(C, mark, nullptr, n, Cidx, cnt + 5, s);
    uint32_t nc = 0;
    rc = kc_read_u32(h, cnt + 5, &nc, s);
    if (rc) return rc;
    if (n_sample) *n_sample = nc;
    if (c_keep) {   // the caller runs the final Gonzalez (a batch's shared launches)
        hipMemcpyAsync(c_keep, Cidx, 4ull * nc, hipMemcpyDeviceToDevice, s);
        *nc_keep = nc;
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
    }
    int64_t* C64 = sample ? sample : (int64_t*)h->ws("e.C64", 8ull * nc);
    if (!C64) return h->fail(KC_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(k_u32_to_i64, g1(nc), dim3(256), 0, s, Cidx, nc, C64);

    // Gonzalez on the sample (first center: its smallest index), then the
    // covering radius over all points
    std::vector<KcGonJob> jobs(1);
    jobs[0].X = nullptr;
    jobs[0].ld = ld;
    jobs[0].len = nc;
    jobs[0].first = 0;
    jobs[0].k = (uint32_t)k;
    KcGonRun RG;
    KcGonHost HG;
    rc = kc_plan_gon(h, "e2.", d, 1024, jobs, RG, HG, s);
    if (rc) return rc;
    const uint32_t padded = kc_pad64(nc);
    hipLaunchKernelGGL(k_gather_soa32, g1(padded), dim3(256), 0, s, X, ld, d, Cidx, nc, padded,
                       (float*)RG.xs, RG.stride);
    kc_enqueue_gon_prep(RG, HG, jobs, s);
    bool done = false;
    if (h->allow_resident) {
        int v = 0;
        uint32_t G = 0;
        if (h->resident_fit(d, nc, &v, &G)) {
            const uint64_t sw = kc_resident_slot_words((int)k, G);
            u64* slots = (u64*)h->ws("e2.slots", 8ull * sw);
            uint32_t* abort_flag = (uint32_t*)h->ws("e2.abort", 64);
            if (!slots || !abort_flag) return h->fail(KC_ENOMEM, "workspace allocation failed");
            kc_fill_u64(slots, 0ull, sw, s);
            kc_fill_u32(abort_flag, 0u, 1, s);
            if (kc_gon_resident(d, v, G, RG.xs, RG.stride, 0, nc, nullptr, 0, (int)k, RG.mind,
                                RG.keys, slots, abort_flag, h->spin_limit, nullptr, 0, 0,
                                h->status_word, nullptr, nullptr, s) == hipSuccess) {
                done = true;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    if (!done) kc_enqueue_gon_steps(RG, s);
    kc_gon_finish(RG, centers, n_centers, nullptr, nullptr, nullptr, C64, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
    return kc_assign_run(h, pts, centers, (uint32_t)k, n_centers, nullptr, radius, s, "e3.");
}
