// kc_eim.hip -- the EIM sampling pass (Algorithm 2 with Select, Algorithm 3,
// and the Section 4.1 changes) on gfx950, followed by Gonzalez on the sample.
//
// Per iteration (host-driven: phases that only queue work, each followed by
// one wait whose readback sizes the next; kc_eim_loops below):
//   k_eim_split_*     Philox4x64-10 Bernoulli draws for every x in R: into
//                     S with probability p_S, into H with probability p_H
//                     (one counter-based block per point and iteration,
//                     recomputed rather than stored); count, scan and
//                     scatter split R stably into dS (new samples), H and the
//                     points that stay candidates (not sampled) -- three
//                     launches shared by every problem still looping;
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
    uint32_t* blk = nullptr;   // [3][nb_cap] block counts / offsets
    uint32_t nb_cap = 0;
};

// ---------------------------------------------------------------------------
// An iteration's draws and the split of R in three launches: the draws of
// a point (counter-based) are recomputed where they are needed instead of
// stored, and dS, H and the candidates (the points not sampled) are each
// compacted in R's order.

__device__ __forceinline__ void kc_eim_flags(uint32_t x, uint64_t seed, int it, double pS,
                                             double pH, bool& s, bool& hh)
{
    uint64_t c[4] = {(uint64_t)x, (uint64_t)it, 0ull, 0ull};
    kc_philox4x64_10(c, seed, 0ull);
    s = (double)(c[0] >> 11) * 0x1.0p-53 < pS;
    hh = (double)(c[1] >> 11) * 0x1.0p-53 < pH;
}

// One problem's share of a shared split launch (the problems of a batch in
// lockstep, or one): its R, outputs, block counts [3][nb] and draw
// parameters; its blocks are blk0 .. blk0 + nb - 1 of the launch.
struct KcEimSplitJob {
    const uint32_t* R;
    uint32_t* outS;   // S + |S| before the draws
    uint32_t* outH;
    uint32_t* outK;   // the candidates
    uint32_t* blk;    // [3][nb]
    uint64_t seed;
    double pS, pH;
    uint32_t nr, nb, blk0;
    int32_t it;
};

// the job whose blocks contain block b (jobs in ascending blk0)
template <class JT>
__device__ __forceinline__ const JT& kc_split_job(const JT* __restrict__ J, int nj, uint32_t b)
{
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (J[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return J[lo];
}

__global__ __launch_bounds__(256) void k_eim_split_count(const KcEimSplitJob* __restrict__ J,
                                                         int nj)
{
    __shared__ uint32_t red[3][4];
    const KcEimSplitJob& jb = kc_split_job(J, nj, blockIdx.x);
    const uint32_t lb = blockIdx.x - jb.blk0;
    const uint32_t base = lb * KC_CMP_ITEMS, nr = jb.nr;
    uint32_t c[3] = {0u, 0u, 0u};
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        if (i < nr) {
            bool sm, hm;
            kc_eim_flags(jb.R[i], jb.seed, jb.it, jb.pS, jb.pH, sm, hm);
            c[0] += sm;
            c[1] += hm;
            c[2] += !sm;   // sampled points always leave R
        }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        for (int off = 32; off >= 1; off >>= 1) c[f] += __shfl_xor(c[f], off, 64);
        if ((threadIdx.x & 63) == 0) red[f][threadIdx.x >> 6] = c[f];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const uint32_t f = threadIdx.x;
        jb.blk[(uint64_t)f * jb.nb + lb] = red[f][0] + red[f][1] + red[f][2] + red[f][3];
    }
}

// One block of 1024 threads: the exclusive scan of nb block counts in
// place; returns the total (to every thread).
__device__ uint32_t kc_scan_block_counts(uint32_t* __restrict__ blk, uint32_t nb)
{
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[16];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? blk[i] : 0u;
        uint32_t x = v;
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
    const uint32_t tot = carry;
    __syncthreads();
    return tot;
}

// block j (1024 threads): job j's three exclusive scans; its totals ->
// count3[3j .. 3j+2]
__global__ __launch_bounds__(1024) void k_eim_split_scan(const KcEimSplitJob* __restrict__ J,
                                                         uint32_t* __restrict__ count3)
{
    const KcEimSplitJob& jb = J[blockIdx.x];
    for (int f = 0; f < 3; ++f) {
        const uint32_t tot = kc_scan_block_counts(jb.blk + (uint64_t)f * jb.nb, jb.nb);
        if (threadIdx.x == 0) count3[3 * blockIdx.x + f] = tot;
    }
}

// R' = the kept candidates of every problem that decided this iteration,
// in three shared launches (stable compaction of the keep flags); per
// problem out4[4j ..] = |R'|, its FP64-decided count and tau's two words.
struct KcKeepJob {
    const uint8_t* f;          // keep flags, per candidate
    const uint32_t* in;        // the candidates
    uint32_t* out;             // R'
    uint32_t* blk;             // [nb]
    const uint32_t* nexact;    // FP64-decided count of the iteration
    const double* tau;
    uint32_t n, nb, blk0, pad;
};

__global__ __launch_bounds__(256) void k_keep_count(const KcKeepJob* __restrict__ J, int nj)
{
    __shared__ uint32_t red[4];
    const KcKeepJob& jb = kc_split_job(J, nj, blockIdx.x);
    const uint32_t lb = blockIdx.x - jb.blk0;
    const uint32_t base = lb * KC_CMP_ITEMS;
    uint32_t c = 0;
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        if (i < jb.n) c += jb.f[i] != 0;
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) jb.blk[lb] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(1024) void k_keep_scan(const KcKeepJob* __restrict__ J,
                                                    uint32_t* __restrict__ out4)
{
    const KcKeepJob& jb = J[blockIdx.x];
    const uint32_t tot = kc_scan_block_counts(jb.blk, jb.nb);
    if (threadIdx.x == 0) {
        uint32_t tw[2];
        memcpy(tw, jb.tau, 8);
        out4[4 * blockIdx.x + 0] = tot;
        out4[4 * blockIdx.x + 1] = *jb.nexact;
        out4[4 * blockIdx.x + 2] = tw[0];
        out4[4 * blockIdx.x + 3] = tw[1];
    }
}

__global__ __launch_bounds__(256) void k_keep_scatter(const KcKeepJob* __restrict__ J, int nj)
{
    __shared__ uint32_t wcnt[4];
    const KcKeepJob& jb = kc_split_job(J, nj, blockIdx.x);
    const uint32_t lb = blockIdx.x - jb.blk0;
    const uint32_t base = lb * KC_CMP_ITEMS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t run = jb.blk[lb];
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        const bool on = i < jb.n && jb.f[i] != 0;
        const u64 mask = __ballot(on);
        if (lane == 0) wcnt[w] = __popcll(mask);
        __syncthreads();
        uint32_t wpre = 0;
        for (int v = 0; v < w; ++v) wpre += wcnt[v];
        if (on) jb.out[run + wpre + __popcll(mask & ((1ull << lane) - 1ull))] = jb.in[i];
        run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_eim_split_scatter(const KcEimSplitJob* __restrict__ J,
                                                           int nj)
{
    __shared__ uint32_t wcnt[3][4];
    const KcEimSplitJob& jb = kc_split_job(J, nj, blockIdx.x);
    const uint32_t lb = blockIdx.x - jb.blk0;
    const uint32_t base = lb * KC_CMP_ITEMS, nr = jb.nr;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t run[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) run[f] = jb.blk[(uint64_t)f * jb.nb + lb];
    uint32_t* out[3] = {jb.outS, jb.outH, jb.outK};
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + q * 256 + threadIdx.x;
        bool on[3] = {false, false, false};
        uint32_t x = 0;
        if (i < nr) {
            x = jb.R[i];
            kc_eim_flags(x, jb.seed, jb.it, jb.pS, jb.pH, on[0], on[1]);
            on[2] = !on[0];
        }
        u64 mask[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            mask[f] = __ballot(on[f]);
            if (lane == 0) wcnt[f][w] = __popcll(mask[f]);
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            uint32_t wpre = 0;
            for (int v = 0; v < w; ++v) wpre += wcnt[f][v];
            if (on[f])
                out[f][run[f] + wpre + __popcll(mask[f] & ((1ull << lane) - 1ull))] = x;
            run[f] += wcnt[f][0] + wcnt[f][1] + wcnt[f][2] + wcnt[f][3];
        }
        __syncthreads();
    }
}

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
//
// Algorithm 2's loop runs as phases that only enqueue work; between phases
// the host reads the few counts that size the next phase's launches, from
// pinned words that every problem in flight fills before one wait.
// kc_eim_loops drives one problem (kcenter_eim) or a batch's in lockstep:
// per iteration the draws and compactions of every problem, a wait; Select,
// the distance pass and the decisions, a wait; the FP32 refinement where it
// applies, a wait; the FP64 decisions and R's compaction, a wait.  Each
// problem's arithmetic and order of operations are those of a run alone.

static inline dim3 g1(uint64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

// One problem's loop state.  Buffers named with `pre` are the problem's own
// (they live across phases); the distance pass's scratch is shared, since a
// problem's use of it starts and ends within one phase on the one stream.
struct KcEimLoop {
    int id = 0;
    const float* X = nullptr;
    int64_t ld = 0;
    uint32_t n = 0;
    int d = 0;
    int64_t k = 0;
    const kc_eim_params* prm = nullptr;
    kc_eim_iter* iters = nullptr;
    std::string pre;
    double A_S = 0.0, A_H = 0.0, thr = 0.0;
    int64_t rsel = 1;
    uint32_t *R = nullptr, *R2 = nullptr, *S = nullptr, *H = nullptr, *cand = nullptr;
    uint32_t *unsure = nullptr, *uns2 = nullptr, *cnt = nullptr;
    uint8_t *fS = nullptr, *keep = nullptr;   // fS: marks when C is formed
    float *lo = nullptr, *hi = nullptr, *mu = nullptr;
    double* tau = nullptr;
    KcCompact C;
    // pinned: [0..2] |dS| |H| |cand|, [3] undecided, [4] |R'|, [5] FP64-decided,
    // [6..7] tau (a double)
    uint32_t* hw = nullptr;
    uint32_t nr = 0, ns = 0;
    int it = 0;
    bool done = false;
    // the current iteration
    double pS = 0.0, pH = 0.0;
    uint32_t nds = 0, nh = 0, nc = 0, nu = 0, refined_it = 0;
    int var = 1;
    bool passed = false;   // S is not empty: distance pass and decisions
    bool whole = false;    // the tuner ran the pass to its end
    bool refine = false;   // FP32 refinement this iteration
};

static int kc_eim_init(kc_handle* h, KcEimLoop& P, const kc_points* pts, int64_t k,
                       const kc_eim_params* prm, kc_eim_iter* iters, hipStream_t s)
{
    P.X = pts->f32;
    P.ld = pts->ld;
    P.n = (uint32_t)pts->n;
    P.d = pts->d;
    P.k = k;
    P.prm = prm;
    P.iters = iters;
    const uint32_t n = P.n;
    // constants of Algorithm 2 and Select, in FP64 on the host (natural log)
    const double L = log((double)n);
    const double ne = pow((double)n, prm->eps);
    P.A_S = 9.0 * (double)k * ne * L;
    P.A_H = 4.0 * ne * L;
    P.thr = (4.0 / prm->eps) * (double)k * ne * L;
    P.rsel = (int64_t)ceil(prm->phi * L);
    if (P.rsel < 1) P.rsel = 1;
    const std::string& p = P.pre;
    P.R = (uint32_t*)h->ws(p + "R", 4ull * n);
    P.R2 = (uint32_t*)h->ws(p + "R2", 4ull * n);
    P.S = (uint32_t*)h->ws(p + "S", 4ull * n);
    P.H = (uint32_t*)h->ws(p + "H", 4ull * n);
    P.cand = (uint32_t*)h->ws(p + "cand", 4ull * n);
    P.fS = (uint8_t*)h->ws(p + "fS", n);
    P.keep = (uint8_t*)h->ws(p + "keep", n);
    P.lo = (float*)h->ws(p + "lo", 4ull * n);
    P.hi = (float*)h->ws(p + "hi", 4ull * n);
    P.tau = (double*)h->ws(p + "tau", 16);
    // [0] dS [1] H [2] cand [3] R [4] FP64 [5] refined-undecided
    P.cnt = (uint32_t*)h->ws(p + "cnt", 64);
    P.unsure = (uint32_t*)h->ws(p + "uns", 4ull * n);
    P.uns2 = (uint32_t*)h->ws(p + "uns2", 4ull * n);
    P.C.nb_cap = (n + KC_CMP_ITEMS - 1) / KC_CMP_ITEMS + 1;
    P.C.blk = (uint32_t*)h->ws(p + "blk", 3 * 4ull * P.C.nb_cap);
    // local origin of the points for the MFMA distance passes (every d: the
    // MFMA variants can run at d <= 8 too): their error bound scales with
    // the norms, measured from it
    P.mu = (float*)h->ws(p + "mu", 4ull * P.d);
    if (!P.R || !P.R2 || !P.S || !P.H || !P.cand || !P.fS || !P.keep ||
        !P.lo || !P.hi || !P.tau || !P.cnt || !P.unsure || !P.uns2 || !P.C.blk || !P.mu)
        return h->fail(KC_ENOMEM, "workspace allocation failed");
    kc_local_origin(P.X, P.ld, P.d, n, P.mu, s);
    hipLaunchKernelGGL(k_iota, g1(n), dim3(256), 0, s, P.R, n);
    kc_fill_u32((uint32_t*)P.lo, 0x7F800000u, n, s);
    kc_fill_u32((uint32_t*)P.hi, 0x7F800000u, n, s);
    P.nr = n;
    P.ns = 0;
    P.it = 0;
    P.done = false;
    return KC_OK;
}

// Phase 1 for one problem: the loop test; an iteration that runs gets its
// draw probabilities and its job in the shared split launches.
static int kc_eim_begin_iter(kc_handle* h, KcEimLoop& P)
{
    if ((double)P.nr <= P.thr) {
        P.done = true;
        return KC_OK;
    }
    if (P.it >= P.prm->max_iters)
        return h->fail(KC_ENOCONV, "R still has %u points after %d iterations", P.nr, P.it);
    P.pS = P.A_S / (double)P.nr;
    if (P.pS > 1.0) P.pS = 1.0;
    P.pH = P.A_H / (double)P.nr;
    if (P.pH > 1.0) P.pH = 1.0;
    return KC_OK;
}

// Phase 1 for every problem still looping, in three shared launches: the
// draws and the split of each R into dS, H and the candidates; the sizes go
// to each problem's hw[0..2] (through one readback).
static int kc_eim_split_phase(kc_handle* h, std::vector<KcEimLoop*>& act, hipStream_t s)
{
    std::vector<KcEimSplitJob> jobs(act.size());
    uint32_t total = 0;
    for (size_t q = 0; q < act.size(); ++q) {
        KcEimLoop& P = *act[q];
        KcEimSplitJob& j = jobs[q];
        j.R = P.R;
        j.outS = P.S + P.ns;
        j.outH = P.H;
        j.outK = P.cand;
        j.blk = P.C.blk;
        j.seed = P.prm->seed;
        j.pS = P.pS;
        j.pH = P.pH;
        j.nr = P.nr;
        j.nb = (P.nr + KC_CMP_ITEMS - 1) / KC_CMP_ITEMS;
        j.blk0 = total;
        j.it = P.it;
        total += j.nb;
    }
    const int nj = (int)jobs.size();
    const KcEimSplitJob* J =
        (const KcEimSplitJob*)h->upload("eim.jobs", jobs.data(), sizeof(KcEimSplitJob) * nj, s);
    uint32_t* c3 = (uint32_t*)h->ws("eim.c3", 12ull * nj);
    uint32_t* c3h = (uint32_t*)h->pinned("eim.c3", 12ull * nj);
    if (!J || !c3 || !c3h) return h->fail(KC_ENOMEM, "workspace allocation failed");
    hipLaunchKernelGGL(k_eim_split_count, dim3(total), dim3(256), 0, s, J, nj);
    hipLaunchKernelGGL(k_eim_split_scan, dim3(nj), dim3(1024), 0, s, J, c3);
    hipLaunchKernelGGL(k_eim_split_scatter, dim3(total), dim3(256), 0, s, J, nj);
    if (hipMemcpyAsync(c3h, c3, 12ull * nj, hipMemcpyDeviceToHost, s) != hipSuccess)
        return h->fail(KC_EHIP, "readback failed");
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

// Select (Algorithm 3): tau over H, exact FP64 against all of S.
static int kc_eim_select(kc_handle* h, KcEimLoop& P, hipStream_t s)
{
    const uint32_t nh = P.nh, ns = P.ns;
    const int d = P.d;
    if (nh == 0) {
        kc_fill_u64((u64*)P.tau, 0xFFF0000000000000ull, 1, s);   // -inf
        return KC_OK;
    }
    double* dH = (double*)h->ws("e.dH", 8ull * nh);
    if (!dH) return h->fail(KC_ENOMEM, "workspace allocation failed");
    kc_fill_u64((u64*)dH, 0x7FF0000000000000ull, nh, s);   // +inf
    if (d <= KC_EXT_MAXD) {
        // the exact pass's tiling: 64 points of H per block, held as
        // doubles, S streamed through LDS in slices (the same FP64
        // arithmetic, so the same values)
        uint32_t* iota = (uint32_t*)h->ws("e.iota", 4ull * nh);
        if (!iota) return h->fail(KC_ENOMEM, "workspace allocation failed");
        hipLaunchKernelGGL(k_iota, g1(nh), dim3(256), 0, s, iota, nh);
        const uint32_t gx = (nh + 63) / 64;
        const uint32_t gy = std::max<uint32_t>(
            1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
        switch (d) {
#define KC_EXH_CASE(DD)                                                                        \
    case DD:                                                                                   \
        hipLaunchKernelGGL(k_eim_exact_split_d<DD>, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld,  \
                           P.H, iota, nh, P.S, ns, dH);                                        \
        break;
            KC_EXH_CASE(10)
            KC_EXH_CASE(16)
            KC_EXH_CASE(32)
#undef KC_EXH_CASE
        default:
            hipLaunchKernelGGL(k_eim_exact_split, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld, d,
                               P.H, iota, nh, P.S, ns, dH);
        }
    } else {
        const uint32_t splits = std::max<uint32_t>(1, std::min<uint32_t>(64, ns / 4096));
        hipLaunchKernelGGL(k_eim_dist_h, dim3((nh + 3) / 4, splits), dim3(256), 0, s, P.X, P.ld,
                           d, P.H, nh, P.S, ns, dH);
    }
    const uint32_t rr = (uint32_t)std::min<int64_t>(P.rsel, nh);
    hipLaunchKernelGGL(k_eim_select, dim3(1), dim3(1024), 0, s, dH, nh, rr, P.tau);
    return KC_OK;
}

// The distance pass of the candidates against this iteration's samples and
// the keep / remove decisions by the intervals.  Variant 0 computes
// canonical FP32 distances on the VALU (d <= 8), 1 the FP32 MFMA, 2 to 5
// split BF16 MFMAs (option mfma_split): 4 or 8 waves per block with 64 KiB
// of staged samples, then 8 or 4 waves with 32 KiB; all MFMA ones on the
// points translated to the local origin.  All decide exactly alike.  With
// d <= KC_EXT_MAXD the undecided count goes to hw[3] (it sizes the next
// phase); above, the exact FP64 decisions follow here.
static int kc_eim_pass_front(kc_handle* h, KcEimLoop& P, int var, hipStream_t s)
{
    const uint32_t nds = P.nds, nc = P.nc, ns = P.ns;
    const int d = P.d;
    P.refined_it = 0;
    P.refine = false;
    if (nds > 0 && nc > 0 && var == 0) {
        const double u32 = 5.9604644775390625e-8, m = d + 2;
        const double g = m * u32 / (1.0 - m * u32);
        hipEvent_t ev = h->span_begin(s);
        switch (d) {
#define KC_DIR_CASE(DD)                                                                     \
    case DD:                                                                                \
        hipLaunchKernelGGL(k_eim_direct<DD>, g1(nc), dim3(256), 0, s, P.X, P.ld, P.cand, nc,  \
                           P.S + ns - nds, nds, g, P.lo, P.hi);                             \
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
        const int dp = split ? kc_mindist_dpad_split(d, kpad) : kc_mindist_dpad(d, false);
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
        Cs.mu = P.mu;
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
        if (hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, kin, kout, vin, vout, (int)nds,
                                               0, 32, s) != hipSuccess)
            return h->fail(KC_EHIP, "sort size query failed");
        void* tmp = h->ws("e.sorttmp", tbytes);
        if (!XR || !Cs.Cf || (!split && !Cs.Ct) || (split && (!Cs.Cb || (!packed && !Cs.Cbl))) ||
            !Cs.cn || !Cs.cnl || !Cs.clen || !Cs.cmax || !O.arg || !O.m1 || !O.lo2 || !O.nx ||
            !kin || !kout || !vin || !vout || !tmp)
            return h->fail(KC_ENOMEM, "workspace allocation failed");
        hipLaunchKernelGGL(k_gather_rows, g1((uint64_t)nc * d), dim3(256), 0, s, P.X, P.ld, d,
                           P.cand, nc, XR);
        hipLaunchKernelGGL(k_sample_norm_keys, g1(nds), dim3(256), 0, s, P.X, P.ld, d,
                           P.S + ns - nds, nds, P.mu, kin, vin);
        if (hipcub::DeviceRadixSort::SortPairs(tmp, tbytes, kin, kout, vin, vout, (int)nds, 0, 32,
                                               s) != hipSuccess) {
            (void)hipGetLastError();
            return h->fail(KC_EHIP, "sample sort failed");
        }
        kc_stage_centers(P.X, nullptr, P.ld, d, P.n, nullptr, vout, nds, nullptr, Cs,
                         h->status_word, s);
        hipEvent_t ev = h->span_begin(s);
        // d(x, S) needs the smallest distance's bounds only
        kc_mindist(XR, nullptr, nullptr, d, nc, d, Cs, O, false, s,
                   (var == 3 || var == 4) ? 8 : 4, var >= 4 ? 32 : 64);
        h->span_end("eim_dist", ev, 1, s);
        hipLaunchKernelGGL(k_eim_bounds, g1(nc), dim3(256), 0, s, nc, d, P.cand, O, Cs, P.lo,
                           P.hi);
    }
    // keep / remove
    kc_fill_u32(P.cnt + 4, 0u, 1, s);
    hipLaunchKernelGGL(k_eim_decide, g1(nc), dim3(256), 0, s, nc, P.cand, P.lo, P.hi, P.tau,
                       P.keep, P.unsure, P.cnt + 4);
    if (d <= KC_EXT_MAXD) {
        if (hipMemcpyAsync(P.hw + 3, P.cnt + 4, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            return h->fail(KC_EHIP, "readback failed");
    } else {
        hipLaunchKernelGGL(k_eim_exact, dim3(2048), dim3(256), 0, s, P.X, P.ld, d, P.cand,
                           P.unsure, P.cnt + 4, P.S, ns, P.tau, P.keep, P.lo, P.hi);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

// The MFMA pass's undecided (hw[3] of the front phase), when there are
// enough of them against S: canonical FP32 over all of S first; what it
// leaves undecided goes to hw[3].
static int kc_eim_pass_refine(kc_handle* h, KcEimLoop& P, int var, hipStream_t s)
{
    P.nu = P.hw[3];
    const uint32_t nu = P.nu, ns = P.ns;
    const int d = P.d;
    if (!(var > 0 && nu > 0 && (uint64_t)nu * ns >= (1ull << 22))) return KC_OK;
    P.refine = true;
    P.refined_it = nu;
    uint32_t* rmin = (uint32_t*)h->ws("e.rmin", 4ull * nu);
    if (!rmin) return h->fail(KC_ENOMEM, "workspace allocation failed");
    const uint32_t gx = (nu + 63) / 64;
    const uint32_t gy =
        std::max<uint32_t>(1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
    kc_fill_u32(rmin, 0x7F800000u, nu, s);   // +inf
    kc_fill_u32(P.cnt + 5, 0u, 1, s);
    switch (d) {
#define KC_RFS_CASE(DD)                                                                        \
    case DD:                                                                                   \
        hipLaunchKernelGGL(k_eim_refine_split<DD>, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld, d, \
                           P.cand, P.unsure, nu, P.S, ns, rmin);                               \
        break;
        KC_RFS_CASE(2)
        KC_RFS_CASE(3)
        KC_RFS_CASE(8)
        KC_RFS_CASE(10)
        KC_RFS_CASE(16)
        KC_RFS_CASE(32)
#undef KC_RFS_CASE
    default:
        hipLaunchKernelGGL(k_eim_refine_split<0>, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld, d,
                           P.cand, P.unsure, nu, P.S, ns, rmin);
    }
    const double u32 = 5.9604644775390625e-8, m = d + 2;
    hipLaunchKernelGGL(k_eim_refine_finish, g1(nu), dim3(256), 0, s, P.cand, P.unsure, nu, rmin,
                       m * u32 / (1.0 - m * u32), d, P.tau, P.keep, P.lo, P.hi, P.uns2,
                       P.cnt + 5);
    // the FP64 pass takes what is still undecided
    if (hipMemcpyAsync(P.cnt + 4, P.cnt + 5, 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(P.hw + 3, P.cnt + 5, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return h->fail(KC_EHIP, "readback failed");
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

// Exact FP64 decisions of what is still undecided (hw[3]).
static int kc_eim_pass_exact(kc_handle* h, KcEimLoop& P, hipStream_t s)
{
    if (P.refine) P.nu = P.hw[3];
    const uint32_t nu = P.nu, ns = P.ns;
    const int d = P.d;
    if (nu == 0) return KC_OK;
    const uint32_t* uns = P.refine ? P.uns2 : P.unsure;
    double* exm = (double*)h->ws("e.exm", 8ull * nu);   // exact minima of the undecided
    if (!exm) return h->fail(KC_ENOMEM, "workspace allocation failed");
    const uint32_t gx = (nu + 63) / 64;
    const uint32_t gy =
        std::max<uint32_t>(1, std::min<uint32_t>({(2048 + gx - 1) / gx, ns / 512, 65535u}));
    kc_fill_u64((u64*)exm, 0x7FF0000000000000ull, nu, s);   // +inf
    switch (d) {
#define KC_EXS_CASE(DD)                                                                       \
    case DD:                                                                                  \
        hipLaunchKernelGGL(k_eim_exact_split_d<DD>, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld,  \
                           P.cand, uns, nu, P.S, ns, exm);                                    \
        break;
        KC_EXS_CASE(10)
        KC_EXS_CASE(16)
        KC_EXS_CASE(32)
#undef KC_EXS_CASE
    default:
        hipLaunchKernelGGL(k_eim_exact_split, dim3(gx, gy), dim3(256), 0, s, P.X, P.ld, d,
                           P.cand, uns, nu, P.S, ns, exm);
    }
    hipLaunchKernelGGL(k_eim_exact_finish, g1(nu), dim3(256), 0, s, P.cand, uns, nu, exm, P.tau,
                       P.keep, P.lo, P.hi);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

static int kc_eim_wait(kc_handle* h, hipStream_t s)
{
    if (hipStreamSynchronize(s) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        return h->fail(KC_EHIP, "readback: %s", hipGetErrorString(e));
    }
    return KC_OK;
}

// The whole pass with its own waits (the tuner's unit of measurement).
static int kc_eim_pass_whole(kc_handle* h, KcEimLoop& P, int var, hipStream_t s)
{
    int rc = kc_eim_pass_front(h, P, var, s);
    if (rc || P.d > KC_EXT_MAXD) return rc;
    if ((rc = kc_eim_wait(h, s))) return rc;
    if ((rc = kc_eim_pass_refine(h, P, var, s))) return rc;
    if (P.refine && (rc = kc_eim_wait(h, s))) return rc;
    return kc_eim_pass_exact(h, P, s);
}

// Phase 2: Select and the front of the distance pass.  An untuned shape
// bucket is measured here: every feasible variant runs whole (the intervals
// restored before each run), and the chosen one's results stand.
static int kc_eim_front_phase(kc_handle* h, KcEimLoop& P, hipStream_t s)
{
    P.nds = P.hw[0];
    P.nh = P.hw[1];
    P.nc = P.hw[2];
    P.ns += P.nds;
    P.passed = P.ns > 0;
    P.whole = false;
    P.refine = false;
    P.nu = 0;
    P.refined_it = 0;
    if (!P.passed) return KC_OK;
    int rc = kc_eim_select(h, P, s);
    if (rc) return rc;
    const int d = P.d;
    if (!(P.nds > 0 && P.nc > 0)) {
        P.var = 1;
        return kc_eim_pass_front(h, P, 1, s);
    }
    const bool feas[6] = {d <= KC_EIM_DIRECT_MAXD, true, h->mfma_split,
                          h->mfma_split, h->mfma_split, h->mfma_split};
    char tkey[96];
    snprintf(tkey, sizeof tkey, "eim/%d/%d/%d", d, (int)floor(2.0 * log2((double)P.nc + 1)),
             (int)floor(2.0 * log2((double)P.nds + 1)));
    bool measure = false;
    P.var = h->choice(tkey, 6, feas, s, &measure);
    if (P.var < 0) return h->fail(KC_EUNSUPPORTED, "no feasible variant for %s", tkey);
    if (!measure) return kc_eim_pass_front(h, P, P.var, s);
    // the intervals every measured run starts from
    const uint32_t n = P.n;
    float* lo0 = (float*)h->ws("e.lo0", 4ull * n);
    float* hi0 = (float*)h->ws("e.hi0", 4ull * n);
    if (!lo0 || !hi0) return h->fail(KC_ENOMEM, "workspace allocation failed");
    if (hipMemcpyAsync(lo0, P.lo, 4ull * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(hi0, P.hi, 4ull * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return h->fail(KC_EHIP, "interval copy failed");
    P.whole = true;
    return h->tune(tkey, 6, feas, s, [&](int v) {
        if (hipMemcpyAsync(P.lo, lo0, 4ull * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(P.hi, hi0, 4ull * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return h->fail(KC_EHIP, "interval copy failed");
        P.var = v;
        return kc_eim_pass_whole(h, P, v, s);
    });
}

// Phase 4: the rest of the decisions, then R' = the kept candidates; |R'|,
// the FP64-decided count and tau go to hw[4..7].
static int kc_eim_keep_phase(kc_handle* h, KcEimLoop& P, hipStream_t s)
{
    if (!P.passed) return KC_OK;
    if (!P.whole && P.d <= KC_EXT_MAXD) {
        const int rc = kc_eim_pass_exact(h, P, s);
        if (rc) return rc;
    }
    h->eim_refined += P.refined_it;
    return KC_OK;
}

// R' of every problem that decided this iteration (kc_eim_keep_phase done):
// shared compaction launches, then |R'|, the FP64-decided count and tau into
// each problem's hw[4..7] through one readback; R and R2 swap.
static int kc_eim_compact_phase(kc_handle* h, std::vector<KcEimLoop*>& dec, hipStream_t s)
{
    if (dec.empty()) return KC_OK;
    std::vector<KcKeepJob> jobs(dec.size());
    uint32_t total = 0;
    for (size_t q = 0; q < dec.size(); ++q) {
        KcEimLoop& P = *dec[q];
        KcKeepJob& j = jobs[q];
        j.f = P.keep;
        j.in = P.cand;
        j.out = P.R2;
        j.blk = P.C.blk;
        j.nexact = P.cnt + 4;
        j.tau = P.tau;
        j.n = P.nc;
        j.nb = (P.nc + KC_CMP_ITEMS - 1) / KC_CMP_ITEMS;
        j.blk0 = total;
        j.pad = 0;
        total += j.nb;
        std::swap(P.R, P.R2);
    }
    const int nj = (int)jobs.size();
    const KcKeepJob* J =
        (const KcKeepJob*)h->upload("eim.kjobs", jobs.data(), sizeof(KcKeepJob) * nj, s);
    uint32_t* o4 = (uint32_t*)h->ws("eim.k4", 16ull * nj);
    uint32_t* o4h = (uint32_t*)h->pinned("eim.k4", 16ull * nj);
    if (!J || !o4 || !o4h) return h->fail(KC_ENOMEM, "workspace allocation failed");
    if (total) hipLaunchKernelGGL(k_keep_count, dim3(total), dim3(256), 0, s, J, nj);
    hipLaunchKernelGGL(k_keep_scan, dim3(nj), dim3(1024), 0, s, J, o4);
    if (total) hipLaunchKernelGGL(k_keep_scatter, dim3(total), dim3(256), 0, s, J, nj);
    if (hipMemcpyAsync(o4h, o4, 16ull * nj, hipMemcpyDeviceToHost, s) != hipSuccess)
        return h->fail(KC_EHIP, "readback failed");
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

// Phase 5 (host): the iteration's record; R' becomes R.
static void kc_eim_end_iter(kc_handle* h, KcEimLoop& P)
{
    double tau_h = -INFINITY;
    uint32_t new_nr = P.nr;
    if (P.passed) {
        new_nr = P.hw[4];
        h->eim_exact += P.hw[5];
        memcpy(&tau_h, P.hw + 6, 8);
    }
    if (P.iters) {
        kc_eim_iter& rec = P.iters[P.it];
        rec.r_size = P.nr;
        rec.ds_size = P.nds;
        rec.h_size = P.nh;
        rec.s_size = P.ns;
        rec.tau = tau_h;
        rec.p_s = P.pS;
        rec.p_h = P.pH;
    }
    P.nr = new_nr;
    ++P.it;
}

// C = S u R in ascending order into P.H; its size goes to hw[0].
static int kc_eim_form_c(kc_handle* h, KcEimLoop& P, hipStream_t s)
{
    uint8_t* mark = P.fS;
    if (hipMemsetAsync(mark, 0, P.n, s) != hipSuccess)
        return h->fail(KC_EHIP, "mark clear failed");
    if (P.ns) hipLaunchKernelGGL(k_mark, g1(P.ns), dim3(256), 0, s, P.S, P.ns, mark);
    if (P.nr) hipLaunchKernelGGL(k_mark, g1(P.nr), dim3(256), 0, s, P.R, P.nr, mark);
    kc_compact(P.C, mark, nullptr, P.n, P.H, P.cnt + 5, s);
    if (hipMemcpyAsync(P.hw, P.cnt + 5, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return h->fail(KC_EHIP, "readback failed");
    return KC_OK;
}

// Drive every loop to its end in lockstep, then form each C (its size in
// hw[0], its indices in H).  A problem that fails stops the call.
static int kc_eim_loops(kc_handle* h, std::vector<KcEimLoop>& L, hipStream_t s)
{
    int rc;
    auto fail_at = [&](const KcEimLoop& P, int code) {
        return L.size() > 1 ? h->fail(code, "problem %d: %s", P.id, h->last_error.c_str())
                            : code;
    };
    std::vector<KcEimLoop*> act;
    for (;;) {
        act.clear();
        for (KcEimLoop& P : L)
            if (!P.done) {
                if ((rc = kc_eim_begin_iter(h, P))) return fail_at(P, rc);
                if (!P.done) act.push_back(&P);
            }
        if (act.empty()) break;
        if ((rc = kc_eim_split_phase(h, act, s))) return rc;
        if ((rc = kc_eim_wait(h, s))) return rc;
        {
            const uint32_t* c3h = (const uint32_t*)h->pinned("eim.c3", 12ull * act.size());
            for (size_t q = 0; q < act.size(); ++q)
                for (int f = 0; f < 3; ++f) act[q]->hw[f] = c3h[3 * q + f];
        }
        bool wait_nu = false;
        for (KcEimLoop& P : L)
            if (!P.done) {
                if ((rc = kc_eim_front_phase(h, P, s))) return fail_at(P, rc);
                wait_nu = wait_nu || (P.passed && !P.whole && P.d <= KC_EXT_MAXD);
            }
        if (wait_nu) {
            if ((rc = kc_eim_wait(h, s))) return rc;
            bool wait_ref = false;
            for (KcEimLoop& P : L)
                if (!P.done && P.passed && !P.whole && P.d <= KC_EXT_MAXD) {
                    if ((rc = kc_eim_pass_refine(h, P, P.var, s))) return fail_at(P, rc);
                    wait_ref = wait_ref || P.refine;
                }
            if (wait_ref && (rc = kc_eim_wait(h, s))) return rc;
        }
        std::vector<KcEimLoop*> dec;
        for (KcEimLoop& P : L)
            if (!P.done) {
                if ((rc = kc_eim_keep_phase(h, P, s))) return fail_at(P, rc);
                if (P.passed) dec.push_back(&P);
            }
        if ((rc = kc_eim_compact_phase(h, dec, s))) return rc;
        if ((rc = kc_eim_wait(h, s))) return rc;
        if (!dec.empty()) {
            const uint32_t* o4h = (const uint32_t*)h->pinned("eim.k4", 16ull * dec.size());
            for (size_t q = 0; q < dec.size(); ++q)
                for (int f = 0; f < 4; ++f) dec[q]->hw[4 + f] = o4h[4 * q + f];
        }
        for (KcEimLoop& P : L)
            if (!P.done) kc_eim_end_iter(h, P);
    }
    for (KcEimLoop& P : L)
        if ((rc = kc_eim_form_c(h, P, s))) return fail_at(P, rc);
    return kc_eim_wait(h, s);
}

int kc_eim_sample_many(kc_handle* h, const kc_problem* probs, const std::vector<int>& ids,
                       std::vector<const uint32_t*>& C, std::vector<uint32_t>& nc,
                       hipStream_t s)
{
    std::vector<KcEimLoop> L(ids.size());
    uint32_t* hw = (uint32_t*)h->pinned("eim.hw", 32 * std::max<size_t>(ids.size(), 1));
    if (!hw) return h->fail(KC_ENOMEM, "pinned host allocation failed");
    h->eim_exact = 0;
    h->eim_refined = 0;
    for (size_t q = 0; q < ids.size(); ++q) {
        const kc_problem& p = probs[ids[q]];
        char pre[32];
        snprintf(pre, sizeof pre, "bL%zu.", q);
        L[q].id = ids[q];
        L[q].pre = pre;
        L[q].hw = hw + 8 * q;
        const int rc = kc_eim_init(h, L[q], &p.pts, p.k, &p.eim, nullptr, s);
        if (rc) return h->fail(rc, "problem %d: %s", ids[q], h->last_error.c_str());
    }
    const int rc = kc_eim_loops(h, L, s);
    if (rc) return rc;
    C.resize(ids.size());
    nc.resize(ids.size());
    for (size_t q = 0; q < ids.size(); ++q) {
        C[q] = L[q].H;
        nc[q] = L[q].hw[0];
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
    const hipStream_t s = (hipStream_t)stream;
    kc_validate_points(h, pts, s);
    const int d = pts->d;
    const float* X = pts->f32;
    const int64_t ld = pts->ld;

    std::vector<KcEimLoop> L(1);
    L[0].pre = "e.";
    L[0].hw = (uint32_t*)h->pinned("eim.hw", 32);
    if (!L[0].hw) return h->fail(KC_ENOMEM, "pinned host allocation failed");
    h->eim_exact = 0;
    h->eim_refined = 0;
    if ((rc = kc_eim_init(h, L[0], pts, k, prm, iters, s))) return rc;
    rc = kc_eim_loops(h, L, s);
    if (n_iters) *n_iters = L[0].it;
    if (rc) return rc;
    const uint32_t nc = L[0].hw[0];
    const uint32_t* Cidx = L[0].H;
    if (n_sample) *n_sample = nc;
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
