// kc_gon.hip -- Gonzalez's farthest-first traversal (Section 3.1) on gfx950.
//
// A run covers one or more independent segments (a whole problem, or one
// partition of MRG's first round, or one instance of a batch) that share a
// dimension d.  Points are staged once into a structure-of-arrays copy
//   xs[j * stride + base + i]   (coordinate j of local point i)
// whose segment bases are 64-aligned, so a wave reads each coordinate row
// with fully coalesced 16-byte loads.  Per point the run keeps mind[] (FP32
// squared distance to the nearest chosen center), per step t and segment one
// packed key keys[keyoff + t] (see kc_device.h).
//
// Two step engines:
//   k_gon_step      one launch per step t over every tile of every segment:
//                   update mind against the newest center, block argmax by
//                   wave shuffles + LDS, grid argmax by one 64-bit atomicMax
//                   per block.  HBM (or MALL) bound: reads d*4+4, writes 4
//                   bytes per point per step.
//   k_gon_resident  all steps in one cooperative launch for one segment that
//                   fits in registers: every thread keeps PPT points and their
//                   min-distances in VGPRs, and the grid meets once per step
//                   at a device-scope barrier.  Bound by VALU + barrier
//                   latency.
// After the steps, k_gon_finish* report centers, the FP64 radius trace and
// the exact FP64 covering radius (candidates within the FP32 error band of
// the FP32 maximum are rescored in FP64).
#include "kc_device.h"
#include "kc_internal.h"

// ---------------------------------------------------------------------------
// fills (graph-capture safe replacements for memset)

__global__ void k_fill_u64(u64* p, u64 v, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}


void kc_fill_u64(u64* p, u64 v, uint64_t n, hipStream_t s)
{
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}
void kc_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s)
{
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
}

// ---------------------------------------------------------------------------
// staging: rows [row0, row0+len) of a caller array [*][ld] -> SoA columns
// [base, base+len) of the FP32 copy and, when asked, of the BF16 copy with
// each point's rounding radius e = |bf16(x) - x| (FP64, rounded up).
// Padding columns up to the next multiple of 64 get a copy of the segment's
// first point (harmless, they are masked from every argmax).
//
// A block moves 64 points at a time through LDS, at most 64 coordinates per
// pass: the reads walk the rows in memory order and each wave's writes are
// 64 consecutive columns of one coordinate row, so both sides coalesce.

#define KC_STG_W 64   // coordinates per pass

// Stage the 64 columns [i0, i0+64) of one segment; all threads of the block
// call it.  sx, sb: LDS of 64 * (KC_STG_W + 1) entries.
// BF16 bits of x rounded to nearest, ties to even (finite x).
__device__ __forceinline__ uint16_t kc_stage_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// With xb and no Xb the BF16 copy is the FP32 rows rounded to nearest even
// (a library-made copy for the BF16 stream).
__device__ void kc_stage_tile64(const float* __restrict__ X, const uint16_t* __restrict__ Xb,
                                int64_t ld, int d, uint64_t row0, uint32_t len, uint32_t i0,
                                float* __restrict__ xs, uint16_t* __restrict__ xb,
                                float* __restrict__ ex, uint64_t stride, uint64_t base,
                                float* sx, uint16_t* sb)
{
    const bool bf = xb != nullptr;
    double ee = 0.0;   // thread p < 64: point i0 + p, coordinates in ascending order
    for (int j0 = 0; j0 < d; j0 += KC_STG_W) {
        const uint32_t w = (uint32_t)min(KC_STG_W, d - j0);
        const uint32_t pitch = w | 1u;   // odd: the transposed reads avoid bank conflicts
        for (uint32_t q = threadIdx.x; q < 64u * w; q += blockDim.x) {
            const uint32_t p = q / w, j = q - p * w;
            const uint32_t i = i0 + p;
            const uint64_t at = (row0 + (i < len ? i : 0)) * (uint64_t)ld + j0 + j;
            const float v = X[at];
            sx[p * pitch + j] = v;
            if (bf) sb[p * pitch + j] = Xb ? Xb[at] : kc_stage_bf16_rne(v);
        }
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < 64u * w; q += blockDim.x) {
            const uint32_t j = q >> 6, p = q & 63u;
            const uint64_t at = (uint64_t)(j0 + j) * stride + base + i0 + p;
            if (xs) xs[at] = sx[p * pitch + j];
            if (bf) xb[at] = sb[p * pitch + j];
        }
        if (bf && threadIdx.x < 64) {
            for (uint32_t j = 0; j < w; ++j) {
                const double e = (double)__uint_as_float((uint32_t)sb[threadIdx.x * pitch + j]
                                                         << 16) -
                                 (double)sx[threadIdx.x * pitch + j];
                ee += e * e;
            }
        }
        __syncthreads();
    }
    if (bf && threadIdx.x < 64)
        ex[base + i0 + threadIdx.x] = (float)(sqrt(ee) * (1.0 + 1e-12)) * (1.f + 1e-6f);
}

// One segment: block b stages columns [64b, 64b + 64).
__global__ __launch_bounds__(256) void k_stage_rows(
    const float* __restrict__ X, const uint16_t* __restrict__ Xb, int64_t ld, int d,
    uint64_t row0, uint32_t len, float* __restrict__ xs, uint16_t* __restrict__ xb,
    float* __restrict__ ex, uint64_t stride, uint64_t base)
{
    __shared__ float sx[64 * (KC_STG_W + 1)];
    __shared__ uint16_t sb[64 * (KC_STG_W + 1)];
    kc_stage_tile64(X, Xb, ld, d, row0, len, blockIdx.x * 64u, xs, xb, ex, stride, base, sx, sb);
}

// FP32 copy only, d and ld multiples of 4 and X 16-byte aligned: one 16-byte
// group of a row per thread, consecutive threads on consecutive groups (the
// reads coalesce with no LDS round trip), four scalar stores into four rows.
__device__ __forceinline__ void kc_stage_vec4(const float* __restrict__ X, int64_t ld, int d,
                                              uint64_t row0, uint32_t len, uint32_t st,
                                              uint32_t end, float* __restrict__ xs,
                                              uint64_t stride, uint64_t base)
{
    const uint32_t g4 = (uint32_t)d >> 2, items = (end - st) * g4;
    for (uint32_t q = threadIdx.x; q < items; q += blockDim.x) {
        const uint32_t i = st + q / g4, g = q - (q / g4) * g4;
        const float4 v = *(const float4*)(X + (row0 + (i < len ? i : 0)) * (uint64_t)ld + 4 * g);
        float* dst = xs + (uint64_t)(4 * g) * stride + base + i;
        dst[0] = v.x;
        dst[stride] = v.y;
        dst[2 * stride] = v.z;
        dst[3 * stride] = v.w;
    }
}

// Every segment of a planned run (all reading the same arrays): block b
// stages the `tile` columns from blk_start[b] of segment blk_seg[b].
__global__ __launch_bounds__(256) void k_stage_rows_batch(
    const float* __restrict__ X, const uint16_t* __restrict__ Xb, int64_t ld, int d,
    const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, uint32_t tile, float* __restrict__ xs,
    uint16_t* __restrict__ xb, float* __restrict__ ex, uint64_t stride, int vec4)
{
    __shared__ float sx[64 * (KC_STG_W + 1)];
    __shared__ uint16_t sb[64 * (KC_STG_W + 1)];
    const KcSeg sg = segs[blk_seg[blockIdx.x]];
    const uint32_t st = blk_start[blockIdx.x];
    const uint32_t padded = (sg.len + 63u) & ~63u;
    const uint32_t end = st + tile < padded ? st + tile : padded;
    if (vec4 && !xb) {
        kc_stage_vec4(X, ld, d, sg.src, sg.len, st, end, xs, stride, sg.base);
        return;
    }
    for (uint32_t i0 = st; i0 < end; i0 += 64)
        kc_stage_tile64(X, Xb, ld, d, sg.src, sg.len, i0, xs, xb, ex, stride, sg.base, sx, sb);
}

// Every segment of a planned run from its own source rows: block b stages
// the `tile` columns from blk_start[b] of segment blk_seg[b] (segments with
// no source are skipped).
__global__ __launch_bounds__(256) void k_stage_rows_src(
    const KcSrc* __restrict__ srcs, int bf, int d, const KcSeg* __restrict__ segs,
    const uint32_t* __restrict__ blk_seg, const uint32_t* __restrict__ blk_start, uint32_t tile,
    float* __restrict__ xs, uint16_t* __restrict__ xb, float* __restrict__ ex, uint64_t stride)
{
    __shared__ float sx[64 * (KC_STG_W + 1)];
    __shared__ uint16_t sb[64 * (KC_STG_W + 1)];
    const uint32_t q = blk_seg[blockIdx.x];
    const KcSrc src = srcs[q];
    if (!src.X) return;
    const KcSeg sg = segs[q];
    const uint32_t st = blk_start[blockIdx.x];
    const uint32_t padded = (sg.len + 63u) & ~63u;
    const uint32_t end = st + tile < padded ? st + tile : padded;
    for (uint32_t i0 = st; i0 < end; i0 += 64)
        kc_stage_tile64(src.X, bf ? src.Xb : nullptr, src.ld, d, sg.src, sg.len, i0, xs,
                        bf ? xb : nullptr, ex, stride, sg.base, sx, sb);
}

void kc_stage_rows_src(const KcSrc* srcs, bool bf, int d, const KcSeg* segs,
                       const uint32_t* blk_seg, const uint32_t* blk_start, uint32_t nblk,
                       uint32_t tile, float* xs, uint16_t* xb, float* ex, uint64_t stride,
                       hipStream_t s)
{
    if (nblk == 0) return;
    hipLaunchKernelGGL(k_stage_rows_src, dim3(nblk), dim3(256), 0, s, srcs, (int)bf, d, segs,
                       blk_seg, blk_start, tile, xs, xb, ex, stride);
}

void kc_stage_rows(const float* X, const uint16_t* Xb, int64_t ld, int d, uint64_t row0,
                   uint32_t len, float* xs, uint16_t* xb, float* ex, uint64_t stride,
                   uint64_t base, hipStream_t s)
{
    const uint32_t padded = kc_pad64(len);
    if (padded == 0) return;
    hipLaunchKernelGGL(k_stage_rows, dim3(padded / 64), dim3(256), 0, s, X, Xb, ld, d, row0, len,
                       xs, xb, ex, stride, base);
}

void kc_stage_soa(const float* X, int64_t ld, int d, uint64_t row0, uint32_t len,
                  float* xs, uint64_t stride, uint64_t base, hipStream_t s)
{
    kc_stage_rows(X, nullptr, ld, d, row0, len, xs, nullptr, nullptr, stride, base, s);
}

void kc_stage_rows_batch(const float* X, const uint16_t* Xb, int64_t ld, int d,
                         const KcSeg* segs, const uint32_t* blk_seg, const uint32_t* blk_start,
                         uint32_t nblk, uint32_t tile, float* xs, uint16_t* xb, float* ex,
                         uint64_t stride, hipStream_t s)
{
    if (nblk == 0) return;
    const int vec4 = d % 4 == 0 && ld % 4 == 0 && ((uintptr_t)X & 15) == 0;
    hipLaunchKernelGGL(k_stage_rows_batch, dim3(nblk), dim3(256), 0, s, X, Xb, ld, d, segs,
                       blk_seg, blk_start, tile, xs, xb, ex, stride, vec4);
}

// ---------------------------------------------------------------------------
// streaming step: one block = 1024 consecutive points of one segment.

#define KC_STEP_PTS 4   // points per lane (one float4 per coordinate row)

template <int D>
__global__ __launch_bounds__(KC_BLOCK) void k_gon_step(
    const float* __restrict__ xs, uint64_t stride, int d_rt,
    float* __restrict__ mind, u64* __restrict__ part,
    const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, int t)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ u64 red[KC_BLOCK / 64];
    const uint32_t b = blockIdx.x;
    const KcSeg sg = segs[blk_seg[b]];
    if ((uint32_t)t >= sg.ksteps) return;
    const uint32_t loc = blk_start[b] + threadIdx.x * KC_STEP_PTS;
    const uint64_t col = sg.base + loc;
    const bool live = loc < sg.len;

    // The min-distances load first; the center is resolved next (every wave
    // on its own from the previous step's partial keys, no barrier); the
    // coordinate rows then stream two at a time, which keeps few VGPRs per
    // lane and many waves per SIMD in flight.
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live) m = *(const float4*)(mind + col);
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
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (live) {
        constexpr int CH = 2;   // coordinate rows per pass
#pragma unroll 1
        for (int j0 = 0; j0 < d; j0 += CH) {
            float4 w[CH];
            float cc[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (j0 + u < d) {
                    w[u] = *(const float4*)(xs + (uint64_t)(j0 + u) * stride + col);
                    cc[u] = xc[(uint64_t)(j0 + u) * stride];
                }
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (j0 + u < d) {
                    s0 = kc_d32_step(s0, w[u].x, cc[u]);
                    s1 = kc_d32_step(s1, w[u].y, cc[u]);
                    s2 = kc_d32_step(s2, w[u].z, cc[u]);
                    s3 = kc_d32_step(s3, w[u].w, cc[u]);
                }
        }
    }
    u64 key = 0;
    if (live) {
        m.x = fminf(m.x, s0);
        m.y = fminf(m.y, s1);
        m.z = fminf(m.z, s2);
        m.w = fminf(m.w, s3);
        *(float4*)(mind + col) = m;
        key = kc_pack(m.x, loc);
        if (loc + 1 < sg.len) key = kc_umax64(key, kc_pack(m.y, loc + 1));
        if (loc + 2 < sg.len) key = kc_umax64(key, kc_pack(m.z, loc + 2));
        if (loc + 3 < sg.len) key = kc_umax64(key, kc_pack(m.w, loc + 3));
    }
    key = kc_block_max64(key, red);
    if (threadIdx.x == 0) kc_part_offer(part, sg.keyoff + t, b % KC_PARTS, key);
}

// keys[q] = max over the partial slots of key q, for every key of a run.
__global__ void k_part_collect(const u64* __restrict__ part, u64* __restrict__ keys,
                               uint64_t nkeys)
{
    const uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (q >= nkeys) return;
    u64 v = 0;
    for (uint32_t s = 0; s < KC_PARTS; ++s) {
        const u64 x = part[(q * KC_PARTS + s) * KC_PSTRIDE];
        v = x > v ? x : v;
    }
    keys[q] = v;
}

void kc_part_collect(const u64* part, u64* keys, uint64_t nkeys, hipStream_t s)
{
    if (nkeys == 0) return;
    hipLaunchKernelGGL(k_part_collect, dim3((unsigned)((nkeys + 255) / 256)), dim3(256), 0, s,
                       part, keys, nkeys);
}

#define KC_STEP_CASE(DD)                                                          \
    case DD:                                                                      \
        hipLaunchKernelGGL(k_gon_step<DD>, dim3(nblk), dim3(KC_BLOCK), 0, s, xs,  \
                           stride, d, mind, part, segs, blk_seg, blk_start, t);   \
        break;

void kc_gon_step(const float* xs, uint64_t stride, int d, float* mind, u64* part,
                 const KcSeg* segs, const uint32_t* blk_seg, const uint32_t* blk_start,
                 uint32_t nblk, int t, hipStream_t s)
{
    switch (d) {
        KC_STEP_CASE(2)
        KC_STEP_CASE(3)
        KC_STEP_CASE(8)
        KC_STEP_CASE(10)
        KC_STEP_CASE(16)
        KC_STEP_CASE(32)
        KC_STEP_CASE(41)
    default:
        hipLaunchKernelGGL(k_gon_step<0>, dim3(nblk), dim3(KC_BLOCK), 0, s, xs, stride,
                           d, mind, part, segs, blk_seg, blk_start, t);
    }
}

// ---------------------------------------------------------------------------
// finishing: per segment n_chosen, centers, center coordinates, FP64 trace
// and exact FP64 radius.

// The finishing kernels are latency-bound (a few hundred waves): every copy
// keeps eight loads in flight, and every FP64 minimum runs two independent
// chains per lane.

// dst[j] = src(j) for the d coordinates of one point.
template <class F>
__device__ __forceinline__ void kc_copy_coords(float* __restrict__ dst, int d, F src)
{
    for (int j0 = 0; j0 < d; j0 += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = j0 + u < d ? src(j0 + u) : 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < d) dst[j0 + u] = v[u];
    }
}

// sC[e] = C[e] for e < N, by the whole block.
__device__ __forceinline__ void kc_fill_lds(float* sC, const float* __restrict__ C, uint32_t N)
{
    for (uint32_t e0 = threadIdx.x; e0 < N; e0 += 8 * blockDim.x) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t e = e0 + u * blockDim.x;
            v[u] = e < N ? C[e] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t e = e0 + u * blockDim.x;
            if (e < N) sC[e] = v[u];
        }
    }
}

// Wave minimum over rows j < nc of C (d floats each) of the FP64 squared
// distance from point P: lane l takes rows l, l+64, ..., two rows per pass.
// Each distance sums separately rounded squares in coordinate order.
__device__ __forceinline__ double kc_min_d64(const float* P, const float* C, int64_t nc, int d)
{
    const int lane = threadIdx.x & 63;
    double best = __builtin_inf();
    for (int64_t j = lane; j < nc; j += 128) {
        const bool two = j + 64 < nc;
        const float* c0 = C + (uint64_t)j * d;
        const float* c1 = two ? c0 + 64ull * (uint64_t)d : c0;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
        for (int u = 0; u < d; ++u) {
            const double x = (double)P[u];
            s0 = kc_d64_step(s0, x, (double)c0[u]);
            s1 = kc_d64_step(s1, x, (double)c1[u]);
        }
        best = fmin(best, s0);
        if (two) best = fmin(best, s1);
    }
    return kc_wave_min_f64(best);
}

// The calling wave copies point `loc` of segment sg (rows xa of lda floats
// from the segment's src, else the SoA copy xs) into P; then P is readable
// by every lane of the wave.
__device__ __forceinline__ void kc_wave_point(float* P, const KcSeg& sg, uint32_t loc,
                                              const float* __restrict__ xs, uint64_t stride,
                                              int d, const float* __restrict__ xa, int64_t lda)
{
    const int lane = threadIdx.x & 63;
    float v[KC_MAXD / 64];
#pragma unroll
    for (int q = 0; q < KC_MAXD / 64; ++q) {
        const int u = q * 64 + lane;
        v[q] = u >= d ? 0.f
                      : xa ? xa[(sg.src + loc) * (uint64_t)lda + u]
                           : xs[(uint64_t)u * stride + sg.base + loc];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < KC_MAXD / 64; ++q)
        if (q * 64 + lane < d) P[q * 64 + lane] = v[q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// n_chosen of a segment = 1 + the first step whose key reached radius 0, else
// ksteps (0 for an empty segment): initialised per segment, then lowered by
// one thread per (segment, step).  Also clears the exact-radius accumulators.
__global__ void k_gon_nchosen_init(const KcSeg* __restrict__ segs, int nseg,
                                   int64_t* __restrict__ n_chosen, uint32_t* __restrict__ ncand,
                                   double* __restrict__ radius2)
{
    int sidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx == 0) *ncand = 0;
    if (sidx >= nseg) return;
    const KcSeg sg = segs[sidx];
    n_chosen[sidx] = (sg.len > 0) ? (int64_t)sg.ksteps : 0;
    radius2[sidx] = 0.0;
}

__global__ void k_gon_nchosen_min(const KcSeg* __restrict__ segs,
                                  const uint32_t* __restrict__ pairs_seg,
                                  const uint32_t* __restrict__ pairs_t, uint32_t npairs,
                                  const u64* __restrict__ keys, int64_t* __restrict__ n_chosen)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const uint32_t sidx = pairs_seg[q];
    const KcSeg sg = segs[sidx];
    const uint32_t t = pairs_t[q];
    if ((keys[sg.keyoff + t] >> 32) == 0)
        atomicMin((long long*)&n_chosen[sidx], (long long)(t + 1));
}

// centers[keyoff + t] = reported index of center t, or -1 past n_chosen.
__global__ void k_gon_centers_out(const KcSeg* __restrict__ segs,
                                  const uint32_t* __restrict__ pairs_seg,
                                  const uint32_t* __restrict__ pairs_t, uint32_t npairs,
                                  const u64* __restrict__ keys,
                                  const int64_t* __restrict__ n_chosen,
                                  const int64_t* __restrict__ report_base,
                                  const int64_t* __restrict__ remap,
                                  int64_t* __restrict__ centers)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const uint32_t sidx = pairs_seg[q];
    const KcSeg sg = segs[sidx];
    const uint32_t t = pairs_t[q];
    int64_t v = -1;
    if ((int64_t)t < n_chosen[sidx]) {
        const uint32_t loc = t == 0 ? sg.first : kc_key_idx(keys[sg.keyoff + t - 1]);
        if (remap)
            v = remap[sg.src + loc];
        else
            v = (report_base ? report_base[sidx] : 0) + (int64_t)loc;
    }
    centers[sg.keyoff + t] = v;
}

// ccoord[(keyoff + t) * d + j] = coordinate j of center t (FP32, compact).
__global__ void k_gon_gather_centers(const KcSeg* __restrict__ segs,
                                     const uint32_t* __restrict__ pairs_seg,
                                     const uint32_t* __restrict__ pairs_t, uint32_t npairs,
                                     const float* __restrict__ xs, uint64_t stride, int d,
                                     const float* __restrict__ xa, int64_t lda,
                                     const u64* __restrict__ keys,
                                     float* __restrict__ ccoord)
{
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npairs) return;
    const KcSeg sg = segs[pairs_seg[q]];
    const uint32_t t = pairs_t[q];
    if (t >= sg.ksteps) return;
    uint32_t c;
    if (t == 0) {
        c = sg.first;
    } else {
        u64 prev = keys[sg.keyoff + t - 1];
        if ((prev >> 32) == 0) return;
        c = kc_key_idx(prev);
    }
    float* dst = ccoord + (uint64_t)(sg.keyoff + t) * d;
    if (xa) {
        const float* row = xa + (sg.src + c) * (uint64_t)lda;
        kc_copy_coords(dst, d, [&](int j) { return row[j]; });
    } else {
        kc_copy_coords(dst, d, [&](int j) { return xs[(uint64_t)j * stride + sg.base + c]; });
    }
}

// One wave per (segment, t): trace[keyoff+t] = sqrt(min_{j<=t} D64(c_{t+1}, c_j))
// for t < n_chosen-1 (the FP64 distance of the point chosen at step t to the
// centers before it); 0 for t >= n_chosen.  The last chosen step is written
// by the exact radius pass.
__device__ __forceinline__ void kc_trace_wave(const KcSeg& sg, uint32_t t, int64_t nch, int d,
                                              const float* __restrict__ ccoord,
                                              double* __restrict__ trace)
{
    const int lane = threadIdx.x & 63;
    if ((int64_t)t + 1 >= nch) {
        if ((int64_t)t >= nch && lane == 0) trace[sg.keyoff + t] = 0.0;
        return;
    }
    const float* C = ccoord + (uint64_t)sg.keyoff * d;
    const double best = kc_min_d64(C + (uint64_t)(t + 1) * d, C, (int64_t)t + 1, d);
    if (lane == 0) trace[sg.keyoff + t] = kc_sqrt_rn(best);
}

__global__ void k_gon_trace(const KcSeg* __restrict__ segs,
                            const uint32_t* __restrict__ pairs_seg,
                            const uint32_t* __restrict__ pairs_t, uint32_t npairs, int d,
                            const int64_t* __restrict__ n_chosen,
                            const float* __restrict__ ccoord, double* __restrict__ trace)
{
    const uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (q >= npairs) return;
    const uint32_t sidx = pairs_seg[q];
    const KcSeg sg = segs[sidx];
    const uint32_t t = pairs_t[q];
    if (t >= sg.ksteps) return;
    kc_trace_wave(sg, t, n_chosen[sidx], d, ccoord, trace);
}

// Candidates for the exact radius: every point whose FP32 min-distance is at
// least M32 * (1 - 2 gamma - 4u), M32 the FP32 maximum after the last step.
// Such a band contains the exact maximiser (FP32 distances are within a
// relative gamma = gamma_{d+2} of the exact ones).  A segment whose FP32
// maximum is 0 has exact radius 0 and no candidates.
__device__ __forceinline__ void kc_radius_cand_block(
    uint32_t b, const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, const float* __restrict__ mind,
    const u64* __restrict__ keys, const int64_t* __restrict__ n_chosen, double band,
    u64* __restrict__ cand, uint32_t* __restrict__ ncand, uint32_t cap)
{
    const uint32_t sidx = blk_seg[b];
    const KcSeg sg = segs[sidx];
    const int64_t nch = n_chosen[sidx];
    if (nch <= 0) return;
    const float M = kc_key_val(keys[sg.keyoff + nch - 1]);
    if (M == 0.f) return;
    const double thr = (double)M * (1.0 - band);
    for (uint32_t p = 0; p < KC_STEP_PTS; ++p) {
        const uint32_t loc = blk_start[b] + p * KC_BLOCK + threadIdx.x;
        if (loc >= sg.len) continue;
        if ((double)mind[sg.base + loc] >= thr) {
            uint32_t slot = atomicAdd(ncand, 1u);
            if (slot < cap) cand[slot] = ((u64)sidx << 32) | loc;
        }
    }
}

__global__ void k_gon_radius_cand(const KcSeg* __restrict__ segs,
                                  const uint32_t* __restrict__ blk_seg,
                                  const uint32_t* __restrict__ blk_start,
                                  const float* __restrict__ mind,
                                  const u64* __restrict__ keys,
                                  const int64_t* __restrict__ n_chosen, double band,
                                  u64* __restrict__ cand, uint32_t* __restrict__ ncand,
                                  uint32_t cap)
{
    kc_radius_cand_block(blockIdx.x, segs, blk_seg, blk_start, mind, keys, n_chosen, band, cand,
                         ncand, cap);
}

// ---- one segment reported as is (no remap or base): three launches.
// Center coordinates are staged in LDS when k*d floats fit KC_FIN1_LDS.
#define KC_FIN1_LDS 12288

// n_chosen (every block scans the keys), the accumulator resets, and the
// centers and center coordinates of this block's 256 steps.
__global__ __launch_bounds__(256) void k_gon_fin1_head(
    const KcSeg* __restrict__ segs, const u64* __restrict__ keys, int64_t* __restrict__ n_chosen,
    uint32_t* __restrict__ ncand, uint32_t* __restrict__ ticket, double* __restrict__ radius2,
    int64_t* __restrict__ centers, float* __restrict__ ccoord, const float* __restrict__ xs,
    uint64_t stride, int d, const float* __restrict__ xa, int64_t lda)
{
    __shared__ int s_nch;
    const KcSeg sg = segs[0];
    if (threadIdx.x == 0) s_nch = sg.len > 0 ? (int)sg.ksteps : 0;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < sg.ksteps; t += blockDim.x)
        if ((keys[sg.keyoff + t] >> 32) == 0) atomicMin(&s_nch, (int)t + 1);
    __syncthreads();
    const int nch = s_nch;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        n_chosen[0] = nch;
        *ncand = 0;
        *ticket = 0;
        radius2[0] = 0.0;
    }
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= sg.ksteps) return;
    int64_t v = -1;
    if ((int)t < nch) {
        const uint32_t c = t == 0 ? sg.first : kc_key_idx(keys[sg.keyoff + t - 1]);
        v = c;
        float* dst = ccoord + (uint64_t)(sg.keyoff + t) * d;
        if (xa) {
            const float* row = xa + (sg.src + c) * (uint64_t)lda;
            kc_copy_coords(dst, d, [&](int j) { return row[j]; });
        } else {
            kc_copy_coords(dst, d, [&](int j) { return xs[(uint64_t)j * stride + sg.base + c]; });
        }
    }
    centers[sg.keyoff + t] = v;
}

// trace[t] of one wave from centers C (rows of d floats)
template <bool LDS>
__device__ __forceinline__ void kc_trace_wave_c(uint32_t t, int64_t nch, int d,
                                                const float* __restrict__ C,
                                                double* __restrict__ trace)
{
    const int lane = threadIdx.x & 63;
    if ((int64_t)t + 1 >= nch) {
        if ((int64_t)t >= nch && lane == 0) trace[t] = 0.0;
        return;
    }
    const double best = kc_min_d64(C + (uint64_t)(t + 1) * d, C, (int64_t)t + 1, d);
    if (lane == 0) trace[t] = kc_sqrt_rn(best);
}

// Blocks [0, tb) compute the FP64 trace (four steps per block), blocks
// [tb, tb + nblk) list the exact-radius candidates of their tile.
__global__ __launch_bounds__(KC_BLOCK) void k_gon_fin1_mid(
    const KcSeg* __restrict__ segs, uint32_t tb, int d, const int64_t* __restrict__ n_chosen,
    const float* __restrict__ ccoord, double* __restrict__ trace, int use_lds,
    const uint32_t* __restrict__ blk_seg, const uint32_t* __restrict__ blk_start,
    const float* __restrict__ mind, const u64* __restrict__ keys, double band,
    u64* __restrict__ cand, uint32_t* __restrict__ ncand, uint32_t cap)
{
    extern __shared__ float sC[];
    if (blockIdx.x < tb) {
        if (!trace) return;
        const KcSeg sg = segs[0];
        const int64_t nch = n_chosen[0];
        const float* C = ccoord + (uint64_t)sg.keyoff * d;
        double* tr = trace + sg.keyoff;
        const uint32_t t = blockIdx.x * (KC_BLOCK / 64) + (threadIdx.x >> 6);
        if (use_lds) {
            // rows 0..t+1 of this block's last step
            const uint32_t rows = min((uint32_t)nch, (blockIdx.x + 1) * (KC_BLOCK / 64) + 1);
            kc_fill_lds(sC, C, rows * (uint32_t)d);
            __syncthreads();
            if (t < sg.ksteps) kc_trace_wave_c<true>(t, nch, d, sC, tr);
        } else if (t < sg.ksteps) {
            kc_trace_wave_c<false>(t, nch, d, C, tr);
        }
    } else {
        kc_radius_cand_block(blockIdx.x - tb, segs, blk_seg, blk_start, mind, keys, n_chosen,
                             band, cand, ncand, cap);
    }
}

// Exact FP64 radius over the candidates (one wave per candidate, centers in
// LDS when they fit); the last block to finish writes sqrt(radius2) to the
// trace's last chosen step and to radius_out.
__global__ __launch_bounds__(KC_BLOCK) void k_gon_fin1_rescore(
    const KcSeg* __restrict__ segs, const u64* __restrict__ cand,
    const uint32_t* __restrict__ ncand, uint32_t cap, const float* __restrict__ xs,
    uint64_t stride, int d, const float* __restrict__ xa, int64_t lda,
    const int64_t* __restrict__ n_chosen, const float* __restrict__ ccoord, int use_lds,
    double* __restrict__ radius2, uint32_t* __restrict__ ticket, double* __restrict__ trace,
    double* __restrict__ radius_out)
{
    extern __shared__ float sC[];
    __shared__ float sP[KC_BLOCK / 64][KC_MAXD];   // each wave's candidate point
    __shared__ int s_last;
    const int lane = threadIdx.x & 63;
    const KcSeg sg = segs[0];
    const int64_t nch = n_chosen[0];
    uint32_t nc = *ncand;
    if (nc > cap) nc = cap;
    const float* C = ccoord + (uint64_t)sg.keyoff * d;
    if (use_lds && nc > blockIdx.x * (KC_BLOCK / 64)) {
        kc_fill_lds(sC, C, (uint32_t)nch * (uint32_t)d);
        __syncthreads();
        C = sC;
    }
    float* P = sP[threadIdx.x >> 6];
    const uint32_t waves = gridDim.x * (KC_BLOCK / 64);
    for (uint32_t q = blockIdx.x * (KC_BLOCK / 64) + (threadIdx.x >> 6); q < nc; q += waves) {
        kc_wave_point(P, sg, (uint32_t)cand[q], xs, stride, d, xa, lda);
        const double best = kc_min_d64(P, C, nch, d);
        if (lane == 0) kc_atomic_max_f64_nonneg(&radius2[0], best);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (s_last && threadIdx.x == 0) {
        __threadfence();
        const u64 bits = __hip_atomic_load((const u64*)radius2, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        const double r = kc_sqrt_rn(__longlong_as_double((long long)bits));
        if (nch > 0 && trace) trace[sg.keyoff + nch - 1] = r;
        if (radius_out) radius_out[0] = nch > 0 ? r : 0.0;
    }
}

// One wave per candidate: exact FP64 min over the segment's chosen centers;
// radius2[seg] = max over candidates (as bits of a non-negative double).
__global__ __launch_bounds__(KC_BLOCK) void k_gon_radius_rescore(const KcSeg* __restrict__ segs,
                                     const u64* __restrict__ cand,
                                     const uint32_t* __restrict__ ncand, uint32_t cap,
                                     const float* __restrict__ xs, uint64_t stride, int d,
                                     const float* __restrict__ xa, int64_t lda,
                                     const int64_t* __restrict__ n_chosen,
                                     const float* __restrict__ ccoord,
                                     double* __restrict__ radius2)
{
    __shared__ float sP[KC_BLOCK / 64][KC_MAXD];   // each wave's candidate point
    const int lane = threadIdx.x & 63;
    uint32_t nc = *ncand;
    if (nc > cap) nc = cap;
    float* P = sP[threadIdx.x >> 6];
    const uint32_t waves = gridDim.x * (KC_BLOCK / 64);
    for (uint32_t q = blockIdx.x * (KC_BLOCK / 64) + (threadIdx.x >> 6); q < nc; q += waves) {
        const u64 e = cand[q];
        const uint32_t sidx = (uint32_t)(e >> 32), loc = (uint32_t)e;
        const KcSeg sg = segs[sidx];
        kc_wave_point(P, sg, loc, xs, stride, d, xa, lda);
        const double best = kc_min_d64(P, ccoord + (uint64_t)sg.keyoff * d, n_chosen[sidx], d);
        if (lane == 0) kc_atomic_max_f64_nonneg(&radius2[sidx], best);
    }
}

// trace[keyoff + n_chosen - 1] = sqrt(radius2); radius_out[seg] likewise.
__global__ void k_gon_radius_finish(const KcSeg* __restrict__ segs, int nseg,
                                    const int64_t* __restrict__ n_chosen,
                                    const double* __restrict__ radius2,
                                    double* __restrict__ trace, double* __restrict__ radius_out)
{
    int sidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nseg) return;
    const KcSeg sg = segs[sidx];
    const int64_t nch = n_chosen[sidx];
    const double r = kc_sqrt_rn(radius2[sidx]);
    if (nch > 0 && trace) trace[sg.keyoff + nch - 1] = r;
    if (radius_out) radius_out[sidx] = nch > 0 ? r : 0.0;
}

void kc_gon_finish_impl(const KcGonRun& R, int64_t* centers, int64_t* n_chosen,
                        double* trace, double* radius_out, const int64_t* report_base,
                        const int64_t* remap, bool gather, hipStream_t s,
                        const std::function<void(hipStream_t)>& radius_cand)
{
    const int nseg = R.nseg;
    const dim3 pg((R.npairs + 255) / 256);
    hipLaunchKernelGGL(k_gon_nchosen_init, dim3((nseg + 63) / 64), dim3(64), 0, s, R.segs,
                       nseg, n_chosen, R.ncand, R.radius2);
    if (R.npairs > 0) {
        hipLaunchKernelGGL(k_gon_nchosen_min, pg, dim3(256), 0, s, R.segs, R.pairs_seg,
                           R.pairs_t, R.npairs, R.keys, n_chosen);
        hipLaunchKernelGGL(k_gon_centers_out, pg, dim3(256), 0, s, R.segs, R.pairs_seg,
                           R.pairs_t, R.npairs, R.keys, n_chosen, report_base, remap,
                           centers);
        if (gather)
            hipLaunchKernelGGL(k_gon_gather_centers, pg, dim3(256), 0, s, R.segs, R.pairs_seg,
                               R.pairs_t, R.npairs, R.xs, R.stride, R.d, R.xa, R.lda, R.keys,
                               R.ccoord);
        if (trace)
            hipLaunchKernelGGL(k_gon_trace, dim3((R.npairs + 3) / 4), dim3(256), 0, s, R.segs,
                               R.pairs_seg, R.pairs_t, R.npairs, R.d, n_chosen, R.ccoord,
                               trace);
    }
    if (R.nblk > 0) radius_cand(s);
    hipLaunchKernelGGL(k_gon_radius_rescore, dim3(1024), dim3(256), 0, s, R.segs, R.cand,
                       R.ncand, R.cand_cap, R.xs, R.stride, R.d, R.xa, R.lda, n_chosen,
                       R.ccoord, R.radius2);
    hipLaunchKernelGGL(k_gon_radius_finish, dim3((nseg + 63) / 64), dim3(64), 0, s, R.segs,
                       nseg, n_chosen, R.radius2, trace, radius_out);
}

void kc_gon_finish(const KcGonRun& R, int64_t* centers, int64_t* n_chosen,
                   double* trace, double* radius_out, const int64_t* report_base,
                   const int64_t* remap, hipStream_t s)
{
    if (R.nseg == 1 && !report_base && !remap) {
        // one segment: 3 launches instead of 9
        const uint32_t kst = R.npairs;   // steps of the one segment
        const int use_lds = (uint64_t)kst * R.d <= KC_FIN1_LDS;
        const size_t lds = use_lds ? sizeof(float) * (size_t)kst * R.d : 0;
        if (kst > 0)
            hipLaunchKernelGGL(k_gon_fin1_head, dim3((kst + 255) / 256), dim3(256), 0, s, R.segs,
                               R.keys, n_chosen, R.ncand, R.ticket, R.radius2, centers, R.ccoord,
                               R.xs, R.stride, R.d, R.xa, R.lda);
        const uint32_t tb = (kst + KC_BLOCK / 64 - 1) / (KC_BLOCK / 64);
        if (tb + R.nblk > 0)
            hipLaunchKernelGGL(k_gon_fin1_mid, dim3(tb + R.nblk), dim3(KC_BLOCK), lds, s, R.segs,
                               tb, R.d, n_chosen, R.ccoord, trace, use_lds, R.blk_seg,
                               R.blk_start, R.mind, R.keys, R.band, R.cand, R.ncand, R.cand_cap);
        hipLaunchKernelGGL(k_gon_fin1_rescore, dim3(256), dim3(KC_BLOCK), lds, s, R.segs, R.cand,
                           R.ncand, R.cand_cap, R.xs, R.stride, R.d, R.xa, R.lda, n_chosen,
                           R.ccoord, use_lds, R.radius2, R.ticket, trace, radius_out);
        return;
    }
    kc_gon_finish_impl(R, centers, n_chosen, trace, radius_out, report_base, remap, true, s,
                       [&](hipStream_t st) {
                           hipLaunchKernelGGL(k_gon_radius_cand, dim3(R.nblk), dim3(KC_BLOCK),
                                              0, st, R.segs, R.blk_seg, R.blk_start, R.mind,
                                              R.keys, n_chosen, R.band, R.cand, R.ncand,
                                              R.cand_cap);
                       });
}
