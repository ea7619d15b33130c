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

__global__ void k_or_status(const uint32_t* flag, uint32_t* status, uint32_t bit)
{
    if (threadIdx.x == 0 && *flag) atomicOr(status, bit);
}

void kc_or_status(const uint32_t* flag, uint32_t* status, uint32_t bit, hipStream_t s)
{
    hipLaunchKernelGGL(k_or_status, dim3(1), dim3(64), 0, s, flag, status, bit);
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
// [base, base+len); padding columns up to the next multiple of 64 get a copy
// of the segment's first point (harmless, they are masked from the argmax).

__global__ void k_stage_soa(const float* __restrict__ X, int64_t ld, int d,
                            uint64_t row0, uint32_t len, float* __restrict__ xs,
                            uint64_t stride, uint64_t base, uint32_t padded)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    uint64_t r = row0 + (i < len ? i : 0);
    const float* src = X + r * (uint64_t)ld;
    for (int j = 0; j < d; ++j) xs[(uint64_t)j * stride + base + i] = src[j];
}

void kc_stage_soa(const float* X, int64_t ld, int d, uint64_t row0, uint32_t len,
                  float* xs, uint64_t stride, uint64_t base, hipStream_t s)
{
    uint32_t padded = kc_pad64(len);
    if (padded == 0) return;
    hipLaunchKernelGGL(k_stage_soa, dim3((padded + 255) / 256), dim3(256), 0, s, X,
                       ld, d, row0, len, xs, stride, base, padded);
}

// ---------------------------------------------------------------------------
// streaming step: one block = 1024 consecutive points of one segment.

#define KC_STEP_PTS 4   // points per lane (one float4 per coordinate row)

template <int D>
__global__ __launch_bounds__(KC_BLOCK) void k_gon_step(
    const float* __restrict__ xs, uint64_t stride, int d_rt,
    float* __restrict__ mind, u64* __restrict__ keys,
    const KcSeg* __restrict__ segs, const uint32_t* __restrict__ blk_seg,
    const uint32_t* __restrict__ blk_start, int t)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ float cc[KC_MAXD];
    __shared__ u64 red[KC_BLOCK / 64];
    const uint32_t b = blockIdx.x;
    const KcSeg sg = segs[blk_seg[b]];
    if ((uint32_t)t >= sg.ksteps) return;
    uint32_t c;
    if (t == 0) {
        c = sg.first;
    } else {
        u64 prev = keys[sg.keyoff + t - 1];
        if ((prev >> 32) == 0) return;   // radius reached 0: segment finished
        c = kc_key_idx(prev);
    }
    for (int j = threadIdx.x; j < d; j += KC_BLOCK)
        cc[j] = xs[(uint64_t)j * stride + sg.base + c];
    __syncthreads();

    const uint32_t loc = blk_start[b] + threadIdx.x * KC_STEP_PTS;
    const uint64_t col = sg.base + loc;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    if (loc < sg.len) {
        if (D > 0) {
            float4 v[D > 0 ? D : 1];
#pragma unroll
            for (int j = 0; j < D; ++j)
                v[j] = *(const float4*)(xs + (uint64_t)j * stride + col);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float cj = cc[j];
                s0 = kc_d32_step(s0, v[j].x, cj);
                s1 = kc_d32_step(s1, v[j].y, cj);
                s2 = kc_d32_step(s2, v[j].z, cj);
                s3 = kc_d32_step(s3, v[j].w, cj);
            }
        } else {
#pragma unroll 4
            for (int j = 0; j < d; ++j) {
                float4 v = *(const float4*)(xs + (uint64_t)j * stride + col);
                const float cj = cc[j];
                s0 = kc_d32_step(s0, v.x, cj);
                s1 = kc_d32_step(s1, v.y, cj);
                s2 = kc_d32_step(s2, v.z, cj);
                s3 = kc_d32_step(s3, v.w, cj);
            }
        }
    }
    u64 key = 0;
    if (loc < sg.len) {
        float4 m = *(float4*)(mind + col);
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
    if (threadIdx.x == 0) atomicMax(&keys[sg.keyoff + t], key);
}

#define KC_STEP_CASE(DD)                                                          \
    case DD:                                                                      \
        hipLaunchKernelGGL(k_gon_step<DD>, dim3(nblk), dim3(KC_BLOCK), 0, s, xs,  \
                           stride, d, mind, keys, segs, blk_seg, blk_start, t);   \
        break;

void kc_gon_step(const float* xs, uint64_t stride, int d, float* mind, u64* keys,
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
                           d, mind, keys, segs, blk_seg, blk_start, t);
    }
}

// ---------------------------------------------------------------------------
// resident persistent engine: one segment, G blocks, PPT points per thread.
// Thread (g, tid) owns local points i = g*KC_BLOCK*PPT + p*KC_BLOCK + tid.
// arrive[t] counts blocks that finished step t; abort is raised by any block
// whose wait exceeds the spin limit, which ends every block's loop.

template <int D, int PPT>
__global__ __launch_bounds__(KC_BLOCK, 1) void k_gon_resident(
    const float* __restrict__ xs, uint64_t stride, uint64_t base, uint32_t len,
    uint32_t first, int k, float* __restrict__ mind, u64* __restrict__ keys,
    uint32_t* __restrict__ arrive, uint32_t* __restrict__ abort_flag,
    uint32_t spin_limit)
{
    __shared__ float cc[D];
    __shared__ u64 red[KC_BLOCK / 64];
    __shared__ u64 bkey;
    const uint32_t G = gridDim.x;
    const uint32_t i0 = blockIdx.x * (KC_BLOCK * PPT) + threadIdx.x;

    float x[PPT][D];
    float m[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint32_t i = i0 + p * KC_BLOCK;
        const uint32_t ii = i < len ? i : 0;
#pragma unroll
        for (int j = 0; j < D; ++j) x[p][j] = xs[(uint64_t)j * stride + base + ii];
        m[p] = __builtin_inff();
    }

    uint32_t c = first;
    int t = 0;
    for (; t < k; ++t) {
        if (threadIdx.x < D) cc[threadIdx.x] = xs[(uint64_t)threadIdx.x * stride + base + c];
        __syncthreads();
        u64 key = 0;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < D; ++j) s = kc_d32_step(s, x[p][j], cc[j]);
            m[p] = fminf(m[p], s);
            const uint32_t i = i0 + p * KC_BLOCK;
            if (i < len) key = kc_umax64(key, kc_pack(m[p], i));
        }
        key = kc_block_max64(key, red);
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_max(&keys[t], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&arrive[t], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t spins = 0;
            while (__hip_atomic_load(&arrive[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < G) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
                if (++spins > spin_limit) {
                    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            u64 kk = __hip_atomic_load(&keys[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                kk = 0;   // abandon: makes every block leave the loop
            bkey = kk;
        }
        __syncthreads();
        const u64 kk = bkey;
        __syncthreads();
        if ((kk >> 32) == 0) break;   // radius 0 (or abort): stop
        c = kc_key_idx(kk);
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint32_t i = i0 + p * KC_BLOCK;
        if (i < len) mind[base + i] = m[p];
    }
}

// Largest points-per-thread whose coordinates fit in about 192 VGPRs.
static int resident_ppt(int d)
{
    switch (d) {
    case 2: return 32;
    case 3: return 32;
    case 8: return 16;
    case 10: return 16;
    case 16: return 8;
    case 32: return 4;
    case 41: return 4;
    default: return 0;
    }
}

uint64_t kc_resident_capacity(int d, int max_blocks)
{
    return (uint64_t)resident_ppt(d) * KC_BLOCK * (uint64_t)max_blocks;
}

template <int D, int PPT>
static hipError_t launch_resident(uint32_t G, const float* xs, uint64_t stride,
                                  uint64_t base, uint32_t len, uint32_t first, int k,
                                  float* mind, u64* keys, uint32_t* arrive,
                                  uint32_t* abort_flag, uint32_t spin_limit, hipStream_t s)
{
    void* args[] = {(void*)&xs,   (void*)&stride, (void*)&base,  (void*)&len,
                    (void*)&first, (void*)&k,     (void*)&mind,  (void*)&keys,
                    (void*)&arrive, (void*)&abort_flag, (void*)&spin_limit};
    return hipLaunchCooperativeKernel((const void*)k_gon_resident<D, PPT>, dim3(G),
                                      dim3(KC_BLOCK), args, 0, s);
}

template <int D, int PPT>
static int max_resident_blocks()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gon_resident<D, PPT>,
                                                     KC_BLOCK, 0) != hipSuccess)
        return 0;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

int kc_resident_max_blocks(int d)
{
    switch (d) {
    case 2: return max_resident_blocks<2, 32>();
    case 3: return max_resident_blocks<3, 32>();
    case 8: return max_resident_blocks<8, 16>();
    case 10: return max_resident_blocks<10, 16>();
    case 16: return max_resident_blocks<16, 8>();
    case 32: return max_resident_blocks<32, 4>();
    case 41: return max_resident_blocks<41, 4>();
    default: return 0;
    }
}

// Returns hipSuccess, or an error when the shape has no resident kernel or
// the grid cannot be co-resident (the caller then streams instead).
hipError_t kc_gon_resident(int d, uint32_t G, const float* xs, uint64_t stride,
                           uint64_t base, uint32_t len, uint32_t first, int k, float* mind,
                           u64* keys, uint32_t* arrive, uint32_t* abort_flag,
                           uint32_t spin_limit, hipStream_t s)
{
    switch (d) {
#define KC_RES_CASE(DD, PP)                                                              \
    case DD:                                                                             \
        return launch_resident<DD, PP>(G, xs, stride, base, len, first, k, mind, keys,   \
                                       arrive, abort_flag, spin_limit, s);
        KC_RES_CASE(2, 32)
        KC_RES_CASE(3, 32)
        KC_RES_CASE(8, 16)
        KC_RES_CASE(10, 16)
        KC_RES_CASE(16, 8)
        KC_RES_CASE(32, 4)
        KC_RES_CASE(41, 4)
#undef KC_RES_CASE
    default:
        return hipErrorInvalidValue;
    }
}

uint32_t kc_resident_blocks_for(int d, uint32_t len)
{
    const uint64_t per = (uint64_t)resident_ppt(d) * KC_BLOCK;
    if (per == 0) return 0;
    return (uint32_t)((len + per - 1) / per);
}

// ---------------------------------------------------------------------------
// finishing: per segment n_chosen, centers, center coordinates, FP64 trace
// and exact FP64 radius.

// One thread per segment: n_chosen = first step whose key reached radius 0
// (+1), else ksteps; centers[keyoff + t] = reported index or -1.
__global__ void k_gon_finish_centers(const KcSeg* __restrict__ segs, int nseg,
                                     const u64* __restrict__ keys,
                                     int64_t* __restrict__ centers,
                                     int64_t* __restrict__ n_chosen,
                                     const int64_t* __restrict__ report_base,
                                     uint32_t kmax)
{
    int sidx = blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nseg) return;
    const KcSeg sg = segs[sidx];
    uint32_t nch = 0;
    if (sg.len > 0 && sg.ksteps > 0) {
        nch = sg.ksteps;
        for (uint32_t t = 0; t < sg.ksteps; ++t)
            if ((keys[sg.keyoff + t] >> 32) == 0) { nch = t + 1; break; }
    }
    const int64_t rb = report_base ? report_base[sidx] : 0;
    for (uint32_t t = 0; t < kmax && t < sg.ksteps; ++t) {
        int64_t v = -1;
        if (t < nch) v = rb + (int64_t)(t == 0 ? sg.first : kc_key_idx(keys[sg.keyoff + t - 1]));
        centers[sg.keyoff + t] = v;
    }
    n_chosen[sidx] = nch;
}

// ccoord[(keyoff + t) * d + j] = coordinate j of center t (FP32, compact).
__global__ void k_gon_gather_centers(const KcSeg* __restrict__ segs,
                                     const uint32_t* __restrict__ pairs_seg,
                                     const uint32_t* __restrict__ pairs_t, uint32_t npairs,
                                     const float* __restrict__ xs, uint64_t stride, int d,
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
    for (int j = 0; j < d; ++j) dst[j] = xs[(uint64_t)j * stride + sg.base + c];
}

// One wave per (segment, t): trace[keyoff+t] = sqrt(min_{j<=t} D64(c_{t+1}, c_j))
// for t < n_chosen-1 (the FP64 distance of the point chosen at step t to the
// centers before it); 0 for t >= n_chosen.  The last chosen step is written
// by the exact radius pass.
__global__ void k_gon_trace(const KcSeg* __restrict__ segs,
                            const uint32_t* __restrict__ pairs_seg,
                            const uint32_t* __restrict__ pairs_t, uint32_t npairs, int d,
                            const int64_t* __restrict__ n_chosen,
                            const float* __restrict__ ccoord, double* __restrict__ trace)
{
    const uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= npairs) return;
    const uint32_t sidx = pairs_seg[q];
    const KcSeg sg = segs[sidx];
    const uint32_t t = pairs_t[q];
    if (t >= sg.ksteps) return;
    const int64_t nch = n_chosen[sidx];
    if ((int64_t)t + 1 >= nch) {
        if ((int64_t)t >= nch && lane == 0) trace[sg.keyoff + t] = 0.0;
        return;
    }
    const float* a = ccoord + (uint64_t)(sg.keyoff + t + 1) * d;
    double best = __builtin_inf();
    for (uint32_t j = lane; j <= t; j += 64) {
        const float* cj = ccoord + (uint64_t)(sg.keyoff + j) * d;
        double s = 0.0;
        for (int u = 0; u < d; ++u) s = kc_d64_step(s, (double)a[u], (double)cj[u]);
        best = fmin(best, s);
    }
    best = kc_wave_min_f64(best);
    if (lane == 0) trace[sg.keyoff + t] = sqrt(best);
}

// Candidates for the exact radius: every point whose FP32 min-distance is at
// least M32 * (1 - 2 gamma - 4u), M32 the FP32 maximum after the last step.
// Such a band contains the exact maximiser (FP32 distances are within a
// relative gamma = gamma_{d+2} of the exact ones).  A segment whose FP32
// maximum is 0 has exact radius 0 and no candidates.
__global__ void k_gon_radius_cand(const KcSeg* __restrict__ segs,
                                  const uint32_t* __restrict__ blk_seg,
                                  const uint32_t* __restrict__ blk_start,
                                  const float* __restrict__ mind,
                                  const u64* __restrict__ keys,
                                  const int64_t* __restrict__ n_chosen, double band,
                                  u64* __restrict__ cand, uint32_t* __restrict__ ncand,
                                  uint32_t cap)
{
    const uint32_t b = blockIdx.x;
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

// One wave per candidate: exact FP64 min over the segment's chosen centers;
// radius2[seg] = max over candidates (as bits of a non-negative double).
__global__ void k_gon_radius_rescore(const KcSeg* __restrict__ segs,
                                     const u64* __restrict__ cand,
                                     const uint32_t* __restrict__ ncand, uint32_t cap,
                                     const float* __restrict__ xs, uint64_t stride, int d,
                                     const int64_t* __restrict__ n_chosen,
                                     const float* __restrict__ ccoord,
                                     double* __restrict__ radius2)
{
    const int lane = threadIdx.x & 63;
    uint32_t nc = *ncand;
    if (nc > cap) nc = cap;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t q = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); q < nc;
         q += waves) {
        const u64 e = cand[q];
        const uint32_t sidx = (uint32_t)(e >> 32), loc = (uint32_t)e;
        const KcSeg sg = segs[sidx];
        const int64_t nch = n_chosen[sidx];
        double best = __builtin_inf();
        for (int64_t j = lane; j < nch; j += 64) {
            const float* cj = ccoord + (uint64_t)(sg.keyoff + j) * d;
            double s = 0.0;
            for (int u = 0; u < d; ++u)
                s = kc_d64_step(s, (double)xs[(uint64_t)u * stride + sg.base + loc],
                                (double)cj[u]);
            best = fmin(best, s);
        }
        best = kc_wave_min_f64(best);
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
    const double r = sqrt(radius2[sidx]);
    if (nch > 0 && trace) trace[sg.keyoff + nch - 1] = r;
    if (radius_out) radius_out[sidx] = nch > 0 ? r : 0.0;
}

void kc_gon_finish(const KcGonRun& R, int64_t* centers, int64_t* n_chosen,
                   double* trace, double* radius_out, const int64_t* report_base,
                   hipStream_t s)
{
    const int nseg = R.nseg;
    hipLaunchKernelGGL(k_gon_finish_centers, dim3((nseg + 63) / 64), dim3(64), 0, s, R.segs,
                       nseg, R.keys, centers, n_chosen, report_base, R.kmax);
    hipLaunchKernelGGL(k_gon_gather_centers, dim3((R.npairs + 255) / 256), dim3(256), 0, s,
                       R.segs, R.pairs_seg, R.pairs_t, R.npairs, R.xs, R.stride, R.d, R.keys,
                       R.ccoord);
    if (trace)
        hipLaunchKernelGGL(k_gon_trace, dim3((R.npairs + 3) / 4), dim3(256), 0, s, R.segs,
                           R.pairs_seg, R.pairs_t, R.npairs, R.d, n_chosen, R.ccoord, trace);
    kc_fill_u32(R.ncand, 0u, 1, s);
    kc_fill_u64((u64*)R.radius2, 0ull, (uint64_t)nseg, s);
    hipLaunchKernelGGL(k_gon_radius_cand, dim3(R.nblk), dim3(KC_BLOCK), 0, s, R.segs,
                       R.blk_seg, R.blk_start, R.mind, R.keys, n_chosen, R.band, R.cand,
                       R.ncand, R.cand_cap);
    hipLaunchKernelGGL(k_gon_radius_rescore, dim3(1024), dim3(256), 0, s, R.segs, R.cand,
                       R.ncand, R.cand_cap, R.xs, R.stride, R.d, n_chosen, R.ccoord,
                       R.radius2);
    hipLaunchKernelGGL(k_gon_radius_finish, dim3((nseg + 63) / 64), dim3(64), 0, s, R.segs,
                       nseg, n_chosen, R.radius2, trace, radius_out);
}
