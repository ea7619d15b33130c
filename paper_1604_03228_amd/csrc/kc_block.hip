// kc_block.hip -- Gonzalez's traversal (Section 3.1) in one workgroup, for
// inputs small enough that every point fits the registers of its 1,024
// lanes.  At that size a step costs its latency -- apply the new center,
// find the farthest point -- and one block pays it without any exchange
// between workgroups: the argmax is a DPP reduction per wave and one LDS
// round between the sixteen waves, and the new center's coordinates come
// from the lane that holds the point.  Same canonical FP32 distances, keys
// and tie rule (largest value, then lowest index) as the other engines.
#include "kc_host.h"

#define KC_BK_THREADS 1024
#define KC_BK_WAVES (KC_BK_THREADS / 64)

// keys[t], t < k: the packed key of the farthest point after centers 0..t
// (its min-distance to them, its index) -- center t+1 for t < k-1; zero
// from the step where every point coincides with a center.  mind[i]: point
// i's min-distance to all chosen centers.
template <int D, int PPT>
__global__ __launch_bounds__(KC_BK_THREADS, 1) void k_gon_block(const float* __restrict__ X,
                                                              int64_t ld, uint32_t n,
                                                              uint32_t first, int k,
                                                              float* __restrict__ mind,
                                                              u64* __restrict__ keys)
{
    __shared__ float sc[D];                 // the current center's coordinates
    __shared__ u64 sred[KC_BK_WAVES];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    float x[PPT][D];
    float m[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint32_t i = tid + (uint32_t)p * KC_BK_THREADS;
        const uint64_t r = i < n ? i : 0u;
#pragma unroll
        for (int j = 0; j < D; ++j) x[p][j] = X[r * (uint64_t)ld + j];
        m[p] = __builtin_inff();
    }
    if (tid < D) sc[tid] = X[(uint64_t)first * (uint64_t)ld + tid];
    __syncthreads();
    for (int t = 0;; ++t) {
        float c[D];
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = sc[j];
        u64 best = 0;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const uint32_t i = tid + (uint32_t)p * KC_BK_THREADS;
            m[p] = kc_fmin_nn(m[p], kc_d32_dist<D>(x[p], c));
            if (i < n) best = kc_umax64(best, kc_pack(m[p], i));
        }
        best = kc_wave_max_key(best);
        if (lane == 0) sred[wave] = best;
        __syncthreads();         // every wave's max in; every read of sc done
        u64 key = sred[0];
#pragma unroll
        for (int w = 1; w < KC_BK_WAVES; ++w) key = kc_umax64(key, sred[w]);
        if ((key >> 32) == 0) {  // every point is a center: the traversal ends
            for (int u = t + (int)tid; u < k; u += KC_BK_THREADS) keys[u] = 0;
            break;
        }
        if (tid == 0) keys[t] = key;
        if (t == k - 1) break;   // the farthest point after the last center
        const uint32_t ci = kc_key_idx(key);
#pragma unroll
        for (int p = 0; p < PPT; ++p)
            if (tid + (uint32_t)p * KC_BK_THREADS == ci) {
#pragma unroll
                for (int j = 0; j < D; ++j) sc[j] = x[p][j];
            }
        __syncthreads();         // the new center's coordinates in
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint32_t i = tid + (uint32_t)p * KC_BK_THREADS;
        if (i < n) mind[i] = m[p];
    }
}

// (d, points per lane): the register file of 1,024 lanes at four waves per
// SIMD holds PPT * (d + 1) floats per lane within 128 VGPRs
#define KC_BK_DIMS(X) X(2, 20) X(3, 16) X(8, 8) X(10, 7) X(16, 4)

bool kc_gon_block_fits(int d, uint64_t n)
{
    switch (d) {
#define KC_CASE(DD, PP) \
    case DD:            \
        return n >= 1 && n <= (uint64_t)KC_BK_THREADS * PP;
        KC_BK_DIMS(KC_CASE)
#undef KC_CASE
    default:
        return false;
    }
}

hipError_t kc_gon_block(int d, const float* X, int64_t ld, uint32_t n, uint32_t first, int k,
                        float* mind, u64* keys, hipStream_t s)
{
    switch (d) {
#define KC_CASE(DD, PP)                                                                      \
    case DD:                                                                                 \
        hipLaunchKernelGGL((k_gon_block<DD, PP>), dim3(1), dim3(KC_BK_THREADS), 0, s, X, ld, n, \
                           first, k, mind, keys);                                            \
        return hipGetLastError();
        KC_BK_DIMS(KC_CASE)
#undef KC_CASE
    default:
        return hipErrorInvalidValue;
    }
}
