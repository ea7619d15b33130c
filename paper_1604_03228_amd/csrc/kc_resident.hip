// kc_resident.hip -- register-resident persistent Gonzalez engine.
//
// One cooperative launch runs all k steps of one segment whose points fit in
// the register file of the grid: thread (g, tid) keeps the coordinates and
// the running FP32 min-distance of local points
//     i = g*KC_BLOCK*PPT + p*KC_BLOCK + tid,  p < PPT
// in VGPRs, so a step reads nothing from memory but the new center's d
// coordinates.  Bound by VALU work plus the per-step grid barrier.
//
// Per-step barrier and argmax in one exchange: block b writes its packed key
// to slots[t*G + b] (keys are never 0: their low word is 0xFFFFFFFF - index)
// and every block polls all G slots until none is 0, then takes their max.
// Only relaxed device-scope atomics carry data, and only keys travel, so no
// cache write-back or invalidation sits on the critical path.  Any block
// whose wait exceeds the spin limit raises abort_flag; every block then
// leaves its loop.
#include "kc_device.h"
#include "kc_internal.h"

template <int D, int PPT>
__global__ __launch_bounds__(KC_BLOCK, 1) void k_gon_resident(
    const float* __restrict__ xs, uint64_t stride, uint64_t base, uint32_t len,
    const uint32_t* __restrict__ len_ptr, uint32_t first, int k, float* __restrict__ mind,
    u64* __restrict__ keys, u64* __restrict__ slots, uint32_t* __restrict__ abort_flag,
    uint32_t spin_limit)
{
    if (len_ptr) len = min(len, *len_ptr);   // actual length known on the device
    __shared__ float cc[D];
    __shared__ u64 red[KC_BLOCK / 64];
    const uint32_t G = gridDim.x;   // <= KC_BLOCK (checked by the host)
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
    for (int t = 0; t < k; ++t) {
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
        // a block without points (the device-side length can be shorter than
        // the grid's capacity) still publishes: key 1 is "no point", it never
        // wins (a real index is below 0xFFFFFFFE) and is not the empty slot 0
        if (key == 0) key = 1;
        u64* row = slots + (uint64_t)t * G;
        if (threadIdx.x == 0)
            __hip_atomic_store(row + blockIdx.x, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // wait until every block of the grid has published its key
        u64 v = 0;
        uint32_t spins = 0;
        int aborted = 0;
        for (;;) {
            int ok = 1;
            if (threadIdx.x < G) {
                v = __hip_atomic_load(row + threadIdx.x, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                ok = v != 0;
            }
            if (__syncthreads_and(ok)) break;
            ++spins;
            if ((spins & 63) == 0) {
                int ab = 0;
                if (threadIdx.x == 0) {
                    ab = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) != 0;
                    if (!ab && spins > spin_limit) {
                        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        ab = 1;
                    }
                }
                if (__syncthreads_or(ab)) {
                    aborted = 1;
                    break;
                }
            }
            __builtin_amdgcn_s_sleep(1);
        }
        u64 kk = kc_block_max64(threadIdx.x < G ? v : 0ull, red);
        if (aborted) kk = 0;   // every block leaves the loop
        if (blockIdx.x == 0 && threadIdx.x == 0) keys[t] = kk;
        if ((kk >> 32) == 0) break;   // radius 0 (or abort): stop
        c = kc_key_idx(kk);
    }
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const uint32_t i = i0 + p * KC_BLOCK;
        if (i < len) mind[base + i] = m[p];
    }
}

// Largest points-per-thread whose coordinates fit in about 200 VGPRs.
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

template <int D, int PPT>
static hipError_t launch_resident(uint32_t G, const float* xs, uint64_t stride,
                                  uint64_t base, uint32_t len, const uint32_t* len_ptr,
                                  uint32_t first, int k,
                                  float* mind, u64* keys, u64* slots, uint32_t* abort_flag,
                                  uint32_t spin_limit, hipStream_t s)
{
    void* args[] = {(void*)&xs,    (void*)&stride, (void*)&base, (void*)&len,
                    (void*)&len_ptr, (void*)&first, (void*)&k,      (void*)&mind, (void*)&keys,
                    (void*)&slots, (void*)&abort_flag, (void*)&spin_limit};
    return hipLaunchCooperativeKernel((const void*)k_gon_resident<D, PPT>, dim3(G),
                                      dim3(KC_BLOCK), args, 0, s);
}

template <int D, int PPT>
static int max_resident_blocks()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gon_resident<D, PPT>,
                                                     KC_BLOCK, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int g = per_cu * cus;
    return g < KC_BLOCK ? g : KC_BLOCK;   // the barrier polls one slot per thread
}

#define KC_RES_DIMS(X) X(2, 32) X(3, 32) X(8, 16) X(10, 16) X(16, 8) X(32, 4) X(41, 4)

int kc_resident_max_blocks(int d)
{
    switch (d) {
#define KC_CASE(DD, PP) \
    case DD: return max_resident_blocks<DD, PP>();
        KC_RES_DIMS(KC_CASE)
#undef KC_CASE
    default: return 0;
    }
}

uint32_t kc_resident_blocks_for(int d, uint32_t len)
{
    const uint64_t per = (uint64_t)resident_ppt(d) * KC_BLOCK;
    if (per == 0) return 0;
    return (uint32_t)((len + per - 1) / per);
}

uint64_t kc_resident_slot_words(int k, uint32_t G) { return (uint64_t)k * G; }

// Returns hipSuccess, or an error when the shape has no resident kernel or
// the grid cannot be co-resident (the caller then streams instead).
hipError_t kc_gon_resident(int d, uint32_t G, const float* xs, uint64_t stride,
                           uint64_t base, uint32_t len, const uint32_t* len_ptr,
                           uint32_t first, int k, float* mind,
                           u64* keys, u64* slots, uint32_t* abort_flag, uint32_t spin_limit,
                           hipStream_t s)
{
    if (G == 0 || G > KC_BLOCK) return hipErrorInvalidValue;
    switch (d) {
#define KC_CASE(DD, PP)                                                                  \
    case DD:                                                                             \
        return launch_resident<DD, PP>(G, xs, stride, base, len, len_ptr, first, k, mind, keys, \
                                       slots, abort_flag, spin_limit, s);
        KC_RES_DIMS(KC_CASE)
#undef KC_CASE
    default:
        return hipErrorInvalidValue;
    }
}
