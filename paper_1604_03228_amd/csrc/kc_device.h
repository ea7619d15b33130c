// kc_device.h -- device helpers shared by the HIP kernels of libkcenter.
//
// Conventions used by every kernel:
//  * A point's squared distance to a center in FP32 is the "canonical" value
//      s = 0; for t in 0..d-1: diff = x_t - c_t; s = fmaf(diff, diff, s)
//    computed by one lane per point in ascending t.  Every path that compares
//    FP32 distances (the FP32 stream, the BF16 path's exact rescoring) uses
//    this one function, so tiling and launch shape never change a result.
//    Its relative error against the exact value is at most gamma_{d+2},
//    gamma_m = m u / (1 - m u), u = 2^-24.
//  * The FP64 distance is the sum of separately rounded squares of exact
//    FP64 differences, ascending t, no FMA contraction.
//  * Farthest-point selection packs (value, index) into one 64-bit key:
//    high word = bits of the non-negative FP32 value (monotone as unsigned),
//    low word  = 0xFFFFFFFF - index, so the maximum key is the farthest point
//    and, among equal values, the lowest index (ties to the lowest index).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define KC_BLOCK 256
#define KC_MAXD 256

typedef unsigned long long u64;

// One problem or partition of a batched Gonzalez run.
struct KcSeg {
    uint64_t src;     // first row of this segment in the caller's [n][ld] array
    uint64_t base;    // first column of this segment in the SoA staging copy
    uint32_t len;     // points in the segment
    uint32_t first;   // local index of the first center
    uint32_t ksteps;  // centers to choose
    uint32_t keyoff;  // this segment's keys live at keys[keyoff + t]
};

__device__ __forceinline__ float kc_d32_step(float s, float x, float c)
{
    float diff = x - c;
    return __builtin_fmaf(diff, diff, s);
}

// The canonical distance over D coordinates.  Its first step, fmaf(t, t,
// +0), equals t * t for every t (one rounding of the exact square, never
// -0), so it is written as the multiply: a two-operand instruction, which
// the VALU issues at a higher rate than the three-operand FMA.
template <int D, class A, class B>
__device__ __forceinline__ float kc_d32_dist(const A& x, const B& c)
{
    const float t = x[0] - c[0];
    float s = t * t;
#pragma unroll
    for (int j = 1; j < D; ++j) s = kc_d32_step(s, x[j], c[j]);
    return s;
}

// Minimum of two non-negative FP32 values (squared distances, +inf) as
// their bit patterns order: one integer instruction, no NaN quieting.
__device__ __forceinline__ float kc_fmin_nn(float a, float b)
{
    return __uint_as_float(min(__float_as_uint(a), __float_as_uint(b)));
}

__device__ __forceinline__ double kc_d64_step(double s, double x, double c)
{
    double diff = x - c;
    double sq = __dmul_rn(diff, diff);
    return __dadd_rn(s, sq);
}

// Correctly rounded FP64 square root (reported radii must equal a host
// sqrt bit for bit).  The hardware-assisted sqrt is within an ulp; Tuckerman's
// test then fixes the last bit: y = RN(sqrt(x)) iff y*pred(y) < x <=
// y*succ(y), and the signs of x - y*y' are exact through one FMA.
__device__ __forceinline__ double kc_sqrt_rn(double x)
{
    if (!(x > 0.0) || x == __builtin_inf()) return __builtin_sqrt(x);
    double y = __builtin_sqrt(x);
    for (int it = 0; it < 3; ++it) {
        const long long b = __double_as_longlong(y);
        const double yd = __longlong_as_double(b - 1), yu = __longlong_as_double(b + 1);
        if (__fma_rn(-y, yd, x) <= 0.0)
            y = yd;
        else if (__fma_rn(-y, yu, x) > 0.0)
            y = yu;
        else
            break;
    }
    return y;
}

__device__ __forceinline__ u64 kc_pack(float v, uint32_t idx)
{
    return ((u64)__float_as_uint(v) << 32) | (u64)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t kc_key_idx(u64 k) { return 0xFFFFFFFFu - (uint32_t)k; }
__device__ __forceinline__ float kc_key_val(u64 k) { return __uint_as_float((uint32_t)(k >> 32)); }

__device__ __forceinline__ u64 kc_umax64(u64 a, u64 b) { return a > b ? a : b; }

__device__ __forceinline__ u64 kc_wave_max64(u64 v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        u64 o = __shfl_xor(v, off, 64);
        v = kc_umax64(v, o);
    }
    return v;
}

// One DPP exchange of a 64-bit value (both halves); lanes the control does
// not write read 0, which never raises an unsigned max.
template <int CTRL, int ROWS>
__device__ __forceinline__ u64 kc_dpp64(u64 v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS,
                                                               0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL,
                                                               ROWS, 0xF, false);
    return ((u64)hi << 32) | lo;
}

// Wave-wide max of a 64-bit key through DPP (no LDS round trips): quad
// swaps, half-row and row mirrors leave every lane with its row's max, the
// row broadcasts of lanes 15 and 31 carry it up to lane 63, which is read
// out.  Must be called with all 64 lanes active; the result is uniform.
__device__ __forceinline__ u64 kc_wave_max64_dpp(u64 v)
{
    v = kc_umax64(v, kc_dpp64<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
    v = kc_umax64(v, kc_dpp64<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
    v = kc_umax64(v, kc_dpp64<0x141, 0xF>(v));   // row_half_mirror
    v = kc_umax64(v, kc_dpp64<0x140, 0xF>(v));   // row_mirror
    v = kc_umax64(v, kc_dpp64<0x142, 0xA>(v));   // row_bcast:15 into rows 1, 3
    v = kc_umax64(v, kc_dpp64<0x143, 0xC>(v));   // row_bcast:31 into rows 2, 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((u64)hi << 32) | lo;
}

// Wave-wide max of a 32-bit unsigned value through DPP (the same exchange
// pattern as kc_wave_max64_dpp, one word).  All 64 lanes active; uniform.
__device__ __forceinline__ uint32_t kc_wave_max_u32_dpp(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Wave-wide max of packed keys in two 32-bit passes: the value word, then
// the index word among the lanes holding that value (skipped when only one
// lane does).  All 64 lanes active; uniform.
__device__ __forceinline__ u64 kc_wave_max_key(u64 v)
{
    const uint32_t hv = (uint32_t)(v >> 32);
    const uint32_t mh = kc_wave_max_u32_dpp(hv);
    const bool tie = hv == mh;
    const u64 bal = __ballot(tie);
    uint32_t lo;
    if (__builtin_popcountll(bal) == 1)
        lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)__builtin_ctzll(bal));
    else
        lo = kc_wave_max_u32_dpp(tie ? (uint32_t)v : 0u);
    return ((u64)mh << 32) | lo;
}

// Block-wide max of a 64-bit key; the result is valid in every thread.
// `red` must hold blockDim.x / 64 entries.
__device__ __forceinline__ u64 kc_block_max64(u64 v, u64* red)
{
    v = kc_wave_max64(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    u64 r = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = kc_umax64(r, red[i]);
    __syncthreads();
    return r;
}

// Partial argmax slots of a streaming step.  Many blocks meeting at one
// 64-bit atomic serialise at the memory side, so each step's key is split
// over KC_PARTS slots on separate 128-byte lines (block b uses slot b mod
// KC_PARTS); the step's key is the max over its slots.
#define KC_PARTS 16
#define KC_PSTRIDE 16   // u64 per slot: one 128-byte line
__device__ __forceinline__ u64* kc_part_slot(u64* part, uint64_t key, uint32_t slot)
{
    return part + (key * KC_PARTS + slot) * KC_PSTRIDE;
}

// Max over the KC_PARTS slots of one key, computed by the first wave of the
// block; the result is valid in every thread.  `red` holds one u64.
__device__ __forceinline__ u64 kc_part_reduce(const u64* part, uint64_t key, u64* red)
{
    if (threadIdx.x < 64) {
        u64 v = 0;
        if (threadIdx.x < KC_PARTS)
            v = __hip_atomic_load(part + (key * KC_PARTS + threadIdx.x) * KC_PSTRIDE,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = kc_wave_max64(v);
        if (threadIdx.x == 0) *red = v;
    }
    __syncthreads();
    u64 r = *red;
    __syncthreads();
    return r;
}

// Offer a block's key to its slot: skip the atomic when the slot already
// holds a larger key (a stale read is never larger than the true value, so
// skipping is always safe).
__device__ __forceinline__ void kc_part_offer(u64* part, uint64_t key, uint32_t slot, u64 v)
{
    u64* p = kc_part_slot(part, key, slot);
    u64 cur = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v > cur) __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double kc_wave_min_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// Non-negative doubles order like their bit patterns as unsigned integers.
__device__ __forceinline__ void kc_atomic_max_f64_nonneg(double* p, double v)
{
    atomicMax((u64*)p, (u64)__double_as_longlong(v));
}
__device__ __forceinline__ void kc_atomic_max_f32_nonneg(float* p, float v)
{
    atomicMax((unsigned*)p, __float_as_uint(v));
}
