// kc_resident.hip -- register-resident persistent Gonzalez engine with
// certified lookahead.
//
// One cooperative launch runs all k steps of one segment whose points fit in
// the register file of the grid, or of several segments at once (each on its
// own consecutive blocks, exchanging only among them: the partitions of an
// MRG round, or the problems of a batch).  A block has one leader wave and
// KC_LA_WORKERS worker waves; worker lane (g, w, lane) keeps the coordinates
// and the running FP32 min-distance of local points
//     i = g*KC_LA_WPTS*PPT + p*KC_LA_WPTS + w*64 + lane,  p < PPT
// in VGPRs (KC_LA_WPTS = 64*KC_LA_WORKERS), so applying a center reads
// nothing from memory but its d coordinates.
//
// Gonzalez's traversal (Section 3.1) adds one farthest point per step, and a
// plain parallel version needs one grid-wide argmax per step.  This engine
// meets the grid once per *round* of several steps instead:
//
//  1. every worker wave publishes its K+1 largest keys (key = FP32
//     min-distance and index, as in kc_device.h);
//  2. every block reads all published words; tau is the largest (K+1)-th key
//     over the waves, and the candidate set C is every published key above
//     tau (at most CMAX of them: when more qualify, tau is raised to the
//     smallest bound that leaves at most that many);
//  3. the leader wave runs Gonzalez's step on C alone (the same canonical
//     FP32 distances the owning lanes use) for as long as the best key of C
//     stays above tau, and queues each chosen center in LDS; the worker
//     waves apply the queued centers to their points as they appear.
//
// A point outside C had a key of at most tau when the round began and keys
// only decrease, so a key of C above tau is the global maximum: the centers,
// keys and min-distances equal those of the step-by-step traversal bit for
// bit.  The first step of every round is always certified (the global
// maximum is some wave's largest key and lies above every (K+1)-th key), so
// each round makes progress.  The sequence of a round depends on C alone,
// so the leader runs ahead of the workers and only the workers' arithmetic
// on their points remains per step.
//
// Exact-integer form.  When every coordinate of a segment is an integer of
// magnitude at most M, with 5 d M^2 <= 2^24, every partial sum of the
// canonical distance and of K + ||c||^2 - 2 x.c (K = d M^2) is an integer
// of magnitude at most 2^24, so both are exact in FP32.  Such a segment's
// workers then keep m' = min over centers of (K + ||c||^2 - 2 x.c), with
// -2x in place of x, and apply a center in d FMAs and one min per point
// instead of 2d + 1 instructions.  m' >= K - ||x||^2 >= 0, so the min is
// the same unsigned compare of bit patterns; a key is (m' - K) + ||x||^2,
// the canonical FP32 value bit for bit.
// Each block checks its own points (and resumed min-distances) while
// loading them and sets bit 63 of its first bound word when one fails
// (keys are non-negative, so that bit is otherwise clear); every block of
// the segment reads all of them in the first exchange and so takes the
// same form.  The leader always computes canonical distances.
//
// Exchange words carry their round in the low word, so no word needs a
// fence: (bits of the FP32 value << 32) | (tag << 16) | block-local index,
// index 0xFFFF = "no point" (waves without points), tag = round + 1 mod 2^16.
// Rounds alternate between two buffers; a block cannot write round r+2
// before every block has read round r, because it first needs every block's
// round r+1 words.  Only relaxed device-scope atomics carry data.  Any block
// whose wait exceeds the spin limit raises abort_flag; every block then
// leaves its loop.
#include <algorithm>
#include <type_traits>

#include "kc_device.h"
#include "kc_internal.h"

#define KC_LA_BLOCK 512                                  // threads: two waves per SIMD
#define KC_LA_WAVES (KC_LA_BLOCK / 64)
#define KC_LA_WORKERS (KC_LA_WAVES - 1)                  // wave 0 leads
#define KC_LA_WPTS (KC_LA_WORKERS * 64)                  // worker lanes per block
#define KC_LA_GMAX 256                                   // blocks of the largest grid
#define KC_LA_K 2                                        // candidates per wave
#define KC_LA_KK (KC_LA_K + 1)                           // plus the wave's bound
#define KC_LA_WPB (KC_LA_WORKERS * KC_LA_K + 1)          // words per block: candidates, bound
#define KC_LA_BUF (KC_LA_GMAX * KC_LA_WPB)               // words per round buffer
#define KC_LA_NPT ((KC_LA_BUF + KC_LA_BLOCK - 1) / KC_LA_BLOCK)   // words per thread
#define KC_LA_NONE 0xFFFFu
#define KC_LA_END 0x80000000u

// Candidate cap: the leader lane keeps CMAX/64 candidates in the registers
// a worker lane uses for its PPT points (so at most PPT of them, and at most
// 8: one candidate per thread when their coordinates are gathered).
template <int PPT>
struct KcLaCap {
    static constexpr int value = 64 * (PPT < KC_LA_WAVES ? PPT : KC_LA_WAVES);
};

__device__ __forceinline__ uint32_t kc_la_tag(uint32_t r) { return (r + 1u) & 0xFFFFu; }

#define KC_LA_NOTINT 0x8000000000000000ull   // bound word of round 0: a block's points fail
// The exact-integer form is built for d >= 8 (at d = 2 and 3 its extra code
// outside the apply loop makes the kernels spill).
#define KC_LA_INT_FORM(d) ((d) >= 8)

// Largest M with 5 d M^2 <= 2^24, and the offset K = d M^2: for integer
// coordinates up to M, every partial sum of a squared distance and of
// K + ||c||^2 - 2 x.c is an integer of magnitude at most 5 d M^2, so exact
// in FP32, and K + ||c||^2 - 2 x.c = K - ||x||^2 + |x - c|^2 >= 0.
constexpr unsigned long long kc_la_int_m(int d)
{
    unsigned long long m = 0;
    while (5ull * (unsigned long long)d * (m + 1) * (m + 1) <= (1ull << 24)) ++m;
    return m;
}
constexpr float kc_la_int_bound(int d) { return (float)kc_la_int_m(d); }
constexpr float kc_la_int_offset(int d)
{
    return (float)((unsigned long long)d * kc_la_int_m(d) * kc_la_int_m(d));
}

__device__ __forceinline__ bool kc_la_small_int(float v, float bound)
{
    return __builtin_fabsf(v) <= bound && v == __builtin_rintf(v);
}

// Exchange word of key `key` (0: no point) of the block whose points start
// at `blk0`, in round tag `tag`.
__device__ __forceinline__ u64 kc_la_word(u64 key, uint32_t blk0, uint32_t tag)
{
    const uint32_t il = key != 0 ? kc_key_idx(key) - blk0 : KC_LA_NONE;
    return (key & 0xFFFFFFFF00000000ull) | (u64)((tag << 16) | il);
}

// Key of exchange word `w` published by block `g`; 0 for "no point".
template <int PPT>
__device__ __forceinline__ u64 kc_la_decode(u64 w, uint32_t g)
{
    const uint32_t il = (uint32_t)w & 0xFFFFu;
    if (il == KC_LA_NONE) return 0;
    const uint32_t i = g * (KC_LA_WPTS * PPT) + il;
    return (w & 0xFFFFFFFF00000000ull) | (u64)(0xFFFFFFFFu - i);
}

// An opaque copy: the compiler cannot hoist expressions of it out of the
// loop it is taken in.
__device__ __forceinline__ uint32_t kc_opaque(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ float kc_opaque_f(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

template <int D, int PPT>
__global__ __launch_bounds__(KC_LA_BLOCK, 1) void k_gon_resident(
    const float* __restrict__ xs, uint64_t stride, uint64_t base, uint32_t len,
    const uint32_t* __restrict__ len_ptr, uint32_t first, int k, float* __restrict__ mind,
    u64* __restrict__ keys, u64* __restrict__ xbuf, uint32_t* __restrict__ abort_flag,
    uint32_t spin_limit, const float* __restrict__ xa, int64_t lda, int xa_rows,
    uint32_t* __restrict__ status, const KcSeg* __restrict__ segs, const uint4* __restrict__ blks,
    const float* mind_in)
{
    static_assert(KC_LA_WPTS * PPT <= KC_LA_NONE, "block-local index must fit in 16 bits");
    constexpr uint32_t CMAX = KcLaCap<PPT>::value;
    constexpr int QL = CMAX / 64;   // candidates per leader lane
    static_assert(CMAX <= KC_LA_BLOCK, "one candidate per thread when gathering");
    // Several segments per launch: blks[b] = (segment, block within it,
    // blocks of the segment, first block of the segment); the segment's
    // blocks are consecutive and exchange only among themselves.  Without
    // blks the launch is one segment described by the scalar arguments.
    uint32_t lb = blockIdx.x, gs = gridDim.x, b0 = 0;
    if (blks) {
        const uint4 bi = blks[blockIdx.x];
        const KcSeg sg = segs[bi.x];
        lb = bi.y;
        gs = bi.z;
        b0 = bi.w;
        base = sg.base;
        len = sg.len;
        first = sg.first;
        k = (int)sg.ksteps;
        keys += sg.keyoff;
        if (xa) xa += sg.src * (uint64_t)lda;
    }
    if (len_ptr) len = min(len, *len_ptr);   // actual length known on the device
    __shared__ u64 sCk[CMAX];                 // candidate keys at the round's start
    __shared__ float sCx[D][CMAX];            // candidate coordinates
    __shared__ float sCc[CMAX];               // K + their squared norms (exact-integer form)
    __shared__ uint32_t sQf[CMAX + 1];        // the round's queue: 0 empty, slot + 1 of a
                                              // center, KC_LA_END | state at the end
    __shared__ u64 sQk[CMAX];                 // the keys of the round's certified steps
    __shared__ float sPm[CMAX];               // the leader's packing of live candidates
    __shared__ uint32_t sPi[CMAX], sPo[CMAX];
    __shared__ float cc0[D];
    __shared__ u64 red[KC_LA_WAVES];
    __shared__ uint32_t sWc[KC_LA_WAVES];
    __shared__ u64 sT[KC_LA_WAVES];           // each worker wave's (K+1)-th key
    __shared__ uint32_t sNi, sNx;             // this block's points / the segment's fail
                                              // the exact-integer check

    const uint32_t NWB = gs * KC_LA_WPB;    // exchange words of this segment
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const bool leader = wave == 0;
    const uint32_t blk0 = lb * (KC_LA_WPTS * PPT);
    const uint32_t i0 = blk0 + (leader ? 0u : (wave - 1) * 64 + lane);
    const bool recorder = lb == 0 && tid == 0;   // the leader of the segment's block 0

    // The points come from the caller's rows when xa_rows is set, else from
    // the SoA staging copy (coalesced per coordinate).  A lane reads its
    // point's row in vector loads: a wave's 64 rows are contiguous, so every
    // cache line it touches is used whole across the row's loads.  Rows past
    // the end read row 0 and are never live.
    auto coord = [&](uint32_t i, int j) -> float {
        return xa_rows ? xa[(uint64_t)i * (uint64_t)lda + j] : xs[(uint64_t)j * stride + base + i];
    };
    float x[PPT][D];
    float m[PPT];
    if (tid < D) cc0[tid] = coord(first, tid);
    if (tid == 0) {
        sNi = 0;
        sNx = 0;
    }
    if (!leader) {
        if (xa_rows) {
            // kc_resident_row_floats(D) floats per load: the host takes this
            // path only when rows and base are aligned to it and byte
            // offsets from the segment's first row fit 32 bits, so each load
            // is the wave-uniform base plus one 32-bit VGPR
            constexpr int VW = D % 4 == 0 ? 4 : D % 2 == 0 ? 2 : 1;
            const char* xb = (const char*)xa;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const uint32_t i = i0 + p * KC_LA_WPTS;
                const uint32_t bo = (i < len ? i : 0u) * (uint32_t)lda * 4u;
#pragma unroll
                for (int j = 0; j < D; j += VW) {
                    if constexpr (VW == 4) {
                        const float4 v = *(const float4*)(xb + bo + 4 * j);
                        x[p][j] = v.x;
                        x[p][j + 1] = v.y;
                        x[p][j + 2] = v.z;
                        x[p][j + 3] = v.w;
                    } else if constexpr (VW == 2) {
                        const float2 v = *(const float2*)(xb + bo + 4 * j);
                        x[p][j] = v.x;
                        x[p][j + 1] = v.y;
                    } else {
                        x[p][j] = *(const float*)(xb + bo + 4 * j);
                    }
                }
            }
        } else {
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const uint32_t i = i0 + p * KC_LA_WPTS;
                const uint32_t ii = i < len ? i : 0;
#pragma unroll
                for (int j = 0; j < D; ++j) x[p][j] = coord(ii, j);
            }
        }
    }
    __syncthreads();
    if (!leader) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < D; ++j) s = kc_d32_step(s, x[p][j], cc0[j]);
            m[p] = s;
        }
        if (mind_in) {
            // resumed run: the min-distances to the centers chosen before
            // `first` (read by the lane that later writes them back)
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const uint32_t i = i0 + p * KC_LA_WPTS;
                if (i < len) m[p] = kc_fmin_nn(m[p], mind_in[base + i]);
            }
        }
        // the exact-integer check of this lane's points and min-distances
        constexpr float KM = kc_la_int_bound(D);
        bool ok = KC_LA_INT_FORM(D);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            if (i0 + p * KC_LA_WPTS < len) {
                bool okp = m[p] == __builtin_rintf(m[p]) && m[p] <= 16777216.f;
#pragma unroll
                for (int j = 0; j < D; ++j) okp = okp && kc_la_small_int(x[p][j], KM);
                ok = ok && okp;
            }
        }
        if (__ballot(!ok) != 0 && lane == 0) sNi = 1u;
    }
    bool exact = false;   // the segment's points passed the check (decided in round 0)

    int t = 0;   // keys recorded (tracked by the leader)
    for (uint32_t r = 0;; ++r) {
        // per-round copies of the thread's position: values derived from
        // them are recomputed each round instead of being held in VGPRs
        // across the whole loop next to the points
        const uint32_t tid_r = kc_opaque(tid);
        const uint32_t i0_r = kc_opaque(i0);
        // ---- 1. this wave's K+1 largest keys (keys are distinct): each lane
        // keeps its own K+1 largest in order, then the wave pops its heads
        u64 mine = 0;
        if (!leader) {
            u64 top[KC_LA_KK];
#pragma unroll
            for (int j = 0; j < KC_LA_KK; ++j) top[j] = 0;
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const uint32_t i = i0_r + p * KC_LA_WPTS;
                float mv = m[p];
                if (exact) {   // (m' - K) + ||x||^2, with x held as -2x
                    // (recomputed each round, not held next to the points)
                    float xx = kc_opaque_f(0.f);
#pragma unroll
                    for (int j = 0; j < D; ++j) xx = __builtin_fmaf(x[p][j], x[p][j], xx);
                    mv = (m[p] - kc_la_int_offset(D)) + 0.25f * xx;
                }
                u64 v = i < len ? kc_pack(mv, i) : 0ull;
#pragma unroll
                for (int j = 0; j < KC_LA_KK; ++j) {
                    const u64 hi = kc_umax64(top[j], v);
                    v = top[j] < v ? top[j] : v;
                    top[j] = hi;
                }
            }
#pragma unroll
            for (int j = 0; j < KC_LA_KK; ++j) {
                const u64 b = kc_wave_max_key(top[0]);
                if (lane == (uint32_t)j) mine = b;
                if (top[0] == b) {   // b != 0 is held by exactly one lane
#pragma unroll
                    for (int q = 0; q + 1 < KC_LA_KK; ++q) top[q] = top[q + 1];
                    top[KC_LA_KK - 1] = 0;
                }
            }
        }
        // block g publishes words g*KC_LA_WPB + (w-1)*K + j (candidate j of
        // worker wave w) and g*KC_LA_WPB + KC_LA_WPB-1 (the block's bound:
        // the largest (K+1)-th key of its waves)
        u64* rb = xbuf + (uint64_t)(r & 1u) * KC_LA_BUF;
        u64* rbb = rb + (uint64_t)blockIdx.x * KC_LA_WPB;
        const uint32_t tag = kc_la_tag(r);
        if (!leader) {
            if (lane < KC_LA_K)
                __hip_atomic_store(rbb + (wave - 1) * KC_LA_K + lane, kc_la_word(mine, blk0, tag),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (lane == KC_LA_K) sT[wave] = mine;
        }
        __syncthreads();
        if (tid == 0) {
            u64 tb = 0;
#pragma unroll
            for (int w = 1; w < KC_LA_WAVES; ++w) tb = kc_umax64(tb, sT[w]);
            u64 wb = kc_la_word(tb, blk0, tag);
            if (r == 0 && sNi != 0) wb |= KC_LA_NOTINT;
            __hip_atomic_store(rbb + KC_LA_WPB - 1, wb, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }

        // ---- 2. every block's words of this round: each thread waits for
        // its own words, then the block meets once
        int ab = 0;
        uint32_t ni = 0;   // a round-0 bound word carried the failed check
        u64 tl = 0;   // largest bound word this thread received
        u64 wv[KC_LA_NPT];   // this thread's words e = tid + q*KC_LA_BLOCK, decoded
#pragma unroll
        for (int q = 0; q < KC_LA_NPT; ++q) wv[q] = 0;
        {
            uint32_t have = 0, spins = 0;
            for (;;) {
                bool all = true;
                // every word load is issued before any is examined, so one
                // wait covers them all (a word already taken, or past this
                // segment's end, is reread from a valid slot and ignored)
                u64 wr[KC_LA_NPT];
#pragma unroll
                for (int q = 0; q < KC_LA_NPT; ++q) {
                    const uint32_t e = tid_r + q * KC_LA_BLOCK;
                    wr[q] = __hip_atomic_load(rb + (uint64_t)b0 * KC_LA_WPB + (e < NWB ? e : 0u),
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int q = 0; q < KC_LA_NPT; ++q) {
                    const uint32_t e = tid_r + q * KC_LA_BLOCK;
                    if (e < NWB && !((have >> q) & 1u)) {
                        u64 w = wr[q];
                        if ((((uint32_t)w) >> 16) == tag) {
                            const bool bound = e % KC_LA_WPB == KC_LA_WPB - 1;
                            if (bound) {
                                ni |= (uint32_t)(w >> 63);
                                w &= ~KC_LA_NOTINT;
                            }
                            const u64 kw = kc_la_decode<PPT>(w, e / KC_LA_WPB);
                            if (bound) tl = kc_umax64(tl, kw);
                            else wv[q] = kw;   // bound words stay 0 here
                            have |= 1u << q;
                        } else {
                            all = false;
                        }
                    }
                }
                if (all) break;
                if ((++spins & 63) == 0) {
                    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        ab = 1;
                        break;
                    }
                    if (spins > spin_limit) {
                        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        atomicOr(status, 1u);
                        ab = 1;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        tl = kc_wave_max_key(tl);
        if (lane == 0) red[wave] = tl;
        for (uint32_t e = tid; e <= CMAX; e += KC_LA_BLOCK) sQf[e] = 0;
        if (ni) sNx = 1u;
        if (__syncthreads_or(ab)) {
            if (recorder && t < k) keys[t] = 0;
            break;
        }
        if (r == 0) {
            exact = KC_LA_INT_FORM(D) && __builtin_amdgcn_readfirstlane(sNx) == 0;
            if (exact && recorder) atomicAdd(status + 2, 1u);
            if (exact && !leader) {
                // into the exact-integer form: m' = (m - ||x||^2) + K, x -> -2x
#pragma unroll
                for (int p = 0; p < PPT; ++p) {
                    float xx = 0.f;
#pragma unroll
                    for (int j = 0; j < D; ++j) xx = __builtin_fmaf(x[p][j], x[p][j], xx);
                    m[p] = (m[p] - xx) + kc_la_int_offset(D);
#pragma unroll
                    for (int j = 0; j < D; ++j) x[p][j] *= -2.f;
                }
            }
        }

        // ---- 3. bound tau (the largest block bound) and candidate set C
        // (candidate words above tau)
        const uint64_t ltmask = (1ull << lane) - 1ull;
        u64 tau = red[0];
#pragma unroll
        for (int w = 1; w < KC_LA_WAVES; ++w) tau = kc_umax64(tau, red[w]);

        // candidates above `thr` in the block, and those of the waves before
        // this one (one barrier; sWc is rewritten only after another)
        auto count_above = [&](u64 thr, uint32_t& before) -> uint32_t {
            uint32_t cw = 0;
#pragma unroll
            for (int q = 0; q < KC_LA_NPT; ++q) {
                const bool pr = wv[q] > thr;
                cw += (uint32_t)__builtin_popcountll(__ballot(pr));
            }
            if (lane == 0) sWc[wave] = cw;
            __syncthreads();
            uint32_t tot = 0;
            before = 0;
#pragma unroll
            for (int w = 0; w < KC_LA_WAVES; ++w) {
                const uint32_t c = sWc[w];
                if (w < (int)wave) before += c;
                tot += c;
            }
            return tot;
        };
        uint32_t before = 0;
        uint32_t nc = count_above(tau, before);
        if (nc > CMAX) {
            // raise tau to the smallest bound leaving at most CMAX candidates:
            // keys are distinct, so count(> hi) >= CMAX at the end
            __syncthreads();
            u64 cl = 0;
#pragma unroll
            for (int q = 0; q < KC_LA_NPT; ++q) cl = kc_umax64(cl, wv[q]);
            u64 lo = tau, hi = kc_block_max64(cl, red);
            while (hi - lo > 1) {
                const u64 mid = lo + (hi - lo) / 2;
                if (count_above(mid, before) > CMAX) lo = mid;
                else hi = mid;
                __syncthreads();
            }
            tau = hi;
            nc = count_above(tau, before);
        }
        {
            uint32_t pos = before;
#pragma unroll
            for (int q = 0; q < KC_LA_NPT; ++q) {
                const bool pr = wv[q] > tau;
                const u64 bal = __ballot(pr);
                if (pr) sCk[pos + (uint32_t)__builtin_popcountll(bal & ltmask)] = wv[q];
                pos += (uint32_t)__builtin_popcountll(bal);
            }
        }
        __syncthreads();
        if (tid_r < nc) {   // one candidate per thread: all loads in flight at once
            const uint32_t ci = kc_key_idx(sCk[tid_r]);
            float v[D];
            if (xa) {   // the caller's rows: one or two cache lines per candidate
                const float* row = xa + (uint64_t)ci * (uint64_t)lda;
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = row[j];
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = xs[(uint64_t)j * stride + base + ci];
            }
            float vv = 0.f;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                sCx[j][tid_r] = v[j];
                vv = __builtin_fmaf(v[j], v[j], vv);
            }
            sCc[tid_r] = vv + kc_la_int_offset(D);   // K + ||c||^2
        }
        __syncthreads();

        // tau and nc are block-uniform: into SGPRs
        tau = ((u64)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(tau >> 32)) << 32) |
              (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)tau);
        nc = __builtin_amdgcn_readfirstlane(nc);

        // ---- 4. certified steps.  state: 0 next step, 1 round over,
        // 2 traversal over, 3 no progress
        uint32_t state = 0;
        if (leader) {
            // The leader shares a SIMD with a worker wave; it issues first so
            // that the workers never wait for a center.
            __builtin_amdgcn_s_setprio(3);
            // Gonzalez's step on C: lane `lane` holds candidates q*64 + lane,
            // q < QL, in the registers of a worker's points (coordinates in
            // x[q], min-distance in m[q], index ni[q] (held complemented, as
            // in the low word of a key), slot in C os[q]).  A
            // candidate at or below tau can no longer be certified this
            // round: it stops competing, and once the live candidates fit in
            // fewer chunks of 64 they are packed (through LDS) into the
            // first nv positions, so a step touches ceil(nv/64) chunks.
            // In the exact-integer form a lane holds -2x for its candidates'
            // coordinates and ||x||^2 - K beside them, and a step computes
            // (K + ||c||^2) - 2 x.c + (||x||^2 - K), the exact distance.
            uint32_t nq = 0;      // centers queued this round
            int ns = 0;           // steps certified this round (at most nc)
            const int t0 = t;     // their keys go to keys[t0 + i] at the round's end
            auto lead = [&](auto form) {
                constexpr bool EX = decltype(form)::value;
                constexpr float K2 = 2.f * kc_la_int_offset(D);
                uint32_t ni[QL], os[QL];
                auto key_of = [](float mv, uint32_t n) -> u64 {
                    return ((u64)__float_as_uint(mv) << 32) | (u64)n;
                };
                float xq[EX ? QL : 1];
                u64 bl = 0;
                uint32_t bs = 0;
                uint32_t nv = nc, qn = (nc + 63) / 64;
#pragma unroll
                for (int q = 0; q < QL; ++q) {
                    // slots past nc hold stale LDS values: their key is taken as 0
                    // (min-distance 0, never live), so their coordinates may be
                    // anything and the loads need no mask (at d = 16 with 9 points
                    // per lane this costs a few spilled VGPRs and is still faster)
                    const uint32_t sl = q * 64 + lane;
                    const bool v = sl < nc;
                    const u64 kraw = sCk[sl];
                    const u64 kq = v ? kraw : 0ull;
                    m[q] = kc_key_val(kq);
                    ni[q] = (uint32_t)kq;   // the key's complemented index
                    os[q] = sl;
#pragma unroll
                    for (int j = 0; j < D; ++j) x[q][j] = EX ? -2.f * sCx[j][sl] : sCx[j][sl];
                    if constexpr (EX) xq[q] = sCc[sl] - K2;
                    if (kq > bl) {   // every key of C is above tau
                        bl = kq;
                        bs = sl;
                    }
                }
                // coordinates of this lane's best candidate, read ahead of the
                // wave's argmax so the winner's come out of registers
                float bx[D], bq = 0.f;
#pragma unroll
                for (int j = 0; j < D; ++j) bx[j] = sCx[j][bs];
                if constexpr (EX) bq = sCc[bs];
                do {
                    // the loop's control values are wave-uniform: keep them in
                    // SGPRs so its branches stay scalar
                    t = __builtin_amdgcn_readfirstlane(t);
                    nq = __builtin_amdgcn_readfirstlane(nq);
                    nv = __builtin_amdgcn_readfirstlane(nv);
                    qn = __builtin_amdgcn_readfirstlane(qn);
                    const u64 b = kc_wave_max_key(bl);
                    if (b > tau) {
                        if (lane == 0) sQk[ns] = b;
                        ++t;
                        ++ns;
                        state = ((b >> 32) == 0 || t >= k) ? 2u : 0u;   // radius 0 or k centers
                    } else if (ns == 0) {
                        // no certified step: only when the segment has no point
                        // (b == 0, reported as radius 0); otherwise impossible
                        if (b == 0) {
                            if (recorder) keys[t] = 0;
                            ++t;
                            state = 2;
                        } else {
                            state = 3;
                        }
                    } else {
                        state = 1;
                    }
                    state = __builtin_amdgcn_readfirstlane(state);
                    if (state == 0) {
                        // the winner's slot, and its coordinates into SGPRs from
                        // the winning lane's copy
                        const int wl = (int)__builtin_ctzll(__ballot(bl == b));
                        const uint32_t wslot = __builtin_amdgcn_readlane(bs, wl) + 1u;
                        // Queue the center for the workers.  In the canonical
                        // form the workers' arithmetic bounds the steps, so they
                        // get it at once; in the exact-integer form the leader's
                        // chain does, and the center is queued after the update
                        // below, so that the worker wave sharing the leader's
                        // SIMD applies it during the leader's next argmax (few
                        // vector instructions) instead of during the update.
                        if constexpr (!EX) {
                            if (lane == 0)
                                __hip_atomic_store(&sQf[nq], wslot, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                            ++nq;
                        }
                        auto from_winner = [&](float v) -> float {
                            return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), wl));
                        };
                        float cc[D];
#pragma unroll
                        for (int j = 0; j < D; ++j) cc[j] = from_winner(bx[j]);
                        const float ccq = EX ? from_winner(bq) : 0.f;
                        bl = 0;
                        uint32_t live = 0;
                        // chunks in pairs without a branch between them
#pragma unroll
                        for (int g = 0; g < QL; g += 2) {
                            if (g < (int)qn) {
#pragma unroll
                                for (int q = g; q < g + 2 && q < QL; ++q) {
                                    float s;
                                    if constexpr (EX) {
                                        s = ccq;
#pragma unroll
                                        for (int j = 0; j < D; ++j)
                                            s = __builtin_fmaf(x[q][j], cc[j], s);
                                        s += xq[q];
                                    } else {
                                        s = 0.f;
#pragma unroll
                                        for (int j = 0; j < D; ++j)
                                            s = kc_d32_step(s, x[q][j], cc[j]);
                                    }
                                    m[q] = kc_fmin_nn(m[q], s);
                                    const u64 kq = key_of(m[q], ni[q]);
                                    // one ballot per compare: their masks
                                    // combine on the scalar unit
                                    const bool in = q * 64 + lane < nv, up = kq > tau;
                                    live += (uint32_t)__builtin_popcountll(
                                        __builtin_amdgcn_ballot_w64(in) &
                                        __builtin_amdgcn_ballot_w64(up));
                                    if (in && up && kq > bl) {
                                        bl = kq;
                                        bs = os[q];
                                    }
                                }
                            }
                        }
                        if constexpr (EX) {
                            if (lane == 0)
                                __hip_atomic_store(&sQf[nq], wslot, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                            ++nq;
                        }
                        if (live + 64 <= qn * 64) {
                            // pack the live candidates into positions 0..live-1
                            uint32_t pos = 0;
#pragma unroll
                            for (int q = 0; q < QL; ++q) {
                                if (q < (int)qn) {
                                    const bool lv =
                                        q * 64 + lane < nv && key_of(m[q], ni[q]) > tau;
                                    const u64 bal = __builtin_amdgcn_ballot_w64(lv);
                                    if (lv) {
                                        const uint32_t p =
                                            pos + (uint32_t)__builtin_popcountll(bal & ltmask);
                                        sPm[p] = m[q];
                                        sPi[p] = ni[q];
                                        sPo[p] = os[q];
                                    }
                                    pos += (uint32_t)__builtin_popcountll(bal);
                                }
                            }
                            nv = pos;
                            qn = (pos + 63) / 64;
#pragma unroll
                            for (int q = 0; q < QL; ++q) {
                                if (q < (int)qn) {
                                    const uint32_t p = q * 64 + lane;
                                    if (p < nv) {
                                        m[q] = sPm[p];
                                        ni[q] = sPi[p];
                                        os[q] = sPo[p];
#pragma unroll
                                        for (int j = 0; j < D; ++j)
                                            x[q][j] = EX ? -2.f * sCx[j][os[q]] : sCx[j][os[q]];
                                        if constexpr (EX) xq[q] = sCc[os[q]] - K2;
                                    }
                                }
                            }
                        }
#pragma unroll
                        for (int j = 0; j < D; ++j) bx[j] = sCx[j][bs];
                        if constexpr (EX) bq = sCc[bs];
                    }
                } while (state == 0);
            };
            if constexpr (KC_LA_INT_FORM(D)) {
                if (exact) lead(std::true_type{});
                else lead(std::false_type{});
            } else {
                lead(std::false_type{});
            }
            for (int u = (int)lane; u < ns; u += 64) {
                if (lb == 0) keys[t0 + u] = sQk[u];
            }
            if (state == 3 && recorder) {
                keys[t] = 0;
                __hip_atomic_store(abort_flag, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicOr(status, 1u);
            }
            if (lane == 0)
                __hip_atomic_store(&sQf[nq], KC_LA_END | state, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_s_setprio(0);
        } else {
            // Two forms of the apply loop: where registers allow, a
            // double-buffered one (no vector copies between steps); for the
            // variants whose points leave no room for it (it would spill
            // VGPRs in this loop), the single-buffer one.  Each is built
            // once per arithmetic form (canonical, or exact-integer), so a
            // loop holds the registers of one form only.
            constexpr bool kDB = PPT * (D + 1) + 3 * D <= 180;
            auto work = [&](auto form) {
                constexpr bool EX = decltype(form)::value;
                // one center: coordinates c, and K + ||c||^2 in the
                // exact-integer form (x then holds -2x)
                auto apply = [&](const float(&c)[D], float cq) {
#pragma unroll
                    for (int p = 0; p < PPT; ++p) {
                        float s;
                        if constexpr (EX) {
                            s = cq;
#pragma unroll
                            for (int j = 0; j < D; ++j) s = __builtin_fmaf(x[p][j], c[j], s);
                        } else {
                            s = 0.f;
#pragma unroll
                            for (int j = 0; j < D; ++j) s = kc_d32_step(s, x[p][j], c[j]);
                        }
                        m[p] = kc_fmin_nn(m[p], s);
                    }
                };
                auto to_sgpr = [](float v) -> float {
                    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
                };
                if constexpr (kDB) {
                    // Apply the queued centers in order.  While the center of
                    // entry i is applied, entry i+1 and its coordinates load
                    // from LDS; the coordinates then move into scalar registers
                    // (they are block-uniform), alternating between two scalar
                    // sets so that no vector copies are needed between steps.
                    auto entry = [&](uint32_t at) -> uint32_t {
                        return __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                            &sQf[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
                    };
                    auto wait_entry = [&](uint32_t at) -> uint32_t {
                        uint32_t e;
                        while ((e = entry(at)) == 0) __builtin_amdgcn_s_sleep(1);
                        return e;
                    };
                    float tv[D], tq = 0.f;   // coordinates (and K + norm) in flight (VGPRs)
                    auto load = [&](uint32_t e) {
#pragma unroll
                        for (int j = 0; j < D; ++j) tv[j] = sCx[j][e - 1];
                        if constexpr (EX) tq = sCc[e - 1];
                    };
                    auto uniform = [&](float(&c)[D], float& cq) {
#pragma unroll
                        for (int j = 0; j < D; ++j) c[j] = to_sgpr(tv[j]);
                        if constexpr (EX) cq = to_sgpr(tq);
                    };
                    float ca[D], cb[D], qa = 0.f, qb = 0.f;   // scalar sets
                    uint32_t i = 0;
                    uint32_t f = wait_entry(0);
                    if (!(f & KC_LA_END)) {
                        load(f);
                        uniform(ca, qa);
                    }
                    while (!(f & KC_LA_END)) {
                        // entry i is a center, its coordinates in ca
                        uint32_t g = entry(++i);
                        if (g != 0 && !(g & KC_LA_END)) load(g);
                        apply(ca, qa);
                        if (g == 0) {
                            g = wait_entry(i);
                            if (!(g & KC_LA_END)) load(g);
                        }
                        if (g & KC_LA_END) {
                            f = g;
                            break;
                        }
                        uniform(cb, qb);
                        // entry i is a center, its coordinates in cb
                        f = entry(++i);
                        if (f != 0 && !(f & KC_LA_END)) load(f);
                        apply(cb, qb);
                        if (f == 0) {
                            f = wait_entry(i);
                            if (!(f & KC_LA_END)) load(f);
                        }
                        if (!(f & KC_LA_END)) uniform(ca, qa);
                    }
                    state = f & ~KC_LA_END;
                } else {
                    // apply the queued centers in order; entry i+1 and its
                    // coordinates are read before center i is applied, so most
                    // of the LDS latency hides behind the arithmetic
                    uint32_t i = 0, f = 0;
                    float cv[D], cvq = 0.f;
                    for (;;) {
                        if (f == 0) {
                            f = __hip_atomic_load(&sQf[i], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
                            if (f == 0) {
                                __builtin_amdgcn_s_sleep(1);
                                continue;
                            }
                            if (!(f & KC_LA_END)) {
#pragma unroll
                                for (int j = 0; j < D; ++j) cv[j] = sCx[j][f - 1];
                                if constexpr (EX) cvq = sCc[f - 1];
                            }
                        }
                        if (f & KC_LA_END) {
                            state = f & ~KC_LA_END;
                            break;
                        }
                        float cc[D];   // uniform: held in SGPRs
#pragma unroll
                        for (int j = 0; j < D; ++j) cc[j] = to_sgpr(cv[j]);
                        const float ccq = EX ? to_sgpr(cvq) : 0.f;
                        ++i;
                        f = __hip_atomic_load(&sQf[i], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (f != 0 && !(f & KC_LA_END)) {
#pragma unroll
                            for (int j = 0; j < D; ++j) cv[j] = sCx[j][f - 1];
                            if constexpr (EX) cvq = sCc[f - 1];
                        }
                        apply(cc, ccq);
                    }
                }
            };
            if constexpr (KC_LA_INT_FORM(D)) {
                if (exact) work(std::true_type{});
                else work(std::false_type{});
            } else {
                work(std::false_type{});
            }
        }
        if (state >= 2) break;
    }
    if (!leader) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const uint32_t i = i0 + p * KC_LA_WPTS;
            float mv = m[p];
            if (exact) {
                float xx = 0.f;
#pragma unroll
                for (int j = 0; j < D; ++j) xx = __builtin_fmaf(x[p][j], x[p][j], xx);
                mv = (m[p] - kc_la_int_offset(D)) + 0.25f * xx;
            }
            if (i < len) mind[base + i] = mv;
        }
    } else if (lb == 0) {
        // keys past an early stop (radius 0, or an abort) read as radius 0
        for (int u = t + (int)lane; u < k; u += 64) keys[u] = 0;
    }
}

// Points per worker lane, two variants per dimension.  Variant 0 balances
// the workers' arithmetic per step against the leader's (the coordinates
// take at most about 130 VGPRs); variant 1 holds as many points as two
// waves per SIMD allow without spilling and serves inputs too large for
// variant 0's co-resident grid.
#define KC_RES_DIMS(X) X(2, 32) X(3, 24) X(8, 12) X(10, 9) X(16, 6) X(32, 3) X(41, 2)
#define KC_RES_DIMS_BIG(X) X(3, 30) X(8, 15) X(10, 14) X(16, 9)

static int resident_ppt(int d, int v)
{
#define KC_CASE(DD, PP) \
    case DD: return PP;
    if (v == 0) {
        switch (d) {
            KC_RES_DIMS(KC_CASE)
        default: return 0;
        }
    }
    if (v == 1) {
        switch (d) {
            KC_RES_DIMS_BIG(KC_CASE)
        default: return 0;
        }
    }
#undef KC_CASE
    return 0;
}

template <int D, int PPT>
static hipError_t launch_resident(uint32_t G, const float* xs, uint64_t stride,
                                  uint64_t base, uint32_t len, const uint32_t* len_ptr,
                                  uint32_t first, int k,
                                  float* mind, u64* keys, u64* xbuf, uint32_t* abort_flag,
                                  uint32_t spin_limit, const float* xa, int64_t lda,
                                  int xa_rows, uint32_t* status, const KcSeg* segs,
                                  const uint4* blks, const float* mind_in, hipStream_t s)
{
    void* args[] = {(void*)&xs,    (void*)&stride, (void*)&base, (void*)&len,
                    (void*)&len_ptr, (void*)&first, (void*)&k,      (void*)&mind, (void*)&keys,
                    (void*)&xbuf, (void*)&abort_flag, (void*)&spin_limit, (void*)&xa,
                    (void*)&lda, (void*)&xa_rows, (void*)&status, (void*)&segs, (void*)&blks,
                    (void*)&mind_in};
    return hipLaunchCooperativeKernel((const void*)k_gon_resident<D, PPT>, dim3(G),
                                      dim3(KC_LA_BLOCK), args, 0, s);
}

template <int D, int PPT>
static int max_resident_blocks()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gon_resident<D, PPT>,
                                                     KC_LA_BLOCK, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;   // no resident grid: the caller streams
    }
    const int g = per_cu * cus;
    return g < KC_LA_GMAX ? g : KC_LA_GMAX;   // the exchange buffer's capacity
}

int kc_resident_max_blocks(int d, int v)
{
#define KC_CASE(DD, PP) \
    case DD: return max_resident_blocks<DD, PP>();
    if (v == 0) {
        switch (d) {
            KC_RES_DIMS(KC_CASE)
        default: return 0;
        }
    }
    if (v == 1) {
        switch (d) {
            KC_RES_DIMS_BIG(KC_CASE)
        default: return 0;
        }
    }
#undef KC_CASE
    return 0;
}

uint32_t kc_resident_block_points(int d, int v)
{
    return (uint32_t)resident_ppt(d, v) * KC_LA_WPTS;
}

uint32_t kc_resident_blocks_for(int d, int v, uint64_t len)
{
    const uint64_t per = (uint64_t)resident_ppt(d, v) * KC_LA_WPTS;
    if (per == 0) return 0;
    const uint64_t g = (len + per - 1) / per;
    return g > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)g;
}

// Estimated cycles of one launch of variant v for k steps: each step costs
// the larger of the leader's selection (about 1,600 cycles) and a worker
// SIMD's arithmetic (two waves, PPT points of 2d+1 VALU instructions, 4
// cycles each); each lookahead round adds about 16,800 cycles (7 us) of
// publication and exchange, and clustered inputs certify about 6 steps per
// round.  Used only to choose between packings of a batch.
double kc_resident_launch_cycles(int d, int v, uint32_t k)
{
    const double ppt = resident_ppt(d, v);
    const double step = std::max(1600.0, ppt * (2.0 * d + 1.0) * 8.0);
    return (double)k * step + ((double)k / 6.0) * 16800.0;
}

// Whether the kernel for dimension d can load its points straight from rows
// xa of lda floats: its vector loads need the base and the row stride
// aligned to their width, and byte offsets of up to `span` rows from a
// segment's first row must fit 32 bits.
bool kc_resident_rows_ok(int d, const float* xa, int64_t lda, uint64_t span)
{
    if (!xa || lda < d) return false;
    const int vw = d % 4 == 0 ? 4 : d % 2 == 0 ? 2 : 1;   // the kernel's load width
    if ((uintptr_t)xa % (uintptr_t)(4 * vw) != 0 || lda % vw != 0) return false;
    return span * (uint64_t)lda * 4ull < (1ull << 32);
}

// Exchange buffer of the engine (two rounds), to be zero-filled before each
// launch; independent of k and of the grid size.
uint64_t kc_resident_slot_words(int k, uint32_t G)
{
    (void)k;
    (void)G;
    return 2ull * KC_LA_BUF;
}

// Returns hipSuccess, or an error when the shape has no resident kernel or
// the grid cannot be co-resident (the caller then streams instead).
hipError_t kc_gon_resident(int d, int v, uint32_t G, const float* xs, uint64_t stride,
                           uint64_t base, uint32_t len, const uint32_t* len_ptr,
                           uint32_t first, int k, float* mind,
                           u64* keys, u64* slots, uint32_t* abort_flag, uint32_t spin_limit,
                           const float* xa, int64_t lda, int xa_rows, uint32_t* status,
                           const KcSeg* segs, const uint4* blks, hipStream_t s,
                           const float* mind_in)
{
    if (G == 0 || G > KC_LA_GMAX) return hipErrorInvalidValue;
    if (xa_rows && !xa) return hipErrorInvalidValue;
#define KC_CASE(DD, PP)                                                                  \
    case DD:                                                                             \
        return launch_resident<DD, PP>(G, xs, stride, base, len, len_ptr, first, k, mind, keys, \
                                       slots, abort_flag, spin_limit, xa, lda, xa_rows,      \
                                       status, segs, blks, mind_in, s);
    if (v == 0) {
        switch (d) {
            KC_RES_DIMS(KC_CASE)
        default: return hipErrorInvalidValue;
        }
    }
    if (v == 1) {
        switch (d) {
            KC_RES_DIMS_BIG(KC_CASE)
        default: return hipErrorInvalidValue;
        }
    }
#undef KC_CASE
    return hipErrorInvalidValue;
}
