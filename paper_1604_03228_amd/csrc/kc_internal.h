// kc_internal.h -- launchers shared between the kernel files and the host
// library of libkcenter (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "kc_device.h"

static inline uint32_t kc_pad64(uint32_t n) { return (n + 63u) & ~63u; }

// Relative error bound of the canonical FP32 squared distance in d
// dimensions: gamma_{d+2} with u = 2^-24.
static inline double kc_gamma32(int d)
{
    const double u = 5.9604644775390625e-8;
    const double m = (double)(d + 2);
    return m * u / (1.0 - m * u);
}

// Everything the step engines and the finishing kernels of one batched
// Gonzalez run need (device pointers unless noted).
struct KcGonRun {
    int d = 0;
    int nseg = 0;
    uint32_t kmax = 0;          // largest ksteps over segments (host)
    const float* xs = nullptr;  // SoA staging copy
    const float* xa = nullptr;  // the caller's rows (nullable): finishing gathers read them
    int64_t lda = 0;            //   row stride of xa, in floats
    uint64_t stride = 0;        // columns per coordinate row
    float* mind = nullptr;      // [stride]
    u64* keys = nullptr;        // [sum ksteps]
    u64* part = nullptr;        // [sum ksteps][KC_PARTS][KC_PSTRIDE] partial keys
    KcSeg* segs = nullptr;      // [nseg]
    uint32_t* blk_seg = nullptr;
    uint32_t* blk_start = nullptr;
    uint32_t nblk = 0;          // tiles of 1024 points (host)
    uint32_t* pairs_seg = nullptr;  // (segment, step) pairs, one per key
    uint32_t* pairs_t = nullptr;
    uint32_t npairs = 0;
    float* ccoord = nullptr;    // [sum ksteps][d]
    double* radius2 = nullptr;  // [nseg]
    u64* cand = nullptr;        // [cand_cap]
    uint32_t* ncand = nullptr;  // [1]
    uint32_t* ticket = nullptr; // [1] blocks done, for the one-segment exact radius
    uint32_t cand_cap = 0;
    double band = 0.0;          // 2 gamma_{d+2} + 4u
    uint64_t keysum = 0;        // keys in use (host)
    uint32_t tile = 1024;       // points per step block (host)
    // host [kmax]: blocks still active at step t when segments are ordered by
    // descending k (their tiles then form a prefix); NULL: all blocks
    const uint32_t* nblk_at = nullptr;
    uint64_t plan_hash = 0;     // geometry of the plan (host), part of graph keys
};

void kc_fill_u64(u64* p, u64 v, uint64_t n, hipStream_t s);
void kc_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void kc_stage_soa(const float* X, int64_t ld, int d, uint64_t row0, uint32_t len,
                  float* xs, uint64_t stride, uint64_t base, hipStream_t s);
// Staging through LDS (kc_gon.hip): FP32 SoA copy (xs) and, with Xb, the
// BF16 SoA copy (xb) and per-point rounding radius (ex); either output may
// be NULL.  The batch form stages every segment of a plan from one array.
void kc_stage_rows(const float* X, const uint16_t* Xb, int64_t ld, int d, uint64_t row0,
                   uint32_t len, float* xs, uint16_t* xb, float* ex, uint64_t stride,
                   uint64_t base, hipStream_t s);
void kc_stage_rows_batch(const float* X, const uint16_t* Xb, int64_t ld, int d,
                         const KcSeg* segs, const uint32_t* blk_seg, const uint32_t* blk_start,
                         uint32_t nblk, uint32_t tile, float* xs, uint16_t* xb, float* ex,
                         uint64_t stride, hipStream_t s);
void kc_part_collect(const u64* part, u64* keys, uint64_t nkeys, hipStream_t s);
uint64_t kc_resident_slot_words(int k, uint32_t G);
void kc_gon_step(const float* xs, uint64_t stride, int d, float* mind, u64* part,
                 const KcSeg* segs, const uint32_t* blk_seg, const uint32_t* blk_start,
                 uint32_t nblk, int t, hipStream_t s);
// Resident engine variants (v = 0: balanced, 1: most points per block; a
// dimension without a kernel of that variant reports 0 points / blocks).
int kc_resident_max_blocks(int d, int v);
uint32_t kc_resident_blocks_for(int d, int v, uint64_t len);
uint32_t kc_resident_block_points(int d, int v);
double kc_resident_launch_cycles(int d, int v, uint32_t k);
bool kc_resident_rows_ok(int d, const float* xa, int64_t lda, uint64_t span);
// `xa` (nullable): the same points as rows of lda floats (the caller's
// array), used to gather candidate coordinates; NULL gathers from xs.  With
// xa_rows (only where kc_resident_rows_ok holds for the longest segment) the
// points are loaded from xa too and xs is not read.  A wait that exceeds the
// spin limit raises abort_flag and bit 0 of *status.
// With `mind_in` (nullable, indexed like `mind`) every point's min-distance
// starts as its value there (a run resumed after earlier centers).
// With `blks` (device, one uint4 per block: segment, block within it, blocks
// of the segment, first block of the segment) the launch runs several
// segments of `segs` at once and base/len/first/k come from each segment
// (keys at its keyoff, xa rows from its src).
hipError_t kc_gon_resident(int d, int v, uint32_t G, const float* xs, uint64_t stride,
                           uint64_t base, uint32_t len, const uint32_t* len_ptr,
                           uint32_t first, int k, float* mind,
                           u64* keys, u64* slots, uint32_t* abort_flag,
                           uint32_t spin_limit, const float* xa, int64_t lda, int xa_rows,
                           uint32_t* status, const KcSeg* segs, const uint4* blks,
                           hipStream_t s, const float* mind_in = nullptr);
void kc_gon_finish(const KcGonRun& R, int64_t* centers, int64_t* n_chosen, double* trace,
                   double* radius_out, const int64_t* report_base, const int64_t* remap,
                   hipStream_t s);
// The finishing sequence with a caller-supplied radius-candidate launch;
// `gather` copies the chosen centers' coordinates from the SoA staging copy.
void kc_gon_finish_impl(const KcGonRun& R, int64_t* centers, int64_t* n_chosen,
                        double* trace, double* radius_out, const int64_t* report_base,
                        const int64_t* remap, bool gather, hipStream_t s,
                        const std::function<void(hipStream_t)>& radius_cand);

// BF16 stream state (kc_bf16.hip); tiles of KC_BLOCK*8 points.
struct KcBf16Run {
    uint16_t* xb = nullptr;       // SoA BF16 copy [d][stride]
    float* ex = nullptr;          // [stride] per-point BF16 rounding radius
    uint32_t* lpart = nullptr;    // [sum ksteps][KC_PARTS][32] max lower bound
    u64* list = nullptr;          // [KC_PARTS * region] listed points of a step
    float* list_hi = nullptr;     // [KC_PARTS * region] their upper bounds
    uint32_t* listcnt = nullptr;  // [kmax][KC_PARTS][32] listed points per region
    uint32_t region = 0;          // entries per list region (host)
    uint32_t* nresc = nullptr;    // [kmax] rescored points per step
    float* exm = nullptr;         // [stride] cached exact FP32 min-distance
    uint32_t* exupto = nullptr;   // [stride] centers covered by exm
    float* Lt = nullptr;          // [nseg] L_t of the current step (many-segment runs)
    uint32_t rescore_blocks = 256;
    float g = 0.f;                // gamma_{d+2} + 16u
};
#define KC_BF_TILE_PTS (KC_BLOCK * 8)

// MFMA nearest-center distances (kc_assign.hip)
int kc_mindist_ksteps(int d, bool bf);
int kc_mindist_dpad(int d, bool bf);
// arg == NULL: only m1 (the smallest |c|^2 - 2x.c) and nx are written.
void kc_mindist(const float* X, const uint16_t* Xb, int64_t ld, uint32_t n, int d,
                const float* Cf, const uint16_t* Cb, const float* cnorm, uint32_t kpad,
                int32_t* arg, float* m1, float* m2, float* nx, hipStream_t s);
void kc_stage_centers(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n,
                      const int64_t* idx, const uint32_t* idx32, uint32_t k,
                      const int64_t* k_dev, uint32_t kpad, int dp, float* Cf, uint16_t* Cb,
                      float* cnorm, float* cmax, uint32_t* status, hipStream_t s);
void kc_bf16_err(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n, float* ex,
                 hipStream_t s);
// Covering radius only (no labels), FP32 points, d <= 8: canonical FP32
// distances to the staged centers Cf (rows of dp floats), then the exact
// FP64 pass over the points that may attain the radius.  Returns false
// (nothing enqueued) for other d.
bool kc_radius_direct(uint32_t n, int d, const float* X, int64_t ld, const float* Cf, int dp,
                      uint32_t k, const int64_t* k_dev, float* hi, uint32_t* list,
                      uint32_t* nlist, float* lo_max, double* radius2, double* radius_out,
                      hipStream_t s);
void kc_assign_finish(uint32_t n, int d, const float* X, int64_t ld, const float* Cf, int dp,
                      uint32_t k, const int64_t* k_dev, const int32_t* arg, const float* m1,
                      const float* m2, const float* nx, const float* ex, const float* cmax,
                      int32_t* labels, float* hi, uint32_t* list, uint32_t* nlist,
                      float* lo_max, double* radius2, double* radius_out, hipStream_t s);
