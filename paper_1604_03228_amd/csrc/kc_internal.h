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

// Source rows of one segment of a run (device table, one per segment, when
// the segments read different arrays): X NULL when the segment is filled
// otherwise (a gathered union).
struct KcSrc {
    const float* X;
    const uint16_t* Xb;
    int64_t ld;
    int64_t pad;
};

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
    const KcSrc* srcs = nullptr;  // per-segment sources, when they differ
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
// The same with each segment's own source rows (srcs[segment]).
void kc_stage_rows_src(const KcSrc* srcs, bool bf, int d, const KcSeg* segs,
                       const uint32_t* blk_seg, const uint32_t* blk_start, uint32_t nblk,
                       uint32_t tile, float* xs, uint16_t* xb, float* ex, uint64_t stride,
                       hipStream_t s);
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

// Staged centers of an MFMA distance pass (device arrays of kpad entries,
// padding entries with cn = cnl = +inf).
struct KcCenters {
    float* Cf = nullptr;     // [kpad][dp] FP32 coordinates
    float* Ct = nullptr;     // [kpad][dp] the same translated to mu (FP32
                             // passes with a local origin; the MFMA reads it)
    uint16_t* Cb = nullptr;  // [kpad][dp] BF16 bits (BF16 passes), or the
                             // high parts of the translated FP32 values
    uint16_t* Cbl = nullptr; // [kpad][dp] their low parts (split passes:
                             // FP32 inputs on three BF16 MFMAs)
    bool pk = false;         // packed split: Cb holds [h | l | h] rows of dp
                             // (kc_split_packed_ksteps), Cbl unused
    float* cn = nullptr;     // |c|^2 of the MFMA inputs, in FP32
    float* cnl = nullptr;    // cn - (g |c|^2 + 2 e_c |c|)
    float* clen = nullptr;   // |c| of the MFMA inputs, rounded up
    float* cerr = nullptr;   // BF16 rounding radius e_c, rounded up (BF16 passes)
    float* cmax = nullptr;   // [2]: the largest clen and cerr
    const float* mu = nullptr;  // FP32 passes: local origin subtracted from
                                // points and centers before the MFMA (or NULL)
    uint32_t kpad = 0;
    int dp = 0;
};

// Per-point outputs of an MFMA distance pass (device arrays of n entries).
struct KcMinOut {
    int32_t* arg = nullptr;  // best center (smallest v, lowest index on ties)
    float* m1 = nullptr;     // its v = |c|^2 - 2 x.c
    float* lo2 = nullptr;    // smallest lower-bound term w over the other
                             // centers (labels pass), or the per-chunk lower
                             // term (radius passes on FP32 inputs)
    float* lob = nullptr;    // the best center's w (labels pass)
    float* nx = nullptr;     // |x|^2 of the MFMA inputs
};

// Relative error constant of the MFMA distance: (6d + 44) u, u = 2^-24
// (including the rounding of a translation to the local origin), plus
// 3.1 * 2^-18 for FP32 inputs split into BF16 high and low parts (the
// dropped products of the split, kc_assign.hip).
__host__ __device__ inline double kc_md_gamma(int d, bool split = false)
{
    return (6.0 * d + 44.0) * 5.9604644775390625e-8 + (split ? 3.1 * 3.814697265625e-6 : 0.0);
}

struct KcMdBounds {
    double hi;        // >= the exact squared distance to the best center
    double lo_min;    // <= the exact squared distance to every center
    double lo_other;  // <= the exact squared distance to every other center
                      // (labels pass; +inf when there is no other)
};

// Certified bounds of point p from an MFMA pass (see kc_assign.hip): with
// a = |x|, b = |c| (of the translated values when a local origin is used),
// E = e_x + e_c,
//   D <= (sqrt(|x|^2 + v + g (a+b)^2) + E)^2,
//   D >= (sqrt(max(0, |x|^2 + v - g (a+b)^2)) - E)^2  (for the best center),
//   D >= |x|^2 - (g a^2 + 2 e_x a) + w                 (labels pass, any center).
// Without labels, FP32 inputs: the kernel's per-chunk terms, min_j D_j in
// [|x|^2 + lo2, |x|^2 + m1]; BF16 inputs: the smallest v, with b and e_c
// the largest over the centers.
__device__ inline KcMdBounds kc_md_bounds(const KcMinOut& O, uint32_t p,
                                          const float* __restrict__ ex, const KcCenters& C,
                                          int d, bool lab)
{
    KcMdBounds B;
    const bool bf_in = C.Cb && !C.Cbl && !C.pk;   // BF16 inputs (not a split)
    const double g = kc_md_gamma(d, C.Cbl != nullptr || C.pk);
    const double nx = O.nx[p];
    if (!lab && !bf_in) {
        B.hi = (nx + (double)O.m1[p]) * (1.0 + 1e-12) + 1e-30 * d;
        const double l = (nx + (double)O.lo2[p]) * (1.0 - 1e-12) - 1e-30 * d;
        B.lo_min = l > 0.0 ? l : 0.0;
        B.lo_other = __builtin_inf();
        return B;
    }
    const double a = sqrt(nx) * (1.0 + (d + 4) * 5.9604644775390625e-8) * (1.0 + 1e-6);
    const double e_x = (bf_in && ex) ? (double)ex[p] : 0.0;
    const double P0 = (g * a * a + 2.0 * e_x * a) * (1.0 + 1e-12);
    const int32_t a1 = lab ? O.arg[p] : 0;
    if (a1 < 0 || (uint32_t)a1 >= C.kpad) {
        B.hi = __builtin_inf();
        B.lo_min = 0.0;
        B.lo_other = 0.0;
        return B;
    }
    const double b1 = lab ? (double)C.clen[a1] : (double)C.cmax[0];
    const double E = e_x + (C.cerr ? (double)(lab ? C.cerr[a1] : C.cmax[1]) : 0.0);
    const double s = a + b1;
    const double err = g * s * s + 1e-30 * d;
    const double d1 = nx + (double)O.m1[p];
    const double rh = sqrt(d1 + err) + E;
    B.hi = rh * rh * (1.0 + 1e-12);
    double l = d1 - err;
    l = l > 0.0 ? sqrt(l) - E : 0.0;
    l = l > 0.0 ? l * l * (1.0 - 1e-12) : 0.0;
    if (lab) {
        const double lo2 = nx - P0 + (double)O.lo2[p];
        const double lb = nx - P0 + (double)O.lob[p];
        if (lb > l) l = lb;
        B.lo_other = lo2;
        B.lo_min = lo2 < l ? lo2 : l;
    } else {
        B.lo_other = __builtin_inf();
        B.lo_min = l;
    }
    if (!(B.lo_min > 0.0)) B.lo_min = 0.0;
    return B;
}

int kc_mindist_ksteps(int d, bool bf);
// Status bit of a non-finite input coordinate (option "validate").
#define KC_STATUS_NONFINITE 8u
int kc_mindist_dpad(int d, bool bf);
// K-steps of the packed split for dimension d (0: it would not use fewer
// MFMAs than the three-chain split); whether a split pass over kpad centers
// packs; and its staged row length (packed or not).
int kc_split_packed_ksteps(int d);
bool kc_split_use_packed(int d, uint32_t kpad);
int kc_mindist_dpad_split(int d, uint32_t kpad);
// One MFMA pass of every point against the staged centers (lab: labels
// pass); ex: the points' BF16 rounding radii (BF16 passes); waves: 4 or 8
// waves per block; lds_kib: 64 or 32 KiB of staged centers per block (more
// blocks per CU, more chunks); the results depend on neither.
// With `rows`, output entry p reads row rows[p]; with `n_dev`, the entries
// are min(n, *n_dev) (a device-side count: the grid covers n, blocks past
// the count leave at once).
void kc_mindist(const float* X, const uint16_t* Xb, const float* ex, int64_t ld, uint32_t n,
                int d, const KcCenters& C, const KcMinOut& O, bool lab, hipStream_t s,
                int waves = 4, int lds_kib = 64, const uint32_t* rows = nullptr,
                const uint32_t* n_dev = nullptr);
void kc_stage_centers(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n,
                      const int64_t* idx, const uint32_t* idx32, uint32_t k,
                      const int64_t* k_dev, const KcCenters& C, uint32_t* status, hipStream_t s);
// mu[j] = the median of coordinate j over up to 256 points spread evenly
// over X (a local origin for FP32 MFMA passes: translating to it shrinks the
// norms the error bound scales with); d <= KC_MAXD.
void kc_local_origin(const float* X, int64_t ld, int d, uint32_t n, float* mu, hipStream_t s);
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
// Second pass of an assignment on BF16 inputs: the points the first pass
// lists (labels it cannot certify, possible maximisers of the radius) run
// the MFMA pass again on their FP32 rows, without the BF16 rounding radii;
// only what that leaves uncertain goes to FP64.
struct KcAssignRefine {
    KcCenters C;            // the centers staged from their FP32 rows
    KcMinOut O;             // per list entry (2n)
    float* hi = nullptr;    // per list entry (2n)
    uint32_t* list = nullptr;    // rows for FP64 (4n)
    uint32_t* nlist = nullptr;
};
void kc_assign_finish(uint32_t n, int d, const float* X, int64_t ld, const KcCenters& C,
                      uint32_t k, const int64_t* k_dev, const KcMinOut& O, const float* ex,
                      int32_t* labels, float* hi, uint32_t* list, uint32_t* nlist,
                      float* lo_max, double* radius2, double* radius_out, hipStream_t s,
                      const KcAssignRefine* R2 = nullptr);
