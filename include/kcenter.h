/*
 * kcenter.h -- C ABI of libkcenter, the MI355X (gfx950) k-center hot path of
 * McClintock & Wirth, "Efficient Parallel Algorithms for k-Center
 * Clustering" (arXiv 1604.03228).
 *
 * Common rules for every entry point
 * ----------------------------------
 * Points.   A kc_points names a row-major FP32 array X[n][ld] in device
 *           memory (only the first d columns are read), optionally with a
 *           BF16 copy B[n][ld] (bit patterns, device memory).  The distance
 *           is Euclidean (Section 7.2: computed from coordinates as needed).
 * Indices.  Point indices are int64 row numbers of X.  Reported radii are
 *           Euclidean distances in FP64.
 * Ties.     Among equally far points the lowest index wins; among equally
 *           near centers the lowest center position wins.  The paper leaves
 *           these choices arbitrary but consistent (Sections 3.1, 6).
 * Streams.  `stream` is a hipStream_t (NULL: the default stream).  Every
 *           call only enqueues work on it and returns; results are valid once
 *           the stream has synchronised.  Exceptions are stated per call.
 * Memory.   The caller owns every input and output buffer.  The library
 *           owns only its workspace (held by the handle, grown on demand with
 *           hipMalloc, freed by kc_destroy) and never frees caller memory.
 *           Calls on one handle must not overlap (one stream at a time).
 *           Small host tables (partition and tile lists) reach the device by
 *           copies ordered on the call's stream, from pinned staging buffers
 *           the handle owns; a call whose tables are unchanged copies none.
 *           Destroy every handle before the process exits (while the HIP
 *           runtime is still up).
 * Errors.   Every entry point returns KC_OK or a negative kc_status.  All
 *           argument checks happen on the host before any device work; a
 *           failed check enqueues nothing.  kc_last_error() gives the text of
 *           the last failure on a handle.  Nothing aborts or throws.
 * Inputs.   Non-finite coordinates give unspecified (but memory-safe)
 *           results; option "validate" flags them in the device status
 *           word.  n must be below 2^32 - 1 and d at most 256.
 */
#ifndef KCENTER_H
#define KCENTER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kc_handle kc_handle;

typedef enum {
    KC_OK = 0,
    KC_EINVAL = -1,        /* invalid argument                              */
    KC_ENOMEM = -2,        /* workspace allocation failed                   */
    KC_EHIP = -3,          /* a HIP runtime call failed                     */
    KC_ENOCONV = -4,       /* EIM did not converge; an MRG pass kept all    */
    KC_EUNSUPPORTED = -6,  /* valid request this library cannot serve       */
    KC_EDEVICE = -7        /* a device-side check failed (see kc_device_status) */
} kc_status;

typedef enum {
    KC_FP32 = 0,           /* stream FP32 points                            */
    KC_BF16_RESCORE = 1    /* stream BF16 points, rescore near-ties in FP32 */
} kc_precision;

typedef struct {
    const float* f32;      /* device [n][ld] FP32, required                  */
    const uint16_t* bf16;  /* device [n][ld] BF16 bits; required iff
                              prec == KC_BF16_RESCORE, ignored otherwise     */
    int64_t n;             /* points, 1 <= n < 2^32 - 1                      */
    int32_t d;             /* coordinates per point, 1 <= d <= 256           */
    int64_t ld;            /* row stride in elements, ld >= d                */
    int32_t prec;          /* kc_precision                                   */
} kc_points;

/* Handle life cycle.  kc_create binds the handle to the current HIP device
 * (and looks up that device's address of the no-allocation array, once per
 * device).  Returns KC_OK, KC_EINVAL (out == NULL), KC_ENOMEM or KC_EHIP. */
int kc_create(kc_handle** out);
void kc_destroy(kc_handle* h);
const char* kc_strerror(int status);
const char* kc_last_error(const kc_handle* h);

/* Options (name, value): "graphs" 0/1 (capture per-step launches in a HIP
 * graph, default 1); "resident" 0/1 (use the register-resident Gonzalez
 * engines -- the persistent grid, or one workgroup for small inputs -- when
 * the points fit, default 1); "resident_blocks" (at
 * most this many blocks per persistent launch, 0 = as many as are
 * co-resident, the default; a testing aid: smaller grids hold fewer points,
 * so more inputs stream and MRG partitions spread over more launches);
 * "timing" 0/1 (record kernel timing events, default 0); "spin_limit"
 * (polls before a persistent kernel's barrier wait gives up, default 2^20);
 * "mfma_split" 0/1 (FP32 distance passes of assignments and EIM on split
 * BF16 MFMAs -- each FP32 operand as a sum of two BF16 values, three
 * products -- instead of the FP32 MFMA, default 1; results are identical,
 * only the certified bounds and so the speed differ); "autotune" 0/1
 * (default 1: the first call of a shape bucket -- dimension, and n, k or
 * sample size rounded to half powers of two -- times every feasible variant
 * of its engine once and the handle keeps the fastest; the variants give
 * identical results; a call made during stream capture never tunes);
 * "tune_force" (-1 default; v >= 0: every tuned operation runs its variant v
 * where that is feasible, else its first feasible one -- a testing aid that
 * reaches each variant; the variants are listed with kc_tune_report);
 * "validate" 0/1 (default 0: every call first scans its points, and the BF16
 * copy when one is used, for non-finite values on the device and sets bit 3
 * of the device status word when it finds one; no host wait -- read it with
 * kc_device_status).
 * KC_EINVAL for an unknown name or a value out of range. */
int kc_set_option(kc_handle* h, const char* name, int64_t value);

/* The autotuner's choices on this handle as text: one line per shape
 * bucket, "<key> <chosen variant> <ms of variant 0> <ms of variant 1> ...",
 * -1 for a variant that could not run.  Keys: "gon/d/a/b/rows" (Gonzalez,
 * a = floor(2 log2 n), b = floor(2 log2 k); variants resident v0, resident
 * v1, streaming, one workgroup for small n), "eim/d/a/b" (EIM distance pass, a and b of the candidate
 * and new-sample counts; variants 0 direct VALU for d <= 8, 1 FP32 MFMA,
 * 2-5 split MFMA with 4 / 8 waves per block and 64 KiB of staged samples,
 * then 8 / 4 waves with 32 KiB; an MFMA pass's undecided candidates are
 * refined in canonical FP32 before FP64), "assign/d/a/b/l/m" (the
 * assignment's MFMA pass, a and b of n and k, l = labels, m = input mode;
 * variants 0-3: 4 / 8 waves per block with 64 KiB of staged centers, then
 * 4 / 8 waves with 32 KiB).  Writes at most `cap` bytes (NUL-terminated) to
 * the host buffer `buf` and the needed size to *need; with cap = 0 (buf may
 * be NULL) it only sets *need.  KC_EINVAL for a NULL handle or need, or
 * when 0 < cap < *need (nothing written). */
int kc_tune_report(kc_handle* h, char* buf, int64_t cap, int64_t* need);

/* Kernel timing.  With option "timing" = 1 every call records a pair of HIP
 * events on its stream around its dominant kernel or launch sequence, under
 * one of the names "gon_resident" (persistent Gonzalez, 1 launch),
 * "gon_step" (k streaming step launches), "gon_bf16" (BF16 stream steps),
 * "mrg_round1" (MRG first round: its persistent launches, or its
 * streaming step launches), "mrg_rounds" (each round of kcenter_mrg_rounds), "assign_mfma" (the MFMA
 * distance kernel of an assignment), "assign_direct" (a radius-only assignment at d <= 8: canonical
 * FP32 distances, candidate listing and the exact FP64 pass), "eim_dist" (EIM distance passes).
 * kc_timing_read synchronises the device, returns the summed milliseconds,
 * the number of kernel launches those intervals cover and the number of
 * intervals, for one name, and forgets them.  KC_EINVAL for NULL args. */
int kc_timing_read(kc_handle* h, const char* name, double* ms, int64_t* launches,
                   int64_t* intervals);

/* Work counters of the most recent BF16+rescore Gonzalez run on the handle
 * (synchronises the device): "bf16_listed" is the number of (point, step)
 * pairs listed by the stream as possible candidates, "bf16_rescored" the
 * number rescored exactly in FP32.  "eim_refined": candidates an MFMA
 * distance pass of the most recent kcenter_eim call (or batch) left
 * undecided, which were then bounded in canonical FP32 (summed over its
 * iterations).
 * "eim_exact": candidates whose keep /
 * remove decision the most recent kcenter_eim call on the handle made in
 * exact FP64 (summed over its iterations; a batch sums over its EIM
 * problems that sample).  "assign_rescored": points the most recent assignment on the
 * handle rescored in FP64 (uncertified nearest center, or a possible
 * maximiser of the radius; a point may count twice).  "resident_integer":
 * segments that the register-resident Gonzalez engine ran in its
 * exact-integer form (d >= 8, every coordinate an integer of magnitude at
 * most M with 5 d M^2 <= 2^24) since kc_device_status last cleared the
 * handle's status (direct calls only: a batch runs on its plan's own
 * status words).  KC_EINVAL for an unknown name. */
int kc_counter_read(kc_handle* h, const char* name, int64_t* value);

/* Synchronises `stream`, then reads and clears the handle's device status
 * word (bit 0: a persistent kernel's grid barrier timed out; bit 2: a center
 * index passed to an assignment is out of range (it is read as point 0);
 * bit 3: a non-finite input coordinate, with option "validate").  *status
 * receives the word.  Returns KC_OK, or KC_EDEVICE when the word was
 * non-zero. */
int kc_device_status(kc_handle* h, void* stream, uint32_t* status);

/*
 * kcenter_gonzalez -- Gonzalez's farthest-first traversal (Section 3.1; its
 * cost model in Section 5.1).  The first center is `first`; each later center
 * is a point farthest from the centers chosen so far, until k are chosen or
 * every point coincides with a center (the problem asks for at most k
 * centers, Section 1.1).
 *   pts           points (prec selects the FP32 or BF16+rescore stream; both
 *                 choose the same centers).  Integer coordinates within the
 *                 bound of counter "resident_integer" (d >= 8) run the
 *                 register-resident engine's exact-integer form; its keys,
 *                 centers and trace equal the canonical FP32 path's.
 *   k             centers wanted, k >= 1 (k >= n is allowed).
 *   first         index of the first center, 0 <= first < n.
 *   centers       device int64 [k]: chosen indices in selection order, -1
 *                 after an early stop.
 *   radius_trace  device double [k] or NULL: radius_trace[t] is the FP64
 *                 distance of the point chosen at step t+1 to its nearest of
 *                 centers 0..t, i.e. the covering radius after t+1 centers
 *                 (within the FP32 tie band of the exact value); the entry of
 *                 the last chosen center is the exact FP64 covering radius of
 *                 all chosen centers; 0 after an early stop.
 *   n_chosen      device int64 [1]: number of centers chosen.
 */
int kcenter_gonzalez(kc_handle* h, const kc_points* pts, int64_t k, int64_t first,
                     int64_t* centers, double* radius_trace, int64_t* n_chosen,
                     void* stream);

/*
 * kcenter_gonzalez_resume -- Gonzalez's traversal continued from a saved
 * prefix of centers (checkpoint / resume).  The traversal of Section 3.1
 * picks each center from the centers chosen so far alone, so with
 * prefix = the first p centers of an earlier run (same points, same or
 * smaller k) the result is exactly the run with k centers.  Centers
 * 0..p-1 are prefix[0..p-1], all kept as given; every later center is a
 * farthest point (lowest index on ties) from the centers so far, until k
 * are chosen or, after the prefix, every point coincides with a center.
 * Runs on the FP32 points in either precision.
 *   prefix        HOST int64 [p]: distinct indices in [0, n); 1 <= p <= k.
 *                 Out-of-range or repeated indices, or p outside [1, k],
 *                 return KC_EINVAL before any work.
 *   k             centers wanted, 1 <= k < 2^24.
 *   centers       device int64 [k] (-1 after an early stop), n_chosen
 *                 device int64 [1].
 *   radius_trace  device double [k] or NULL: entry t < n_chosen-1 is the FP64
 *                 distance of center t+1 to its nearest of centers 0..t (for
 *                 a free step: the covering radius after t+1 centers, as in
 *                 kcenter_gonzalez); the last chosen entry is the exact FP64
 *                 covering radius of all chosen centers; 0 after it.
 */
int kcenter_gonzalez_resume(kc_handle* h, const kc_points* pts, const int64_t* prefix,
                            int64_t p, int64_t k, int64_t* centers, double* radius_trace,
                            int64_t* n_chosen, void* stream);

/*
 * kcenter_mrg -- two-round MRG (Algorithm 1 with one pass of its loop;
 * Lemma 2 gives the factor 4).  Round 1 runs Gonzalez(k) on each partition
 * (first center: the partition's first point), all partitions in the same
 * launches; round 2 runs Gonzalez(k) on the union of their centers in
 * ascending index order (first center: the smallest index); the result is
 * assigned to all points for its covering radius.  When every partition
 * fits a register-resident grid, round 1 runs on the resident engine from
 * the FP32 points in either precision (there is then no stream for BF16 to
 * shorten); otherwise it streams, in BF16 with exact FP32 rescoring when
 * pts->prec asks for it.  Both precisions choose the same centers.
 *   offsets   HOST int64 [m+1], 0 = o_0 <= o_1 <= ... <= o_m = n: partition
 *             p is rows [o_p, o_{p+1}); empty partitions are allowed.
 *   m         partitions, 1 <= m.
 *   k         centers, k >= 1.
 *   centers   device int64 [k] (-1 padded), n_centers device int64 [1].
 *   radius    device double [1]: exact FP64 covering radius over all points.
 *   round1    device int64 [m*k] or NULL: partition p's centers at p*k.
 *   r1        device double [m] or NULL: round-1 covering radius per
 *             partition (0 if empty).
 *   uni       device int64 [m*k] or NULL: the union, ascending, and
 *   n_union   device int64 [1] or NULL: its size.
 *   r2        device double [1] or NULL: round-2 covering radius of the union.
 */
int kcenter_mrg(kc_handle* h, const kc_points* pts, const int64_t* offsets, int32_t m,
                int64_t k, int64_t* centers, int64_t* n_centers, double* radius,
                int64_t* round1, double* r1, int64_t* uni, int64_t* n_union,
                double* r2, void* stream);

/*
 * kcenter_mrg_rounds -- MRG with its loop (Algorithm 1 with machine capacity
 * c; Lemma 3 and Eq. 1: i passes of the loop then the last round give a
 * 2(i+1)-approximation).  The sample S starts as all points.  While |S| > c,
 * S is split into ceil(|S| / c) contiguous blocks of its ascending index
 * order (sizes differ by at most one), Gonzalez(k) runs on every block
 * (first center: the block's smallest index) and S becomes the ascending
 * union of their centers.  Then Gonzalez(k) on S (first center: S[0]), and
 * the covering radius over all points.  The FP32 points are used in either
 * precision.  SYNCHRONISES the stream once per pass (to size the next one).
 *   k          centers, 1 <= k < 2^24.
 *   capacity   c >= 1; a pass that does not shrink S (k too close to c)
 *              returns KC_ENOCONV.
 *   centers    device int64 [k] (-1 padded), n_centers device int64 [1].
 *   radius     device double [1]: exact FP64 covering radius over all points.
 *   rounds     HOST int32 [1] or NULL: passes of the loop plus the last round.
 */
int kcenter_mrg_rounds(kc_handle* h, const kc_points* pts, int64_t k, int64_t capacity,
                       int64_t* centers, int64_t* n_centers, double* radius, int32_t* rounds,
                       void* stream);

/*
 * kcenter_assign -- nearest-center assignment and covering radius (the
 * k-center objective of Section 1.1: each point is served by its nearest
 * center; the solution value is the largest such distance).  Distances run
 * as |x|^2 + |c|^2 - 2 x.c on MFMA (FP32, or BF16 when pts->prec is
 * KC_BF16_RESCORE); every point whose nearest center is not certified by the
 * a-priori error bound, and every point that may attain the maximum, is
 * rescored exactly in FP64.  With labels NULL, FP32 points and d <= 8 the
 * distances are instead the canonical FP32 ones (relative error at most
 * gamma_{d+2}), whose tighter bound leaves fewer points to rescore.
 *   centers  device int64 [k], point indices, 1 <= k < 2^24 (streamed
 *            through LDS in chunks, so k is limited only by that check).
 *   labels   device int32 [n] or NULL: position in centers of the nearest.
 *   radius   device double [1]: exact FP64 covering radius.
 */
int kcenter_assign(kc_handle* h, const kc_points* pts, const int64_t* centers,
                   int64_t k, int32_t* labels, double* radius, void* stream);

/* EIM parameters (Algorithm 2 and Select, Algorithm 3, with phi). */
typedef struct {
    double eps;          /* 0 < eps < 1                                     */
    double phi;          /* phi > 0; the original algorithm has phi = 8      */
    uint64_t seed;       /* Philox4x64-10 key word 0                          */
    int32_t max_iters;   /* >= 1; KC_ENOCONV if R is still large after it    */
} kc_eim_params;

/* Per-iteration record of kcenter_eim. */
typedef struct {
    int64_t r_size;      /* |R| at the start of the iteration                 */
    int64_t ds_size;     /* points drawn into S in this iteration             */
    int64_t h_size;      /* |H|                                               */
    int64_t s_size;      /* |S| after the draw                                */
    double tau;          /* squared threshold d(v,S)^2 (-inf if H is empty)   */
    double p_s, p_h;     /* sampling probabilities                            */
} kc_eim_iter;

/*
 * kcenter_eim -- EIM-MapReduce-Sample (Algorithm 2) with Select (Algorithm
 * 3, parameter phi) and the termination changes of Section 4.1, then
 * Gonzalez on the sample C = S u R (the extra round) and the covering radius
 * over all points.  With L = ln n: while |R| > (4/eps) k n^eps L, every
 * x in R joins S with probability min(1, 9 k n^eps L / |R|) and H with
 * probability min(1, 4 n^eps L / |R|) (independent Philox4x64-10 draws:
 * key (seed, 0), counter (x, iteration, 0, 0), words 0 and 1, top 53 bits);
 * tau is the min(ceil(phi L), |H|)-th largest d(h,S)^2 over H; R keeps x iff
 * x is not in S and d(x,S)^2 > tau.  Distances of R to the new samples run on
 * MFMA; every keep/remove decision the error bound cannot certify is made in
 * FP64.  SYNCHRONISES the stream once per iteration (to size the next one).
 *   centers    device int64 [k]; n_centers device int64 [1]; radius device
 *              double [1].
 *   sample     device int64 [n] or NULL: C ascending; n_sample HOST int64.
 *   iters      HOST kc_eim_iter [max_iters] or NULL; n_iters HOST int32.
 */
int kcenter_eim(kc_handle* h, const kc_points* pts, int64_t k, const kc_eim_params* prm,
                int64_t* centers, int64_t* n_centers, double* radius, int64_t* sample,
                int64_t* n_sample, kc_eim_iter* iters, int32_t* n_iters, void* stream);

/*
 * kcenter_gonzalez_noalloc -- kcenter_gonzalez for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and kernels as
 * kcenter_gonzalez with FP32 points; it calls no hipMalloc, hipFree or
 * allocating library routine and uploads no host table.  Its workspace is
 * one 32 MiB device array per GPU, held until the process ends: the points'
 * min-distances (4 B per point, padded to 64), radius candidates (8 B per
 * point), per center 8 + 4d B plus, when the points stream instead of
 * fitting the register-resident grid, 2 KiB per center and a 4d-byte SoA
 * copy per point (also taken when the rows' layout does not suit the
 * resident kernel's vector loads).  A request that needs more returns
 * KC_EINVAL (stating the size) before any work; BF16 points return
 * KC_EUNSUPPORTED.  Every call on a GPU uses that GPU's array: calls that
 * overlap on one GPU (on other streams or handles) race.
 */
int kcenter_gonzalez_noalloc(kc_handle* h, const kc_points* pts, int64_t k, int64_t first,
                             int64_t* centers, double* radius_trace, int64_t* n_chosen,
                             void* stream);

typedef enum { KC_ALGO_GON = 0, KC_ALGO_MRG = 1, KC_ALGO_EIM = 2 } kc_algo;

/* One independent problem of a batch. */
typedef struct {
    kc_points pts;
    int32_t algo;              /* kc_algo                                      */
    int64_t k;
    int64_t first;             /* GON only                                     */
    const int64_t* offsets;    /* MRG only: HOST [m+1]                         */
    int32_t m;                 /* MRG only                                     */
    kc_eim_params eim;         /* EIM only                                     */
    int64_t* centers;          /* device int64 [k]                             */
    int64_t* n_centers;        /* device int64 [1]                             */
    double* radius;            /* device double [1]: exact covering radius     */
} kc_problem;

/*
 * kcenter_batch -- solve `count` independent problems of mixed n, d, k and
 * algorithm.  Gonzalez problems and MRG first rounds of equal d share the
 * same launches (register-resident, several per cooperative launch, when
 * every one fits a co-resident grid, else one streamed tile list over all of
 * them with a HIP graph per plan; a streamed list of n points with
 * n (2d - 4) >= 1e8 streams a BF16 copy the library rounds from the FP32
 * rows, with exact FP32 rescoring, which gives the FP32 stream's centers);
 * MRG second rounds likewise.  An EIM
 * problem whose n does not exceed Algorithm 2's threshold (4/eps) k n^eps
 * ln n never samples, so its result is Gonzalez's from point 0 with the
 * covering radius, and it joins those launches as such.  The other EIM
 * problems run their sampling loops in lockstep: each phase of an iteration
 * (draws and splits -- three launches shared by all of them; Select,
 * distance pass and decisions; FP32 refinement; FP64 decisions, then R's
 * compaction -- again three shared launches) is queued for every one of
 * them before one wait, whose readback sizes the next phase.  Then, per d,
 * the final Gonzalez of all of them runs as the segments of one run on
 * their samples C, and each covering radius by the assignment.  Gonzalez
 * and MRG problems in BF16 run one after another through their
 * single-problem entry points.  Outputs as for the single-problem calls.
 */
int kcenter_batch(kc_handle* h, const kc_problem* probs, int32_t count, void* stream);

/*
 * A batch planned once and run many times (the same problems; the points'
 * values may change between runs, their arrays, sizes and the other fields
 * may not).
 *
 * kcenter_batch_plan -- check the problems as kcenter_batch does, copy them
 * (MRG offsets included) and decide their grouping.  The plan owns a private
 * workspace on the handle's device: its tables, buffers and captured graphs
 * are never reallocated or evicted by other calls.  No GPU work; *plan is
 * NULL on error.  KC_EINVAL / KC_ENOMEM / KC_EHIP.
 *
 * kcenter_batch_run -- run the plan on `stream`: the first run builds and
 * uploads every group's launch plan and captures the graphs of the streamed
 * steps and of the finishing passes; later runs only launch (cached graphs;
 * the register-resident engine's cooperative launches are issued directly,
 * since a graph carries no co-residency guarantee).  EIM problems run as in
 * kcenter_batch (lockstep loops, one wait per phase) and BF16 Gonzalez and
 * MRG problems through their single-problem paths, on the plan's
 * workspace.  The plan's
 * device status is folded into `h`'s (see kc_device_status).  Outputs, as
 * for kcenter_batch, land in the arrays the problems name.  Runs of one plan
 * must not overlap.
 *
 * kcenter_batch_free -- synchronise the device and release the plan (NULL:
 * no-op).
 */
typedef struct kc_batch_plan kc_batch_plan;
int kcenter_batch_plan(kc_handle* h, const kc_problem* probs, int32_t count,
                       kc_batch_plan** plan);
int kcenter_batch_run(kc_handle* h, kc_batch_plan* plan, void* stream);
void kcenter_batch_free(kc_batch_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* KCENTER_H */
