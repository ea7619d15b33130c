// kc_noalloc.hip -- Gonzalez's traversal for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc): the same kernels as kcenter_gonzalez, with every buffer
// carved from one file-scope device array instead of the handle's workspace.
//
// The array, `scratch`, is KC_NOALLOC_BYTES per GPU and lives as long as the
// process.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): kc_noalloc_setup looks up its
// device address once per device with hipGetSymbolAddress, with that device
// current, and every launch takes that address.  All calls on one GPU share
// the array, so calls that overlap on one GPU race; each call rewrites every
// word it later reads (plan tables, exchange words, min-distances, keys,
// accumulators) before reading it.
#include <mutex>

#include "kc_host.h"

#define KC_NOALLOC_BYTES (32ull << 20)
#define KC_NOALLOC_DEVICES 64

static __device__ __align__(256) unsigned char scratch[KC_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[KC_NOALLOC_DEVICES];
static bool g_scratch_done[KC_NOALLOC_DEVICES];

// The device address of `scratch` on `device` (which must be current), looked
// up on the first call for that device.  Returns hipSuccess and sets *out, or
// the lookup's error (then *out is NULL).
hipError_t kc_noalloc_setup(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= KC_NOALLOC_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        g_scratch_ptr[device] = p;
        g_scratch_done[device] = true;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// The one-segment plan tables of a run, written on the device (no host
// upload): segment 0 covers points [0, n), first center `first`, k steps;
// tile b starts at b * tile; step pair t is (0, t).
__global__ void k_plan_one(KcSeg* __restrict__ segs, uint32_t* __restrict__ blk_seg,
                           uint32_t* __restrict__ blk_start, uint32_t nblk,
                           uint32_t* __restrict__ pairs_seg, uint32_t* __restrict__ pairs_t,
                           uint32_t k, uint32_t n, uint32_t first, uint32_t tile)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        KcSeg sg;
        sg.src = 0;
        sg.base = 0;
        sg.len = n;
        sg.first = first;
        sg.ksteps = k;
        sg.keyoff = 0;
        segs[0] = sg;
    }
    if (i < nblk) {
        blk_seg[i] = 0;
        blk_start[i] = i * tile;
    }
    if (i < k) {
        pairs_seg[i] = 0;
        pairs_t[i] = i;
    }
}

namespace {

// Bump allocation from the scratch array, 256-byte aligned.
struct Carve {
    char* base;
    uint64_t used = 0;
    explicit Carve(void* p) : base((char*)p) {}
    void* take(uint64_t bytes)
    {
        void* p = base + used;
        used += (bytes + 255) & ~255ull;
        return p;
    }
};

}  // namespace

extern "C" int kcenter_gonzalez_noalloc(kc_handle* h, const kc_points* pts, int64_t k,
                                        int64_t first, int64_t* centers, double* radius_trace,
                                        int64_t* n_chosen, void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, false);
    if (rc) return rc;
    if (pts->prec != KC_FP32)
        return h->fail(KC_EUNSUPPORTED, "no-allocation Gonzalez takes FP32 points only");
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k=%lld out of range", (long long)k);
    if (first < 0 || first >= pts->n) return h->fail(KC_EINVAL, "first out of range");
    if (!centers || !n_chosen) return h->fail(KC_EINVAL, "centers/n_chosen NULL");
    if (!h->scratch)
        return h->fail(KC_EHIP, "the device address of the scratch array is unknown");
    hipStream_t s = (hipStream_t)stream;
    const int d = pts->d;
    const uint32_t n = (uint32_t)pts->n, kk = (uint32_t)k;
    const uint32_t tile = 1024;
    const uint32_t nblk = (n + tile - 1) / tile;
    const uint64_t stride = std::max<uint64_t>(kc_pad64(n), 64);

    // engine: register-resident when the points fit a co-resident grid
    int v = 0;
    uint32_t G = 0;
    const bool resident = h->allow_resident && h->resident_fit(d, n, &v, &G);
    const int rows = resident && kc_resident_rows_ok(d, pts->f32, pts->ld, n);
    const bool need_xs = !resident || !rows;
    const uint64_t bw = kc_resident_slot_words(kk, G) + 8;

    // every buffer's size, checked against the array before anything runs
    const uint64_t sz_segs = sizeof(KcSeg), sz_tab = 4ull * nblk, sz_pairs = 4ull * kk;
    const uint64_t sz_keys = 8ull * kk, sz_cc = 4ull * kk * (uint64_t)d;
    const uint64_t sz_mind = 4ull * stride, sz_cand = 8ull * n;
    const uint64_t sz_part = resident ? 0 : 8ull * KC_PARTS * KC_PSTRIDE * kk;
    const uint64_t sz_bar = resident ? 8ull * bw : 0;
    const uint64_t sz_xs = need_xs ? 4ull * (uint64_t)d * stride : 0;
    uint64_t need = 0;
    for (uint64_t b : {sz_segs, sz_tab, sz_tab, sz_pairs, sz_pairs, sz_keys, sz_cc,
                       (uint64_t)16, (uint64_t)16, sz_mind, sz_cand, sz_part, sz_bar, sz_xs})
        need += (b + 255) & ~255ull;
    if (need > KC_NOALLOC_BYTES)
        return h->fail(KC_EINVAL,
                       "no-allocation Gonzalez needs %llu bytes of scratch for n=%u d=%d k=%u; "
                       "the limit is %llu",
                       (unsigned long long)need, n, d, kk, (unsigned long long)KC_NOALLOC_BYTES);

    Carve C(h->scratch);
    KcGonRun R;
    R.d = d;
    R.nseg = 1;
    R.kmax = kk;
    R.stride = stride;
    R.nblk = nblk;
    R.tile = tile;
    R.npairs = kk;
    R.keysum = kk;
    R.band = 2.0 * kc_gamma32(d) + 4.0 * 5.9604644775390625e-8;
    R.cand_cap = n;
    R.segs = (KcSeg*)C.take(sz_segs);
    R.blk_seg = (uint32_t*)C.take(sz_tab);
    R.blk_start = (uint32_t*)C.take(sz_tab);
    R.pairs_seg = (uint32_t*)C.take(sz_pairs);
    R.pairs_t = (uint32_t*)C.take(sz_pairs);
    R.keys = (u64*)C.take(sz_keys);
    R.ccoord = (float*)C.take(sz_cc);
    R.radius2 = (double*)C.take(16);
    R.ncand = (uint32_t*)C.take(16);
    R.ticket = R.ncand + 1;
    R.mind = (float*)C.take(sz_mind);
    R.cand = (u64*)C.take(sz_cand);
    R.part = sz_part ? (u64*)C.take(sz_part) : nullptr;
    u64* bar = sz_bar ? (u64*)C.take(sz_bar) : nullptr;
    R.xs = sz_xs ? (float*)C.take(sz_xs) : nullptr;
    R.xa = pts->f32;   // center and candidate gathers read the caller's rows
    R.lda = pts->ld;

    kc_validate_points(h, pts, s);
    const uint32_t ng = std::max<uint32_t>(std::max(nblk, kk), 1);
    hipLaunchKernelGGL(k_plan_one, dim3((ng + 255) / 256), dim3(256), 0, s, R.segs, R.blk_seg,
                       R.blk_start, nblk, R.pairs_seg, R.pairs_t, kk, n, (uint32_t)first, tile);
    if (resident) {
        if (!rows)
            kc_stage_soa(pts->f32, pts->ld, d, 0, n, (float*)R.xs, R.stride, 0, s);
        kc_fill_u64(bar, 0ull, bw, s);   // exchange words and the abort flag
        uint32_t* abort_flag = (uint32_t*)(bar + (bw - 8));
        hipEvent_t ev = h->span_begin(s);
        hipError_t e = kc_gon_resident(d, v, G, R.xs, R.stride, 0, n, nullptr, (uint32_t)first,
                                       (int)kk, R.mind, R.keys, bar, abort_flag, h->spin_limit,
                                       pts->f32, pts->ld, rows, h->status_word, nullptr, nullptr,
                                       s);
        h->span_end("gon_resident", ev, 1, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return h->fail(KC_EHIP, "resident launch: %s", hipGetErrorString(e));
        }
    } else {
        kc_stage_soa(pts->f32, pts->ld, d, 0, n, (float*)R.xs, R.stride, 0, s);
        kc_fill_u32((uint32_t*)R.mind, 0x7F800000u, R.stride, s);   // +inf
        kc_fill_u64(R.part, 0ull, (uint64_t)kk * KC_PARTS * KC_PSTRIDE, s);
        hipEvent_t ev = h->span_begin(s);
        kc_enqueue_gon_steps(R, s);
        h->span_end("gon_step", ev, kk, s);
    }
    kc_gon_finish(R, centers, n_chosen, radius_trace, nullptr, nullptr, nullptr, s);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}
