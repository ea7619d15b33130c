// kc_resume.hip -- Gonzalez's traversal resumed from a saved prefix of
// centers (checkpoint / resume).  Section 3.1's traversal picks each center
// from the current center set alone, so forcing the first p centers and then
// continuing gives, for a prefix of an earlier run, exactly the longer run.
//
//   apply   every point's canonical FP32 min-distance to prefix centers
//           0..p-2 (one lane per point, the centers through LDS);
//   engine  the register-resident or streaming engine runs steps p-1..k-1
//           with first center prefix[p-1], starting from those
//           min-distances (the min over centers is exact, so the values
//           equal the uninterrupted run's bit for bit);
//   keys    the keys of the forced steps 0..p-2: prefix[t+1] with its
//           canonical FP32 distance to prefix centers 0..t;
//   finish  the usual centers, FP64 trace and exact radius.
#include <algorithm>
#include <vector>

#include "kc_host.h"

#define KC_RS_LDS 8192   // floats of prefix coordinates per LDS chunk

// mind[i] = min over prefix centers 0..np-1 of D32(x_i, c) (+inf if np = 0).
template <int D>
__global__ __launch_bounds__(256) void k_prefix_apply(const float* __restrict__ X, int64_t ld,
                                                     int d_rt, uint32_t n,
                                                     const int64_t* __restrict__ prefix,
                                                     uint32_t np, float* __restrict__ mind)
{
    const int d = D > 0 ? D : d_rt;
    __shared__ float sC[KC_RS_LDS];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    const float* xi = X + (uint64_t)(live ? i : 0) * (uint64_t)ld;
    float xr[D > 0 ? D : 1];
    if constexpr (D > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) xr[j] = xi[j];
    }
    float m = __builtin_inff();
    const uint32_t per = KC_RS_LDS / (uint32_t)d;   // centers per chunk
    for (uint32_t c0 = 0; c0 < np; c0 += per) {
        const uint32_t cn = min(per, np - c0);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < cn * (uint32_t)d; e += blockDim.x) {
            const uint32_t c = e / (uint32_t)d, j = e - c * (uint32_t)d;
            sC[e] = X[(uint64_t)prefix[c0 + c] * (uint64_t)ld + j];
        }
        __syncthreads();
        if (live) {
            for (uint32_t c = 0; c < cn; ++c) {
                const float* cc = sC + c * (uint32_t)d;
                float s = 0.f;
                if constexpr (D > 0) {
                    s = kc_d32_dist<D>(xr, cc);
                } else {
                    for (int j = 0; j < d; ++j) s = kc_d32_step(s, xi[j], cc[j]);
                }
                m = kc_fmin_nn(m, s);
            }
        }
    }
    if (live) mind[i] = m;
}

// keys[t], t < p-1: block t packs prefix[t+1] with its canonical FP32 squared
// distance to prefix centers 0..t.  A forced center is kept whatever that
// distance: a zero distance is recorded as the smallest positive value, since
// a zero key marks the end of the traversal.
__global__ __launch_bounds__(256) void k_prefix_keys(const float* __restrict__ X, int64_t ld,
                                                    int d, const int64_t* __restrict__ prefix,
                                                    uint32_t p, u64* __restrict__ keys)
{
    __shared__ float sP[KC_MAXD];
    __shared__ uint32_t sMin;
    const uint32_t t = blockIdx.x;
    if (t + 1 >= p) return;
    const uint64_t g = (uint64_t)prefix[t + 1];
    for (int j = threadIdx.x; j < d; j += blockDim.x) sP[j] = X[g * (uint64_t)ld + j];
    if (threadIdx.x == 0) sMin = 0x7F800000u;
    __syncthreads();
    float m = __builtin_inff();
    for (uint32_t c = threadIdx.x; c <= t; c += blockDim.x) {
        const float* cc = X + (uint64_t)prefix[c] * (uint64_t)ld;
        float s = 0.f;
        for (int j = 0; j < d; ++j) s = kc_d32_step(s, sP[j], cc[j]);
        m = kc_fmin_nn(m, s);
    }
    atomicMin(&sMin, __float_as_uint(m));
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t v = sMin > 0u ? sMin : 1u;
        keys[t] = ((u64)v << 32) | (u64)(0xFFFFFFFFu - (uint32_t)g);
    }
}

#define KC_PA_CASE(DD)                                                                    \
    case DD:                                                                              \
        hipLaunchKernelGGL(k_prefix_apply<DD>, grid, dim3(256), 0, s, X, ld, d, n, prefix, \
                           np, mind);                                                     \
        break;

static void kc_prefix_apply(const float* X, int64_t ld, int d, uint32_t n,
                            const int64_t* prefix, uint32_t np, float* mind, hipStream_t s)
{
    const dim3 grid((n + 255) / 256);
    switch (d) {
        KC_PA_CASE(2)
        KC_PA_CASE(3)
        KC_PA_CASE(8)
        KC_PA_CASE(10)
        KC_PA_CASE(16)
        KC_PA_CASE(32)
        KC_PA_CASE(41)
    default:
        hipLaunchKernelGGL(k_prefix_apply<0>, grid, dim3(256), 0, s, X, ld, d, n, prefix, np,
                           mind);
    }
}

extern "C" int kcenter_gonzalez_resume(kc_handle* h, const kc_points* pts,
                                       const int64_t* prefix, int64_t p, int64_t k,
                                       int64_t* centers, double* radius_trace,
                                       int64_t* n_chosen, void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, false);
    if (rc) return rc;
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k=%lld out of range", (long long)k);
    if (!prefix || p < 1 || p > k)
        return h->fail(KC_EINVAL, "prefix: need 1 <= p <= k (p=%lld, k=%lld)", (long long)p,
                       (long long)k);
    if (!centers || !n_chosen) return h->fail(KC_EINVAL, "centers/n_chosen NULL");
    {
        std::vector<int64_t> srt(prefix, prefix + p);
        for (int64_t t = 0; t < p; ++t)
            if (srt[t] < 0 || srt[t] >= pts->n)
                return h->fail(KC_EINVAL, "prefix[%lld]=%lld out of range", (long long)t,
                               (long long)srt[t]);
        std::sort(srt.begin(), srt.end());
        for (int64_t t = 1; t < p; ++t)
            if (srt[t] == srt[t - 1])
                return h->fail(KC_EINVAL, "prefix repeats point %lld", (long long)srt[t]);
    }
    hipStream_t s = (hipStream_t)stream;
    kc_validate_points(h, pts, s);
    const int d = pts->d;
    const uint32_t n = (uint32_t)pts->n, kk = (uint32_t)k, pp = (uint32_t)p;
    const uint32_t ks = kk - pp + 1;   // engine steps: p-1 .. k-1

    // the finishing plan: the whole traversal, first center prefix[0]
    std::vector<KcGonJob> jobs(1);
    jobs[0] = KcGonJob{pts->f32, pts->ld, 0, n, (uint32_t)prefix[0], kk};
    KcGonRun R;
    KcGonHost H;
    rc = kc_plan_gon(h, "r.", d, 1024, jobs, R, H, s);
    if (rc) return rc;
    R.xa = pts->f32;
    R.lda = pts->ld;
    const int64_t* pre_d = (const int64_t*)h->upload("r.prefix", prefix, 8ull * p, s);
    if (!pre_d) return h->fail(KC_ENOMEM, "workspace allocation failed");

    // the engine's plan: steps p-1.. from prefix[p-1], keys from p-1
    KcSeg es = H.segs[0];
    es.first = (uint32_t)prefix[p - 1];
    es.ksteps = ks;
    es.keyoff = pp - 1;
    const KcSeg* esd = (const KcSeg*)h->upload("r.esegs", &es, sizeof es, s);
    if (!esd) return h->fail(KC_ENOMEM, "workspace allocation failed");

    kc_prefix_apply(pts->f32, pts->ld, d, n, pre_d, pp - 1, R.mind, s);
    bool done = false;
    if (h->allow_resident) {
        int v = 0;
        uint32_t G = 0;
        if (h->resident_fit(d, n, &v, &G)) {
            const uint64_t bw = kc_resident_slot_words(ks, G);
            u64* bar = (u64*)h->ws("r.bar", sizeof(u64) * (bw + 8));
            if (!bar) return h->fail(KC_ENOMEM, "workspace allocation failed");
            const int rows = kc_resident_rows_ok(d, pts->f32, pts->ld, n);
            if (!rows)
                kc_stage_soa(pts->f32, pts->ld, d, 0, n, (float*)R.xs, R.stride, 0, s);
            kc_fill_u64(bar, 0ull, bw + 1, s);
            hipEvent_t ev = h->span_begin(s);
            hipError_t e = kc_gon_resident(d, v, G, R.xs, R.stride, 0, n, nullptr,
                                           (uint32_t)prefix[p - 1], (int)ks, R.mind,
                                           R.keys + (pp - 1), bar, (uint32_t*)(bar + bw),
                                           h->spin_limit, pts->f32, pts->ld, rows,
                                           h->status_word, nullptr, nullptr, s, R.mind);
            h->span_end("gon_resident", ev, 1, s);
            if (e == hipSuccess) done = true;
            else (void)hipGetLastError();   // not co-resident: stream instead
        }
    }
    if (!done) {
        kc_enqueue_stage(R, H, jobs, s);
        kc_fill_u64(R.part, 0ull, R.keysum * KC_PARTS * KC_PSTRIDE, s);
        hipEvent_t ev = h->span_begin(s);
        for (uint32_t t = 0; t < ks; ++t)
            kc_gon_step(R.xs, R.stride, d, R.mind, R.part, esd, R.blk_seg, R.blk_start, R.nblk,
                        (int)t, s);
        kc_part_collect(R.part + (uint64_t)(pp - 1) * KC_PARTS * KC_PSTRIDE, R.keys + (pp - 1),
                        ks, s);
        h->span_end("gon_step", ev, ks, s);
    }
    if (pp > 1)
        hipLaunchKernelGGL(k_prefix_keys, dim3(pp - 1), dim3(256), 0, s, pts->f32, pts->ld, d,
                           pre_d, pp, R.keys);
    kc_gon_finish(R, centers, n_chosen, radius_trace, nullptr, nullptr, nullptr, s);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}
