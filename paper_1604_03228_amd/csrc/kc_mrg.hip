// kc_mrg.hip -- two-round MRG (Algorithm 1, one pass of its loop), the BF16
// Gonzalez entry, and the assignment entry point.
//
// MRG on the device, without host synchronisation:
//   round 1   all m partitions are segments of one batched Gonzalez run:
//             register-resident, several partitions per cooperative
//             launch, when every partition fits a co-resident grid (in
//             either precision), else streamed (FP32, or BF16 + exact FP32
//             rescoring);
//   union     k_mrg_union sorts each partition's centers (global indices)
//             by rank and concatenates them in partition order, which is
//             ascending global order because partitions are contiguous row
//             ranges; it also writes the union size into round 2's segment
//             table, so round 2's kernels see the true length;
//   round 2   Gonzalez on the gathered union (register-resident when it
//             fits, else streamed), first center = smallest index;
//   radius    the MFMA assignment of every point to the final centers.
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "kc_host.h"

// One block per partition p: its n_p centers (distinct global indices),
// ranked by value, land at uni[off_p + rank], off_p = sum_{q<p} n_q.
__global__ void k_mrg_union(const int64_t* __restrict__ cent, const int64_t* __restrict__ nch,
                            int m, int k, int64_t* __restrict__ uni,
                            int64_t* __restrict__ n_union, uint32_t* __restrict__ seg_len)
{
    const int p = blockIdx.x;
    __shared__ int64_t off;
    if (threadIdx.x == 0) {
        int64_t o = 0;
        for (int q = 0; q < p; ++q) o += nch[q];
        off = o;
        if (p == m - 1) {
            const int64_t tot = o + nch[p];
            *n_union = tot;
            *seg_len = (uint32_t)tot;
        }
    }
    __syncthreads();
    const int64_t np = nch[p];
    const int64_t* c = cent + (int64_t)p * k;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
        const int64_t v = c[i];
        int64_t r = 0;
        for (int64_t j = 0; j < np; ++j) r += c[j] < v;
        uni[off + r] = v;
    }
}

// Row-major copy of the listed rows: Y[i][*] = X[idx[i]][*] (d columns).
__global__ void k_gather_rows64(const float* __restrict__ X, int64_t ld, int d,
                                const int64_t* __restrict__ idx, uint64_t n,
                                float* __restrict__ Y)
{
    const uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (q >= n * (uint64_t)d) return;
    const uint64_t i = q / (uint64_t)d, j = q - i * (uint64_t)d;
    Y[q] = X[(uint64_t)idx[i] * (uint64_t)ld + j];
}

// SoA copy of the listed rows: column i <- row uni[i] (padding repeats uni[0]).
__global__ void k_gather_soa(const float* __restrict__ X, int64_t ld, int d,
                             const int64_t* __restrict__ uni, const int64_t* __restrict__ nu,
                             uint32_t padded, float* __restrict__ xs, uint64_t stride)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    const int64_t cnt = *nu;
    const uint64_t r = (uint64_t)((int64_t)i < cnt ? uni[i] : uni[0]);
    for (int j = 0; j < d; ++j) xs[(uint64_t)j * stride + i] = X[r * ld + j];
}

static std::string kc_key(const char* tag, std::initializer_list<const void*> ptrs,
                          std::initializer_list<long long> vals)
{
    std::string s(tag);
    char b[40];
    for (const void* p : ptrs) {
        snprintf(b, sizeof b, ":%p", p);
        s += b;
    }
    for (long long v : vals) {
        snprintf(b, sizeof b, ":%lld", v);
        s += b;
    }
    return s;
}

// ---------------------------------------------------------------------------
// BF16 engine buffers for a planned run

int kc_bf16_alloc(kc_handle* h, const std::string& pre, const KcGonRun& R, KcBf16Run& B)
{
    B.xb = (uint16_t*)h->ws(pre + "xb", sizeof(uint16_t) * (size_t)R.d * R.stride);
    B.ex = (float*)h->ws(pre + "ex", sizeof(float) * R.stride);
    B.lpart = (uint32_t*)h->ws(pre + "lpart", sizeof(uint32_t) * KC_PARTS * 32 *
                                                  std::max<uint64_t>(R.keysum, 1));
    // region r of the list takes the tiles b with b mod KC_PARTS == r
    B.region = ((R.nblk + KC_PARTS - 1) / KC_PARTS) * KC_BF_TILE_PTS;
    const size_t ents = (size_t)KC_PARTS * std::max<uint32_t>(B.region, 1);
    B.list = (u64*)h->ws(pre + "list", sizeof(u64) * ents);
    B.list_hi = (float*)h->ws(pre + "listhi", sizeof(float) * ents);
    B.exm = (float*)h->ws(pre + "exm", sizeof(float) * R.stride);
    B.exupto = (uint32_t*)h->ws(pre + "exupto", sizeof(uint32_t) * R.stride);
    B.listcnt = (uint32_t*)h->ws(pre + "listcnt", sizeof(uint32_t) * KC_PARTS * 32 *
                                                      std::max<uint32_t>(R.kmax, 1));
    B.nresc = (uint32_t*)h->ws(pre + "nresc", sizeof(uint32_t) * std::max<uint32_t>(R.kmax, 1));
    B.Lt = (float*)h->ws(pre + "lt", sizeof(float) * std::max<int>(R.nseg, 1));
    if (!B.xb || !B.ex || !B.lpart || !B.list || !B.list_hi || !B.exm || !B.exupto ||
        !B.listcnt || !B.nresc || !B.Lt)
        return h->fail(KC_ENOMEM, "workspace allocation failed");
    h->last_bf16_listcnt = B.listcnt;
    h->last_bf16_nresc = B.nresc;
    h->last_bf16_kmax = R.kmax;
    const double u = 5.9604644775390625e-8;
    B.g = (float)((kc_gamma32(R.d) + 16.0 * u) * (1.0 + 1e-6));
    // about one listed point per rescoring wave: a wave rescores its kept
    // points one after another, each a chain of dependent loads
    B.rescore_blocks = std::min<uint32_t>(2048, std::max<uint32_t>(256, R.nblk / 2));
    return KC_OK;
}

// prep / steps (timed under `span`) / finish graphs of a BF16 run
int kc_run_bf16(kc_handle* h, const std::string& key0, const KcGonRun& R, const KcBf16Run& B,
                const KcGonHost& H, const std::vector<KcGonJob>& jobs, const char* span,
                hipStream_t s, const std::function<void(hipStream_t)>& finish)
{
    const std::string key = key0 + kc_hash_str(R.plan_hash);
    int rc = h->run_graph(key + ":prep", s,
                          [&](hipStream_t st) { kc_enqueue_bf16_prep(R, B, H, jobs, st); });
    if (rc) return rc;
    hipEvent_t ev = h->span_begin(s);
    rc = h->run_graph(key + ":steps", s, [&](hipStream_t st) { kc_enqueue_bf16_steps(R, B, st); });
    h->span_end(span, ev, 3 * (int64_t)R.kmax, s);
    if (rc) return rc;
    return h->run_graph(key + ":finish", s, finish);
}

int kc_gonzalez_bf16(kc_handle* h, const kc_points* pts, int64_t k, int64_t first,
                     int64_t* centers, double* radius_trace, int64_t* n_chosen, hipStream_t s)
{
    std::vector<KcGonJob> jobs(1);
    jobs[0].X = pts->f32;
    jobs[0].Xb = pts->bf16;
    jobs[0].ld = pts->ld;
    jobs[0].row0 = 0;
    jobs[0].len = (uint32_t)pts->n;
    jobs[0].first = (uint32_t)first;
    jobs[0].k = (uint32_t)k;
    KcGonRun R;
    KcGonHost H;
    int rc = kc_plan_gon(h, "g.", pts->d, KC_BF_TILE_PTS, jobs, R, H, s);
    if (rc) return rc;
    KcBf16Run B;
    rc = kc_bf16_alloc(h, "gb.", R, B);
    if (rc) return rc;
    const std::string key = kc_key("gonbf", {pts->f32, pts->bf16, centers, radius_trace, n_chosen},
                                   {pts->n, pts->d, pts->ld, k, first});
    return kc_run_bf16(h, key, R, B, H, jobs, "gon_bf16", s, [&](hipStream_t st) {
        kc_bf16_finish(R, B, centers, n_chosen, radius_trace, nullptr, nullptr, st);
    });
}

// ---------------------------------------------------------------------------
// assignment

int kc_assign_run(kc_handle* h, const kc_points* pts, const int64_t* centers, uint32_t k,
                  const int64_t* k_dev, int32_t* labels, double* radius, hipStream_t s,
                  const std::string& pre)
{
    const bool bf = pts->prec == KC_BF16_RESCORE;
    // FP32 inputs run the distance pass on split BF16 MFMAs (option
    // mfma_split) or on the FP32 MFMA; every staged row has the MFMA's K
    const bool split = !bf && h->mfma_split;
    const uint32_t n = (uint32_t)pts->n;
    const int d = pts->d;
    const uint32_t kpad = (k + 15u) & ~15u;
    const int dp = split ? kc_mindist_dpad_split(d, kpad) : kc_mindist_dpad(d, bf);
    const bool packed = split && kc_split_use_packed(d, kpad);
    KcCenters C;
    C.kpad = kpad;
    C.dp = dp;
    C.Cf = (float*)h->ws(pre + "cf", sizeof(float) * (size_t)kpad * dp);
    C.Cb = bf ? (uint16_t*)h->ws(pre + "cb", sizeof(uint16_t) * (size_t)kpad * dp) : nullptr;
    C.cn = (float*)h->ws(pre + "cn", sizeof(float) * kpad);
    C.cnl = (float*)h->ws(pre + "cnl", sizeof(float) * kpad);
    C.clen = (float*)h->ws(pre + "clen", sizeof(float) * kpad);
    C.cerr = bf ? (float*)h->ws(pre + "cerr", sizeof(float) * kpad) : nullptr;
    C.cmax = (float*)h->ws(pre + "cmax", 16);
    // FP32 passes measure from a local origin of the points (smaller norms,
    // tighter bounds); BF16 inputs are used as stored
    float* mu = bf ? nullptr : (float*)h->ws(pre + "mu", sizeof(float) * (size_t)d);
    C.mu = mu;
    // FP32 inputs: the translated copy for the FP32 MFMA, or its BF16 high
    // and low parts for the split MFMAs
    C.Ct = (bf || split) ? nullptr : (float*)h->ws(pre + "ct", sizeof(float) * (size_t)kpad * dp);
    if (split) {
        C.Cb = (uint16_t*)h->ws(pre + "cb", sizeof(uint16_t) * (size_t)kpad * dp);
        if (packed)
            C.pk = true;
        else
            C.Cbl = (uint16_t*)h->ws(pre + "cbl", sizeof(uint16_t) * (size_t)kpad * dp);
    }
    KcMinOut O;
    O.arg = (int32_t*)h->ws(pre + "arg", sizeof(int32_t) * n);
    O.m1 = (float*)h->ws(pre + "m1", sizeof(float) * n);
    O.lo2 = (float*)h->ws(pre + "lo2", sizeof(float) * n);
    O.lob = (float*)h->ws(pre + "lob", sizeof(float) * n);
    O.nx = (float*)h->ws(pre + "nx", sizeof(float) * n);
    float* hi = (float*)h->ws(pre + "hi", sizeof(float) * n);
    uint32_t* list = (uint32_t*)h->ws(pre + "list", sizeof(uint32_t) * 2 * (size_t)n);
    uint32_t* nlist = (uint32_t*)h->ws(pre + "nlist", 16);
    float* lo_max = (float*)h->ws(pre + "lomax", 16);
    double* r2 = (double*)h->ws(pre + "r2", 16);
    float* ex = bf ? (float*)h->ws(pre + "ex", sizeof(float) * n) : nullptr;
    if (!C.Cf || (bf && (!C.Cb || !C.cerr)) || (!bf && !mu) || (!bf && !split && !C.Ct) ||
        (split && (!C.Cb || (!packed && !C.Cbl))) || !C.cmax || !C.cn || !C.cnl ||
        !C.clen || !O.arg || !O.m1 ||
        !O.lo2 || !O.lob || !O.nx || !hi || !list || !nlist || !lo_max || !r2 || (bf && !ex))
        return h->fail(KC_ENOMEM, "workspace allocation failed");
    // BF16 inputs: the points their pass lists run again on their FP32 rows
    // (split BF16 MFMAs, or the FP32 MFMA) against the centers staged from
    // their FP32 rows, measured from a local origin; FP64 takes the rest
    KcAssignRefine R2;
    float* mu2 = nullptr;
    if (bf) {
        const bool sp2 = h->mfma_split;
        const int dp2 = sp2 ? kc_mindist_dpad_split(d, kpad) : kc_mindist_dpad(d, false);
        const bool pk2 = sp2 && kc_split_use_packed(d, kpad);
        KcCenters& C2 = R2.C;
        C2.kpad = kpad;
        C2.dp = dp2;
        C2.Cf = (float*)h->ws(pre + "2cf", sizeof(float) * (size_t)kpad * dp2);
        C2.cn = (float*)h->ws(pre + "2cn", sizeof(float) * kpad);
        C2.cnl = (float*)h->ws(pre + "2cnl", sizeof(float) * kpad);
        C2.clen = (float*)h->ws(pre + "2clen", sizeof(float) * kpad);
        C2.cmax = (float*)h->ws(pre + "2cmax", 16);
        mu2 = (float*)h->ws(pre + "mu", sizeof(float) * (size_t)d);
        C2.mu = mu2;
        if (sp2) {
            C2.Cb = (uint16_t*)h->ws(pre + "2cb", sizeof(uint16_t) * (size_t)kpad * dp2);
            if (pk2)
                C2.pk = true;
            else
                C2.Cbl = (uint16_t*)h->ws(pre + "2cbl", sizeof(uint16_t) * (size_t)kpad * dp2);
        } else {
            C2.Ct = (float*)h->ws(pre + "2ct", sizeof(float) * (size_t)kpad * dp2);
        }
        const size_t cap = 2 * (size_t)n;
        R2.O.arg = (int32_t*)h->ws(pre + "2arg", sizeof(int32_t) * cap);
        R2.O.m1 = (float*)h->ws(pre + "2m1", sizeof(float) * cap);
        R2.O.lo2 = (float*)h->ws(pre + "2lo2", sizeof(float) * cap);
        R2.O.lob = (float*)h->ws(pre + "2lob", sizeof(float) * cap);
        R2.O.nx = (float*)h->ws(pre + "2nx", sizeof(float) * cap);
        R2.hi = (float*)h->ws(pre + "2hi", sizeof(float) * cap);
        R2.list = (uint32_t*)h->ws(pre + "2list", sizeof(uint32_t) * 2 * cap);
        R2.nlist = (uint32_t*)h->ws(pre + "2nlist", 16);
        if (!C2.Cf || !C2.cn || !C2.cnl || !C2.clen || !C2.cmax || !C2.mu ||
            (sp2 && (!C2.Cb || (!pk2 && !C2.Cbl))) || (!sp2 && !C2.Ct) || !R2.O.arg ||
            !R2.O.m1 || !R2.O.lo2 || !R2.O.lob || !R2.O.nx || !R2.hi || !R2.list || !R2.nlist)
            return h->fail(KC_ENOMEM, "workspace allocation failed");
    }
    h->last_assign_nlist = bf ? R2.nlist : nlist;
    const std::string key =
        kc_key(("assign:" + pre).c_str(), {pts->f32, pts->bf16, centers, k_dev, labels, radius},
               {pts->n, d, pts->ld, k, bf, split, h->mfma_split});
    int rc = h->run_graph(key + ":stage", s, [&](hipStream_t st) {
        if (bf) kc_bf16_err(pts->f32, pts->bf16, pts->ld, d, n, ex, st);
        if (mu) kc_local_origin(pts->f32, pts->ld, d, n, mu, st);
        kc_stage_centers(pts->f32, bf ? pts->bf16 : nullptr, pts->ld, d, n, centers, nullptr, k,
                         k_dev, C, h->status_word, st);
        if (bf) {
            kc_local_origin(pts->f32, pts->ld, d, n, mu2, st);
            kc_stage_centers(pts->f32, nullptr, pts->ld, d, n, centers, nullptr, k, k_dev, R2.C,
                             h->status_word, st);
        }
    });
    if (rc) return rc;
    if (!labels && !bf && d <= 8) {
        // radius only at small d: canonical FP32 distances bound each
        // point's min-distance tightly, so few points need FP64
        hipEvent_t ev = h->span_begin(s);
        rc = h->run_graph(key + ":direct", s, [&](hipStream_t st) {
            kc_radius_direct(n, d, pts->f32, pts->ld, C.Cf, dp, k, k_dev, hi, list, nlist,
                             lo_max, r2, radius, st);
        });
        h->span_end("assign_direct", ev, 1, s);
        return rc;
    }
    // the MFMA pass with 4 or 8 waves per block and 64 or 32 KiB of staged
    // centers, a measured choice per shape
    const bool feas[4] = {true, true, true, true};
    char tkey[96];
    snprintf(tkey, sizeof tkey, "assign/%d/%d/%d/%d/%d", d, (int)floor(2.0 * log2((double)n + 1)),
             (int)floor(2.0 * log2((double)k + 1)), labels != nullptr, bf ? 1 : split ? 2 : 0);
    rc = h->tune(tkey, 4, feas, s, [&](int var) {
        hipEvent_t ev = h->span_begin(s);
        char vk[16];
        snprintf(vk, sizeof vk, ":mfma%d", var);
        const int r = h->run_graph(key + vk, s, [&](hipStream_t st) {
            kc_mindist(pts->f32, bf ? pts->bf16 : nullptr, ex, pts->ld, n, d, C, O,
                       labels != nullptr, st, (var & 1) ? 8 : 4, var >= 2 ? 32 : 64);
        });
        h->span_end("assign_mfma", ev, 1, s);
        return r;
    });
    if (rc) return rc;
    return h->run_graph(key + ":finish", s, [&](hipStream_t st) {
        kc_assign_finish(n, d, pts->f32, pts->ld, C, k, k_dev, O, ex, labels, hi, list, nlist,
                         lo_max, r2, radius, st, bf ? &R2 : nullptr);
    });
}

// ---------------------------------------------------------------------------
// public entry points

extern "C" {

int kcenter_assign(kc_handle* h, const kc_points* pts, const int64_t* centers, int64_t k,
                   int32_t* labels, double* radius, void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, true);
    if (rc) return rc;
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k=%lld out of range", (long long)k);
    if (!centers || !radius) return h->fail(KC_EINVAL, "centers/radius NULL");
    kc_validate_points(h, pts, (hipStream_t)stream);
    return kc_assign_run(h, pts, centers, (uint32_t)k, nullptr, labels, radius,
                         (hipStream_t)stream, "a.");
}

int kcenter_mrg(kc_handle* h, const kc_points* pts, const int64_t* offsets, int32_t m,
                int64_t k, int64_t* centers, int64_t* n_centers, double* radius,
                int64_t* round1, double* r1, int64_t* uni, int64_t* n_union, double* r2,
                void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, true);
    if (rc) return rc;
    if (m < 1) return h->fail(KC_EINVAL, "m=%d", m);
    if (!offsets) return h->fail(KC_EINVAL, "offsets NULL");
    if (offsets[0] != 0 || offsets[m] != pts->n)
        return h->fail(KC_EINVAL, "offsets must start at 0 and end at n");
    for (int p = 0; p < m; ++p)
        if (offsets[p + 1] < offsets[p]) return h->fail(KC_EINVAL, "offsets not monotone");
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k=%lld out of range", (long long)k);
    if ((int64_t)m * k >= (int64_t)0xFFFFFFFFll) return h->fail(KC_EINVAL, "m*k too large");
    if (!centers || !n_centers || !radius) return h->fail(KC_EINVAL, "outputs NULL");
    hipStream_t s = (hipStream_t)stream;
    kc_validate_points(h, pts, s);
    const bool bf = pts->prec == KC_BF16_RESCORE;
    const int d = pts->d;

    // ---- round 1: every partition is a segment of one run
    std::vector<KcGonJob> jobs(m);
    for (int p = 0; p < m; ++p) {
        jobs[p].X = pts->f32;
        jobs[p].Xb = pts->bf16;
        jobs[p].ld = pts->ld;
        jobs[p].row0 = (uint64_t)offsets[p];
        jobs[p].len = (uint32_t)(offsets[p + 1] - offsets[p]);
        jobs[p].first = 0;
        jobs[p].k = (uint32_t)k;
    }
    KcGonRun R1;
    KcGonHost H1;
    rc = kc_plan_gon(h, "m1.", d, 1024, jobs, R1, H1, s);
    if (rc) return rc;
    const int64_t* rb =
        (const int64_t*)h->upload("m1.rb", offsets, sizeof(int64_t) * (size_t)m, s);
    int64_t* cent1 = round1 ? round1 : (int64_t*)h->ws("m1.cent", sizeof(int64_t) * m * k);
    int64_t* nch1 = (int64_t*)h->ws("m1.nch", sizeof(int64_t) * m);
    double* rad1 = r1 ? r1 : (double*)h->ws("m1.rad", sizeof(double) * m);
    if (!rb || !cent1 || !nch1 || !rad1) return h->fail(KC_ENOMEM, "workspace allocation failed");
    const std::string key1 = kc_key("mrg1", {pts->f32, pts->bf16, cent1, rad1},
                                    {pts->n, d, pts->ld, k, m, bf});
    // All partitions on the resident engine, packed several per launch, when
    // each one's points fit a co-resident grid.  This holds in BF16 mode too
    // (from the full-precision copy): register-resident points are read from
    // HBM once, so there is no stream for BF16 to halve, and the sequences
    // are the FP32 path's by construction.  Otherwise the partitions stream,
    // in BF16 with exact rescoring or in FP32.
    // Round 1's finishing pass reads the caller's rows, so the resident
    // engine can load its points from them without a staging copy.
    R1.xa = pts->f32;
    R1.lda = pts->ld;
    bool done = false;
    if (h->allow_resident) {
        rc = kc_run_gon_resident_batch(h, key1, R1, H1, jobs, "mrg_round1", s, &done);
        if (rc) return rc;
    }
    if (done) {
        rc = h->run_graph(key1 + kc_hash_str(R1.plan_hash) + ":finish", s, [&](hipStream_t st) {
            kc_fill_u64((u64*)cent1, ~0ull, (uint64_t)m * k, st);
            kc_gon_finish(R1, cent1, nch1, nullptr, rad1, rb, nullptr, st);
        });
    } else if (bf) {
        KcGonRun Rb;
        KcGonHost Hb;
        rc = kc_plan_gon(h, "m1s.", d, KC_BF_TILE_PTS, jobs, Rb, Hb, s);
        if (rc) return rc;
        KcBf16Run B1;
        rc = kc_bf16_alloc(h, "m1b.", Rb, B1);
        if (rc) return rc;
        rc = kc_run_bf16(h, key1 + ":bf", Rb, B1, Hb, jobs, "mrg_round1", s, [&](hipStream_t st) {
            kc_fill_u64((u64*)cent1, ~0ull, (uint64_t)m * k, st);
            kc_bf16_finish(Rb, B1, cent1, nch1, nullptr, rad1, rb, st);
        });
    } else {
        rc = kc_run_gon_stream(h, key1, R1, H1, jobs, "mrg_round1", s, [&](hipStream_t st) {
            kc_fill_u64((u64*)cent1, ~0ull, (uint64_t)m * k, st);
            kc_gon_finish(R1, cent1, nch1, nullptr, rad1, rb, nullptr, st);
        });
    }
    if (rc) return rc;

    // ---- union and round 2
    const uint64_t cap = std::min<uint64_t>((uint64_t)m * k, (uint64_t)pts->n);
    std::vector<KcGonJob> jobs2(1);
    jobs2[0].X = nullptr;   // filled by the gather kernel
    jobs2[0].ld = pts->ld;
    jobs2[0].len = (uint32_t)cap;
    jobs2[0].first = 0;
    jobs2[0].k = (uint32_t)k;
    KcGonRun R2;
    KcGonHost H2;
    rc = kc_plan_gon(h, "m2.", d, 1024, jobs2, R2, H2, s);
    if (rc) return rc;
    int64_t* uni_b = uni ? uni : (int64_t*)h->ws("m2.uni", sizeof(int64_t) * cap);
    int64_t* nu = n_union ? n_union : (int64_t*)h->ws("m2.nu", 16);
    double* r2b = r2 ? r2 : (double*)h->ws("m2.r2", 16);
    if (!uni_b || !nu || !r2b) return h->fail(KC_ENOMEM, "workspace allocation failed");
    uint32_t* len_ptr = (uint32_t*)((char*)R2.segs + offsetof(KcSeg, len));
    const std::string key2 = kc_key("mrg2", {pts->f32, cent1, uni_b, nu, centers, n_centers, r2b},
                                    {pts->n, d, pts->ld, k, m}) +
                             kc_hash_str(R2.plan_hash);
    rc = h->run_graph(key2 + ":prep", s, [&](hipStream_t st) {
        hipLaunchKernelGGL(k_mrg_union, dim3(m), dim3(256), 0, st, cent1, nch1, m, (int)k, uni_b,
                           nu, len_ptr);
        const uint32_t padded = kc_pad64((uint32_t)cap);
        hipLaunchKernelGGL(k_gather_soa, dim3((padded + 255) / 256), dim3(256), 0, st,
                           pts->f32, pts->ld, d, uni_b, nu, padded, (float*)R2.xs, R2.stride);
        kc_enqueue_gon_prep(R2, H2, jobs2, st);
    });
    if (rc) return rc;
    done = false;
    if (h->allow_resident) {
        int v = 0;
        uint32_t G = 0;
        if (h->resident_fit(d, cap, &v, &G)) {
            const uint64_t sw = kc_resident_slot_words((int)k, G);
            u64* slots = (u64*)h->ws("m2.slots", sizeof(u64) * sw);
            uint32_t* abort_flag = (uint32_t*)h->ws("m2.abort", 64);
            if (!slots || !abort_flag) return h->fail(KC_ENOMEM, "workspace allocation failed");
            kc_fill_u64(slots, 0ull, sw, s);
            kc_fill_u32(abort_flag, 0u, 1, s);
            hipError_t e = kc_gon_resident(d, v, G, R2.xs, R2.stride, 0, (uint32_t)cap, len_ptr, 0,
                                           (int)k, R2.mind, R2.keys, slots, abort_flag,
                                           h->spin_limit, nullptr, 0, 0, h->status_word,
                                           nullptr, nullptr, s);
            if (e == hipSuccess) {
                done = true;
            } else {
                (void)hipGetLastError();
            }
        }
    }
    if (!done) {
        rc = h->run_graph(key2 + ":steps", s, [&](hipStream_t st) { kc_enqueue_gon_steps(R2, st); });
        if (rc) return rc;
    }
    rc = h->run_graph(key2 + ":finish", s, [&](hipStream_t st) {
        kc_gon_finish(R2, centers, n_centers, nullptr, r2b, nullptr, uni_b, st);
    });
    if (rc) return rc;

    // ---- covering radius over all points: FP32 MFMA in either precision (one
    // pass over the points; the FP32 bound leaves far fewer points for FP64)
    kc_points p32 = *pts;
    p32.prec = KC_FP32;
    p32.bf16 = nullptr;
    return kc_assign_run(h, &p32, centers, (uint32_t)k, n_centers, nullptr, radius, s, "m3.");
}


// Multi-round MRG: Algorithm 1 with its while loop (Lemma 3 and Eq. 1 give
// the factor 2(i+1) after i passes).  The sample S starts as all points; while
// |S| > capacity it is split into ceil(|S| / capacity) contiguous blocks of
// its ascending order (sizes differ by at most one) and Gonzalez(k) runs on
// every block (first center: the block's smallest index), all blocks as the
// segments of one batched run; S becomes the ascending union of their
// centers.  Then Gonzalez(k) on S, first center S[0], and the covering radius
// over all points.  The host reads |S| once per pass.
int kcenter_mrg_rounds(kc_handle* h, const kc_points* pts, int64_t k, int64_t capacity,
                       int64_t* centers, int64_t* n_centers, double* radius, int32_t* rounds,
                       void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, false);
    if (rc) return rc;
    if (k < 1 || k >= (1 << 24)) return h->fail(KC_EINVAL, "k=%lld out of range", (long long)k);
    if (capacity < 1) return h->fail(KC_EINVAL, "capacity must be >= 1");
    if (!centers || !n_centers || !radius) return h->fail(KC_EINVAL, "outputs NULL");
    hipStream_t s = (hipStream_t)stream;
    kc_validate_points(h, pts, s);
    const int d = pts->d;
    const float* Xc = pts->f32;   // rows of the current sample
    int64_t ldc = pts->ld;
    const int64_t* S = nullptr;   // global index of each row of Xc (NULL: identity)
    int64_t ns = pts->n;
    int r = 0;
    while (ns > capacity) {
        const int64_t mi = (ns + capacity - 1) / capacity;
        if (mi * k >= (int64_t)0xFFFFFFFFll || mi > (1 << 24))
            return h->fail(KC_EINVAL, "too many blocks (%lld) for one pass", (long long)mi);
        std::vector<KcGonJob> jobs((size_t)mi);
        std::vector<int64_t> base((size_t)mi);
        for (int64_t p = 0; p < mi; ++p) {
            const int64_t lo = p * ns / mi, hi = (p + 1) * ns / mi;
            jobs[p].X = Xc;
            jobs[p].ld = ldc;
            jobs[p].row0 = (uint64_t)lo;
            jobs[p].len = (uint32_t)(hi - lo);
            jobs[p].first = 0;
            jobs[p].k = (uint32_t)k;
            base[p] = lo;
        }
        const std::string pre = r & 1 ? "mr1." : "mr0.";
        KcGonRun R;
        KcGonHost H;
        rc = kc_plan_gon(h, pre, d, 1024, jobs, R, H, s);
        if (rc) return rc;
        int64_t* cent = (int64_t*)h->ws("mr.cent", sizeof(int64_t) * (size_t)(mi * k));
        int64_t* nch = (int64_t*)h->ws("mr.nch", sizeof(int64_t) * (size_t)mi);
        int64_t* uni = (int64_t*)h->ws(pre + "uni", sizeof(int64_t) * (size_t)(mi * k));
        int64_t* nu = (int64_t*)h->ws("mr.nu", 16);
        uint32_t* segl = (uint32_t*)h->ws("mr.segl", 16);
        const int64_t* rb = S ? nullptr
                              : (const int64_t*)h->upload("mr.rb", base.data(),
                                                          sizeof(int64_t) * base.size(), s);
        if (!cent || !nch || !uni || !nu || !segl || (!S && !rb))
            return h->fail(KC_ENOMEM, "workspace allocation failed");
        const std::string key = kc_key("mrr", {pts->f32, cent, Xc, S},
                                       {pts->n, d, pts->ld, k, capacity, r, ns});
        R.xa = Xc;   // the finishing pass reads the rows (no staging copy needed)
        R.lda = ldc;
        rc = kc_run_gon(h, key, R, H, jobs, "mrg_rounds", s, [&](hipStream_t st) {
            kc_fill_u64((u64*)cent, ~0ull, (uint64_t)(mi * k), st);
            kc_gon_finish(R, cent, nch, nullptr, nullptr, rb, S, st);
        });
        if (rc) return rc;
        hipLaunchKernelGGL(k_mrg_union, dim3((unsigned)mi), dim3(256), 0, s, cent, nch, (int)mi,
                           (int)k, uni, nu, segl);
        int64_t nn = 0;
        if (hipMemcpyAsync(&nn, nu, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return h->fail(KC_EHIP, "readback failed");
        ++r;
        if (nn >= ns)
            return h->fail(KC_ENOCONV, "pass %d left %lld of %lld points (k too close to the "
                           "capacity)", r, (long long)nn, (long long)ns);
        float* Xg = (float*)h->ws(pre + "x", sizeof(float) * (size_t)nn * d);
        if (!Xg) return h->fail(KC_ENOMEM, "workspace allocation failed");
        const uint64_t tot = (uint64_t)nn * d;
        hipLaunchKernelGGL(k_gather_rows64, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                           pts->f32, pts->ld, d, uni, (uint64_t)nn, Xg);
        S = uni;
        Xc = Xg;
        ldc = d;
        ns = nn;
    }
    // the last round: Gonzalez(k) on S, first center its smallest index
    std::vector<KcGonJob> jobs(1);
    jobs[0] = KcGonJob{Xc, ldc, 0, (uint32_t)ns, 0, (uint32_t)k};
    KcGonRun R;
    KcGonHost H;
    rc = kc_plan_gon(h, "mrf.", d, 1024, jobs, R, H, s);
    if (rc) return rc;
    const std::string key = kc_key("mrf", {pts->f32, Xc, S, centers, n_centers},
                                   {pts->n, d, pts->ld, k, capacity, r, ns});
    R.xa = Xc;
    R.lda = ldc;
    rc = kc_run_gon(h, key, R, H, jobs, "mrg_rounds", s, [&](hipStream_t st) {
        kc_gon_finish(R, centers, n_centers, nullptr, nullptr, nullptr, S, st);
    });
    if (rc) return rc;
    ++r;
    if (rounds) *rounds = r;
    kc_points p32 = *pts;
    p32.prec = KC_FP32;
    p32.bf16 = nullptr;
    return kc_assign_run(h, &p32, centers, (uint32_t)k, n_centers, nullptr, radius, s, "mra.");
}

}  // extern "C"
