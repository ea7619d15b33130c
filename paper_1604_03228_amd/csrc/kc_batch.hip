// kc_batch.hip -- many independent k-center problems of mixed n, d, k and
// algorithm in shared launches.
//
// For every dimension d present, the problems whose points fit a
// co-resident register-resident grid (every partition, for MRG) and the
// others form two groups; for each group:
//   stage 1  every Gonzalez problem and every partition of every MRG problem
//            is one segment of a single batched run: register-resident,
//            several segments per cooperative launch, when every segment
//            fits a co-resident grid, else streamed (segments in descending
//            order of k, so step t launches only the tiles of segments that
//            still have centers to choose; one HIP graph per plan);
//   stage 2  the MRG unions (built on the device) are the segments of a
//            second batched run;
//   stage 3  each MRG problem's covering radius by the MFMA assignment.
// EIM problems that never sample (n at most Algorithm 2's threshold) are
// Gonzalez problems from point 0 and join stage 1; the others run their
// sampling loop (which synchronises per iteration) and finish on the
// single-problem path; problems streamed in BF16 also take their
// single-problem entry point.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <numeric>

#include "kc_host.h"

struct KcBatchOut {
    int64_t keyoff;       // first key / center slot of the segment
    int64_t k;
    int64_t seg;          // segment index (n_chosen, radius)
    int64_t* centers;     // caller's [k]
    int64_t* n_centers;   // caller's [1] or NULL
    double* radius;       // caller's [1] or NULL
};

__global__ void k_batch_out(const KcBatchOut* __restrict__ tab, int count,
                            const int64_t* __restrict__ cent, const int64_t* __restrict__ nch,
                            const double* __restrict__ rad)
{
    const int i = blockIdx.x;
    if (i >= count) return;
    const KcBatchOut o = tab[i];
    for (int64_t t = threadIdx.x; t < o.k; t += blockDim.x) o.centers[t] = cent[o.keyoff + t];
    if (threadIdx.x == 0) {
        if (o.n_centers) *o.n_centers = nch[o.seg];
        if (o.radius) *o.radius = rad[o.seg];
    }
}

// MRG unions of several problems: block p of problem q sorts its partition's
// centers into uni[uoff_q + ...]; see k_mrg_union for one problem.
struct KcUnionJob {
    int64_t keyoff;       // first center slot of the problem's first partition
    int64_t seg0;         // its first segment (n_chosen index)
    int64_t m, k;
    int64_t uoff;         // offset of the problem's union in uni
    int64_t seg2;         // the problem's segment in the round-2 run
};

__global__ void k_batch_union(const KcUnionJob* __restrict__ jobs, const int32_t* __restrict__ blk_job,
                              const int32_t* __restrict__ blk_part,
                              const int64_t* __restrict__ cent, const int64_t* __restrict__ nch,
                              int64_t* __restrict__ uni, int64_t* __restrict__ nuni,
                              KcSeg* __restrict__ segs2)
{
    const KcUnionJob J = jobs[blk_job[blockIdx.x]];
    const int64_t p = blk_part[blockIdx.x];
    __shared__ int64_t off;
    if (threadIdx.x == 0) {
        int64_t o = 0;
        for (int64_t q = 0; q < p; ++q) o += nch[J.seg0 + q];
        off = o;
        if (p == J.m - 1) {
            const int64_t tot = o + nch[J.seg0 + p];
            nuni[blk_job[blockIdx.x]] = tot;
            segs2[J.seg2].len = (uint32_t)tot;
        }
    }
    __syncthreads();
    const int64_t np = nch[J.seg0 + p];
    const int64_t* c = cent + J.keyoff + p * J.k;
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
        const int64_t v = c[i];
        int64_t r = 0;
        for (int64_t j = 0; j < np; ++j) r += c[j] < v;
        uni[J.uoff + off + r] = v;
    }
}

// SoA columns [base, base+padded) <- rows uni[uoff + i] of X (padding repeats
// the union's first row)
__global__ void k_batch_gather(const float* __restrict__ X, int64_t ld, int d,
                               const int64_t* __restrict__ uni, int64_t uoff,
                               const int64_t* __restrict__ nu, uint32_t padded,
                               float* __restrict__ xs, uint64_t stride, uint64_t base)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    const int64_t cnt = *nu;
    const uint64_t r = (uint64_t)((int64_t)i < cnt ? uni[uoff + i] : uni[uoff]);
    for (int j = 0; j < d; ++j) xs[(uint64_t)j * stride + base + i] = X[r * ld + j];
}

// SoA columns [base, base+padded) <- rows idx[i] of X (padding repeats the
// first row), and the segment's remap entries map[off + i] = idx[i]
__global__ void k_batch_gather_u32(const float* __restrict__ X, int64_t ld, int d,
                                   const uint32_t* __restrict__ idx, uint32_t n, uint32_t padded,
                                   float* __restrict__ xs, uint64_t stride, uint64_t base,
                                   int64_t* __restrict__ map, uint64_t off)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= padded) return;
    const uint64_t r = idx[i < n ? i : 0];
    if (i < n) map[off + i] = (int64_t)r;
    for (int j = 0; j < d; ++j) xs[(uint64_t)j * stride + base + i] = X[r * ld + j];
}

static int check_problem(kc_handle* h, const kc_problem& p, int i)
{
    int rc = kc_check_points(h, &p.pts, true);
    if (rc) return h->fail(rc, "problem %d: %s", i, h->last_error.c_str());
    if (p.k < 1 || p.k >= (1 << 24)) return h->fail(KC_EINVAL, "problem %d: k out of range", i);
    if (!p.centers || !p.n_centers || !p.radius)
        return h->fail(KC_EINVAL, "problem %d: outputs NULL", i);
    switch (p.algo) {
    case KC_ALGO_GON:
        if (p.first < 0 || p.first >= p.pts.n)
            return h->fail(KC_EINVAL, "problem %d: first out of range", i);
        return KC_OK;
    case KC_ALGO_MRG:
        if (p.m < 1 || !p.offsets || p.offsets[0] != 0 || p.offsets[p.m] != p.pts.n)
            return h->fail(KC_EINVAL, "problem %d: bad offsets", i);
        for (int q = 0; q < p.m; ++q)
            if (p.offsets[q + 1] < p.offsets[q])
                return h->fail(KC_EINVAL, "problem %d: offsets not monotone", i);
        return KC_OK;
    case KC_ALGO_EIM:
        if (!(p.eim.eps > 0.0 && p.eim.eps < 1.0) || !(p.eim.phi > 0.0) || p.eim.max_iters < 1)
            return h->fail(KC_EINVAL, "problem %d: bad EIM parameters", i);
        return KC_OK;
    default:
        return h->fail(KC_EINVAL, "problem %d: unknown algorithm %d", i, p.algo);
    }
}

// An EIM problem whose n does not exceed Algorithm 2's threshold
// (4/eps) k n^eps ln n never samples: its sample is all of V and its result
// Gonzalez's traversal from V's smallest index, 0, with the covering radius
// -- exactly a Gonzalez problem with first = 0, which the batch runs in the
// shared launches (the same constants and comparison as kcenter_eim).
static bool eim_as_gon(const kc_problem& p)
{
    if (p.algo != KC_ALGO_EIM) return false;
    const double n = (double)p.pts.n;
    const double thr = (4.0 / p.eim.eps) * (double)p.k * pow(n, p.eim.eps) * log(n);
    return !(n > thr);
}

static bool gon_like(const kc_problem& p)
{
    return p.algo == KC_ALGO_GON || eim_as_gon(p);
}

struct SegTag {
    int prob;   // problem index
    int part;   // partition (MRG) or -1 (GON)
};

// One group's prepared launches: the plans, tables and workspace of its
// stages, built by group_prepare and run (any number of times, while the
// problems' sizes stay those it was built for) by group_execute.
struct KcBatchGroup {
    int d = 0;
    std::string P, key;
    std::vector<int> ids;
    // stage 1
    std::vector<KcGonJob> sj;
    KcGonRun R;
    KcGonHost H;
    const int64_t* rb = nullptr;
    int64_t* cent = nullptr;
    int64_t* nch = nullptr;
    double* rad = nullptr;
    std::vector<KcBatchOut> outs;
    const KcBatchOut* outs_d = nullptr;
    bool bf = false;   // streamed on a BF16 copy the library rounds, exact rescoring
    KcBf16Run B;
    // stage 2 (MRG problems)
    std::vector<KcUnionJob> uj;
    std::vector<int32_t> blk_job, blk_part;
    std::vector<int> o2, mrg_ids;
    std::vector<KcGonJob> sj2;
    KcGonRun R2;
    KcGonHost H2;
    int64_t* uni = nullptr;
    int64_t* nuni = nullptr;
    int64_t* cent2 = nullptr;
    int64_t* nch2 = nullptr;
    const KcUnionJob* uj_d = nullptr;
    const int32_t* bj_d = nullptr;
    const int32_t* bp_d = nullptr;
    const KcBatchOut* outs2_d = nullptr;
    uint64_t uh = 0;
};

static int group_prepare(kc_handle* h, const kc_problem* probs, const std::vector<int>& ids, int d,
                         const char* tag, hipStream_t s, KcBatchGroup& G)
{
    char pre[32];
    snprintf(pre, sizeof pre, "b%d%s.", d, tag);
    G.d = d;
    G.P = pre;
    G.ids = ids;
    const std::string& P = G.P;

    // ---- stage 1: one run over all Gonzalez problems and MRG partitions
    std::vector<KcGonJob> jobs;
    std::vector<SegTag> tags;
    std::vector<int64_t> rbase;
    for (int i : ids) {
        const kc_problem& p = probs[i];
        if (gon_like(p)) {
            KcGonJob j;
            j.X = p.pts.f32;
            j.ld = p.pts.ld;
            j.row0 = 0;
            j.len = (uint32_t)p.pts.n;
            j.first = p.algo == KC_ALGO_GON ? (uint32_t)p.first : 0u;
            j.k = (uint32_t)p.k;
            jobs.push_back(j);
            tags.push_back({i, -1});
            rbase.push_back(0);
        } else {
            for (int q = 0; q < p.m; ++q) {
                KcGonJob j;
                j.X = p.pts.f32;
                j.ld = p.pts.ld;
                j.row0 = (uint64_t)p.offsets[q];
                j.len = (uint32_t)(p.offsets[q + 1] - p.offsets[q]);
                j.first = 0;
                j.k = (uint32_t)p.k;
                jobs.push_back(j);
                tags.push_back({i, q});
                rbase.push_back(p.offsets[q]);
            }
        }
    }
    // descending k, stable (an MRG problem's partitions stay together)
    std::vector<int> ord(jobs.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return jobs[a].k > jobs[b].k; });
    std::vector<SegTag> st;
    std::vector<int64_t> sr;
    for (int q : ord) {
        G.sj.push_back(jobs[q]);
        st.push_back(tags[q]);
        sr.push_back(rbase[q]);
    }
    // A group that streams reads every point at every step: with enough
    // points the stream runs on a BF16 copy rounded from the FP32 rows (2d
    // bytes less per point and step, 4 more for its rounding radius) with
    // exact FP32 rescoring of the candidates, whose centers are the FP32
    // stream's.  The rescoring adds about 10 us per step (5e7 bytes at
    // 5 TB/s), so it runs from twice that in saved bytes: n (2d - 4) >= 1e8
    // (a d = 32 group of 1.7e6 points, a d = 8 group of 8.3e6).
    const uint64_t per = 2 * d > 4 ? (uint64_t)(2 * d - 4) : 0u;
    uint64_t saved = 0;
    for (const KcGonJob& j : G.sj) saved += (uint64_t)j.len * per;
    G.bf = !strcmp(tag, "s") && saved >= 100000000ull;
    int rc = kc_plan_gon(h, P + "1.", d, G.bf ? KC_BF_TILE_PTS : 1024, G.sj, G.R, G.H, s);
    if (rc) return rc;
    if (G.bf && (rc = kc_bf16_alloc(h, P + "1b.", G.R, G.B))) return rc;
    const int nseg = (int)G.sj.size();
    G.rb = (const int64_t*)h->upload(P + "1.rb", sr.data(), 8 * sr.size(), s);
    G.cent = (int64_t*)h->ws(P + "1.cent", 8 * std::max<uint64_t>(G.R.keysum, 1));
    G.nch = (int64_t*)h->ws(P + "1.nch", 8 * (size_t)nseg);
    G.rad = (double*)h->ws(P + "1.rad", 8 * (size_t)nseg);
    if (!G.rb || !G.cent || !G.nch || !G.rad)
        return h->fail(KC_ENOMEM, "workspace allocation failed");

    // outputs of the Gonzalez problems; layout of the MRG problems
    std::map<int, int> first_seg;   // MRG problem -> its first segment
    for (int q = 0; q < nseg; ++q) {
        const SegTag& t = st[q];
        const kc_problem& p = probs[t.prob];
        if (t.part < 0)
            G.outs.push_back(
                {(int64_t)G.H.segs[q].keyoff, p.k, q, p.centers, p.n_centers, p.radius});
        else if (t.part == 0)
            first_seg[t.prob] = q;
    }
    if (!G.outs.empty()) {
        G.outs_d = (const KcBatchOut*)h->upload(P + "1.outs", G.outs.data(),
                                                sizeof(KcBatchOut) * G.outs.size(), s);
        if (!G.outs_d) return h->fail(KC_ENOMEM, "workspace allocation failed");
    }
    G.key = P + "run1";
    // every problem's arrays, sizes and algorithm (the graphs embed their
    // pointers, strides and grids; the partition offsets enter through the
    // plans' signatures)
    for (int i : ids) {
        char b[160];
        const kc_problem& p = probs[i];
        snprintf(b, sizeof b, ":%p:%lld:%lld:%lld:%d:%lld:%d:%p:%p:%p", (const void*)p.pts.f32,
                 (long long)p.pts.n, (long long)p.pts.ld, (long long)p.k, p.algo,
                 (long long)p.first, p.m, (void*)p.centers, (void*)p.n_centers,
                 (void*)p.radius);
        G.key += b;
    }
    if (first_seg.empty()) return KC_OK;

    // ---- stage 2: MRG second rounds as the segments of one run
    std::vector<KcGonJob> j2;
    int64_t uoff = 0;
    for (auto& kv : first_seg) {
        const kc_problem& p = probs[kv.first];
        const int64_t cap = std::min<int64_t>((int64_t)p.m * p.k, p.pts.n);
        KcUnionJob J;
        J.keyoff = G.H.segs[kv.second].keyoff;
        J.seg0 = kv.second;
        J.m = p.m;
        J.k = p.k;
        J.uoff = uoff;
        J.seg2 = 0;   // set after the round-2 order is known
        for (int q = 0; q < p.m; ++q) {
            G.blk_job.push_back((int32_t)G.uj.size());
            G.blk_part.push_back(q);
        }
        G.uj.push_back(J);
        KcGonJob g;
        g.X = nullptr;   // gathered
        g.ld = p.pts.ld;
        g.row0 = (uint64_t)uoff;
        g.len = (uint32_t)cap;
        g.first = 0;
        g.k = (uint32_t)p.k;
        j2.push_back(g);
        G.mrg_ids.push_back(kv.first);
        uoff += cap;
    }
    G.o2.resize(j2.size());
    std::iota(G.o2.begin(), G.o2.end(), 0);
    std::stable_sort(G.o2.begin(), G.o2.end(), [&](int a, int b) { return j2[a].k > j2[b].k; });
    for (int q = 0; q < (int)G.o2.size(); ++q) {
        G.sj2.push_back(j2[G.o2[q]]);
        G.uj[G.o2[q]].seg2 = q;
    }
    rc = kc_plan_gon(h, P + "2.", d, 1024, G.sj2, G.R2, G.H2, s);
    if (rc) return rc;
    const int nu = (int)G.uj.size();
    G.uni = (int64_t*)h->ws(P + "2.uni", 8 * (size_t)std::max<int64_t>(uoff, 1));
    G.nuni = (int64_t*)h->ws(P + "2.nu", 8 * (size_t)nu);
    G.cent2 = (int64_t*)h->ws(P + "2.cent", 8 * std::max<uint64_t>(G.R2.keysum, 1));
    G.nch2 = (int64_t*)h->ws(P + "2.nch", 8 * (size_t)nu);
    G.uj_d = (const KcUnionJob*)h->upload(P + "2.uj", G.uj.data(), sizeof(KcUnionJob) * nu, s);
    G.bj_d = (const int32_t*)h->upload(P + "2.bj", G.blk_job.data(), 4 * G.blk_job.size(), s);
    G.bp_d = (const int32_t*)h->upload(P + "2.bp", G.blk_part.data(), 4 * G.blk_part.size(), s);
    if (!G.uni || !G.nuni || !G.cent2 || !G.nch2 || !G.uj_d || !G.bj_d || !G.bp_d)
        return h->fail(KC_ENOMEM, "workspace allocation failed");
    std::vector<KcBatchOut> outs2;
    for (int q = 0; q < nu; ++q) {
        const kc_problem& p = probs[G.mrg_ids[G.o2[q]]];
        outs2.push_back({(int64_t)G.H2.segs[q].keyoff, p.k, q, p.centers, p.n_centers, nullptr});
    }
    G.outs2_d =
        (const KcBatchOut*)h->upload(P + "2.outs", outs2.data(), sizeof(KcBatchOut) * nu, s);
    if (!G.outs2_d) return h->fail(KC_ENOMEM, "workspace allocation failed");
    // the union graph's grids follow the union jobs and round 2's plan
    G.uh = kc_hash_vec(G.blk_job, kc_hash_vec(G.uj, G.R2.plan_hash));
    return KC_OK;
}

static int group_execute(kc_handle* h, const kc_problem* probs, const KcBatchGroup& G,
                         hipStream_t s)
{
    const int d = G.d;
    const std::string& P = G.P;
    auto finish1 = [&](hipStream_t sst) {
        if (G.bf)
            kc_bf16_finish(G.R, G.B, G.cent, G.nch, nullptr, G.rad, G.rb, sst);
        else
            kc_gon_finish(G.R, G.cent, G.nch, nullptr, G.rad, G.rb, nullptr, sst);
        if (!G.outs.empty())
            hipLaunchKernelGGL(k_batch_out, dim3((unsigned)G.outs.size()), dim3(256), 0, sst,
                               G.outs_d, (int)G.outs.size(), G.cent, G.nch, G.rad);
    };
    int rc = G.bf ? kc_run_bf16(h, G.key + ":bf", G.R, G.B, G.H, G.sj, "batch_gon", s, finish1)
                  : kc_run_gon(h, G.key, G.R, G.H, G.sj, "batch_gon", s, finish1);
    if (rc || G.mrg_ids.empty()) return rc;
    const int nu = (int)G.uj.size();
    rc = h->run_graph(G.key + kc_hash_str(G.uh) + ":u", s, [&](hipStream_t sst) {
        hipLaunchKernelGGL(k_batch_union, dim3((unsigned)G.blk_job.size()), dim3(256), 0, sst,
                           G.uj_d, G.bj_d, G.bp_d, G.cent, G.nch, G.uni, G.nuni, G.R2.segs);
        for (int q = 0; q < nu; ++q) {
            const KcUnionJob& J = G.uj[G.o2[q]];
            const kc_problem& p = probs[G.mrg_ids[G.o2[q]]];
            const uint32_t padded = kc_pad64(G.sj2[q].len);
            hipLaunchKernelGGL(k_batch_gather, dim3((padded + 255) / 256), dim3(256), 0, sst,
                               p.pts.f32, p.pts.ld, d, G.uni, J.uoff, G.nuni + G.o2[q], padded,
                               (float*)G.R2.xs, G.R2.stride, G.H2.segs[q].base);
        }
    });
    if (rc) return rc;
    rc = kc_run_gon(h, G.key + ":r2", G.R2, G.H2, G.sj2, "batch_gon", s, [&](hipStream_t sst) {
        kc_gon_finish(G.R2, G.cent2, G.nch2, nullptr, nullptr, nullptr, G.uni, sst);
        hipLaunchKernelGGL(k_batch_out, dim3((unsigned)nu), dim3(256), 0, sst, G.outs2_d, nu,
                           G.cent2, G.nch2, (const double*)nullptr);
    });
    if (rc) return rc;

    // ---- stage 3: covering radius of every MRG problem (FP32 MFMA)
    for (int i : G.mrg_ids) {
        const kc_problem& p = probs[i];
        kc_points p32 = p.pts;
        p32.prec = KC_FP32;
        p32.bf16 = nullptr;
        rc = kc_assign_run(h, &p32, p.centers, (uint32_t)p.k, p.n_centers, nullptr, p.radius, s,
                           P + "a.");
        if (rc) return rc;
    }
    return KC_OK;
}

// The problems' grouping: per dimension, the FP32 Gonzalez and MRG problems
// whose points (every partition, for MRG) fit a co-resident register-resident
// grid ("r"), and the others ("s"), which stream -- one problem too large for
// the register file then leaves the others on the resident engine; EIM
// problems that sample run their loops in lockstep (`eim`); Gonzalez and MRG
// problems in BF16 run alone (`single`).
struct KcBatchLayout {
    std::vector<std::pair<int, std::vector<int>>> groups;   // (d, ids), tag r then s
    std::vector<const char*> tags;
    std::vector<int> eim;      // EIM problems that sample
    std::vector<int> single;
};

static void batch_layout(kc_handle* h, const kc_problem* probs, int count, KcBatchLayout& L)
{
    std::map<int, std::vector<int>> byd;
    for (int i = 0; i < count; ++i) {
        const kc_problem& p = probs[i];
        if ((p.algo != KC_ALGO_EIM || eim_as_gon(p)) && p.pts.prec == KC_FP32)
            byd[p.pts.d].push_back(i);
        else if (p.algo == KC_ALGO_EIM)
            L.eim.push_back(i);
        else
            L.single.push_back(i);
    }
    for (auto& g : byd) {
        const int d = g.first;
        std::vector<int> fit, other;
        for (int i : g.second) {
            const kc_problem& p = probs[i];
            bool ok = h->allow_resident;
            int v = 0;
            uint32_t G = 0;
            if (ok && gon_like(p)) ok = h->resident_fit(d, (uint64_t)p.pts.n, &v, &G);
            for (int q = 0; ok && p.algo == KC_ALGO_MRG && q < p.m; ++q) {
                const uint64_t len = (uint64_t)(p.offsets[q + 1] - p.offsets[q]);
                ok = len == 0 || h->resident_fit(d, len, &v, &G);
            }
            (ok ? fit : other).push_back(i);
        }
        if (!fit.empty()) {
            L.groups.push_back({d, fit});
            L.tags.push_back("r");
        }
        if (!other.empty()) {
            L.groups.push_back({d, other});
            L.tags.push_back("s");
        }
    }
}

// The EIM problems that sample: their Algorithm 2 loops run in lockstep (one
// wait per phase for all of them), each keeping its sample C; then, per
// dimension, the final Gonzalez of every problem on its C runs as the
// segments of one shared run (C's rows gathered, first center C's smallest
// index), and each problem's covering radius by the assignment.
static int run_eim_group(kc_handle* h, const kc_problem* probs, const std::vector<int>& ids,
                         hipStream_t s)
{
    if (ids.empty()) return KC_OK;
    std::vector<const uint32_t*> keep;
    std::vector<uint32_t> ncs;
    int rc0 = kc_eim_sample_many(h, probs, ids, keep, ncs, s);
    if (rc0) return rc0;
    std::map<int, std::vector<size_t>> byd;
    for (size_t q = 0; q < ids.size(); ++q) byd[probs[ids[q]].pts.d].push_back(q);
    for (auto& g : byd) {
        const int d = g.first;
        std::vector<size_t> ord = g.second;   // descending k, stable
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            return probs[ids[a]].k > probs[ids[b]].k;
        });
        std::vector<KcGonJob> jobs;
        uint64_t off = 0;
        for (size_t q : ord) {
            const kc_problem& p = probs[ids[q]];
            KcGonJob j;
            j.X = nullptr;   // gathered
            j.ld = p.pts.ld;
            j.row0 = off;    // its entries of the remap
            j.len = ncs[q];
            j.first = 0;
            j.k = (uint32_t)p.k;
            jobs.push_back(j);
            off += ncs[q];
        }
        char pre[32];
        snprintf(pre, sizeof pre, "bE%d.", d);
        const std::string P(pre);
        KcGonRun R;
        KcGonHost H;
        int rc = kc_plan_gon(h, P, d, 1024, jobs, R, H, s);
        if (rc) return rc;
        int64_t* map = (int64_t*)h->ws(P + "map", 8 * std::max<uint64_t>(off, 1));
        int64_t* cent = (int64_t*)h->ws(P + "cent", 8 * std::max<uint64_t>(R.keysum, 1));
        int64_t* nch = (int64_t*)h->ws(P + "nch", 8 * jobs.size());
        std::vector<KcBatchOut> outs;
        for (size_t q = 0; q < ord.size(); ++q) {
            const kc_problem& p = probs[ids[ord[q]]];
            outs.push_back({(int64_t)H.segs[q].keyoff, p.k, (int64_t)q, p.centers, p.n_centers,
                            nullptr});
        }
        const KcBatchOut* outs_d =
            (const KcBatchOut*)h->upload(P + "outs", outs.data(), sizeof(KcBatchOut) * outs.size(), s);
        if (!map || !cent || !nch || !outs_d)
            return h->fail(KC_ENOMEM, "workspace allocation failed");
        for (size_t q = 0; q < ord.size(); ++q) {
            const kc_problem& p = probs[ids[ord[q]]];
            const uint32_t padded = kc_pad64(ncs[ord[q]]);
            hipLaunchKernelGGL(k_batch_gather_u32, dim3((padded + 255) / 256), dim3(256), 0, s,
                               p.pts.f32, p.pts.ld, d, keep[ord[q]], ncs[ord[q]], padded,
                               (float*)R.xs, R.stride, H.segs[q].base, map, jobs[q].row0);
        }
        std::string key = P + "run";
        for (size_t q : ord) {
            char b[96];
            const kc_problem& p = probs[ids[q]];
            snprintf(b, sizeof b, ":%p:%lld:%p:%p", (const void*)p.pts.f32, (long long)p.k,
                     (void*)p.centers, (void*)p.n_centers);
            key += b;
        }
        rc = kc_run_gon(h, key, R, H, jobs, "batch_gon", s, [&](hipStream_t sst) {
            kc_gon_finish(R, cent, nch, nullptr, nullptr, nullptr, map, sst);
            hipLaunchKernelGGL(k_batch_out, dim3((unsigned)outs.size()), dim3(256), 0, sst,
                               outs_d, (int)outs.size(), cent, nch, (const double*)nullptr);
        });
        if (rc) return rc;
        for (size_t q : ord) {
            const kc_problem& p = probs[ids[q]];
            kc_points p32 = p.pts;
            p32.prec = KC_FP32;
            p32.bf16 = nullptr;
            rc = kc_assign_run(h, &p32, p.centers, (uint32_t)p.k, p.n_centers, nullptr,
                               p.radius, s, P + "a.");
            if (rc) return rc;
        }
    }
    return KC_OK;
}

static int run_single(kc_handle* h, const kc_problem& p, int i, hipStream_t s)
{
    int rc;
    if (p.algo == KC_ALGO_EIM) {
        int64_t ns = 0;
        int32_t ni = 0;
        rc = kcenter_eim(h, &p.pts, p.k, &p.eim, p.centers, p.n_centers, p.radius, nullptr, &ns,
                         nullptr, &ni, s);
    } else if (p.algo == KC_ALGO_GON) {
        double* tr = (double*)h->ws("bo.trace", 8 * (size_t)p.k);
        if (!tr) return h->fail(KC_ENOMEM, "workspace allocation failed");
        rc = kcenter_gonzalez(h, &p.pts, p.k, p.first, p.centers, tr, p.n_centers, s);
        if (!rc) {
            // radius: the last chosen entry of the trace, via the assignment
            rc = kc_assign_run(h, &p.pts, p.centers, (uint32_t)p.k, p.n_centers, nullptr,
                               p.radius, s, "bo.a.");
        }
    } else {
        rc = kcenter_mrg(h, &p.pts, p.offsets, p.m, p.k, p.centers, p.n_centers, p.radius,
                         nullptr, nullptr, nullptr, nullptr, nullptr, s);
    }
    if (rc) return h->fail(rc, "problem %d: %s", i, h->last_error.c_str());
    return KC_OK;
}

extern "C" int kcenter_batch(kc_handle* h, const kc_problem* probs, int32_t count, void* stream)
{
    if (!h) return KC_EINVAL;
    if (count < 0 || (count > 0 && !probs)) return h->fail(KC_EINVAL, "bad problem list");
    for (int i = 0; i < count; ++i) {
        int rc = check_problem(h, probs[i], i);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) kc_validate_points(h, &probs[i].pts, s);
    KcBatchLayout L;
    batch_layout(h, probs, count, L);
    for (size_t g = 0; g < L.groups.size(); ++g) {
        KcBatchGroup G;
        int rc = group_prepare(h, probs, L.groups[g].second, L.groups[g].first, L.tags[g], s, G);
        if (!rc) rc = group_execute(h, probs, G, s);
        if (rc) return rc;
    }
    {
        const int rc = run_eim_group(h, probs, L.eim, s);
        if (rc) return rc;
    }
    for (int i : L.single) {
        int rc = run_single(h, probs[i], i, s);
        if (rc) return rc;
    }
    return KC_OK;
}

// ---------------------------------------------------------------------------
// a batch planned once and run many times

struct kc_batch_plan {
    kc_handle* sub = nullptr;             // private workspace, tables and graphs
    std::vector<kc_problem> probs;        // the problems, offsets copied
    std::vector<std::vector<int64_t>> offsets;
    KcBatchLayout layout;
    std::vector<KcBatchGroup> groups;     // prepared on the first run
    bool prepared = false;
};

__global__ void k_status_fold(uint32_t* __restrict__ dst, uint32_t* __restrict__ src)
{
    if (threadIdx.x == 0) {
        const uint32_t v = *src;
        if (v) {
            atomicOr(dst, v);
            *src = 0u;
        }
    }
}

extern "C" int kcenter_batch_plan(kc_handle* h, const kc_problem* probs, int32_t count,
                                  kc_batch_plan** plan)
{
    if (!h) return KC_EINVAL;
    if (!plan) return h->fail(KC_EINVAL, "plan NULL");
    *plan = nullptr;
    if (count < 0 || (count > 0 && !probs)) return h->fail(KC_EINVAL, "bad problem list");
    for (int i = 0; i < count; ++i) {
        int rc = check_problem(h, probs[i], i);
        if (rc) return rc;
    }
    kc_batch_plan* B = new (std::nothrow) kc_batch_plan();
    if (!B) return h->fail(KC_ENOMEM, "plan allocation failed");
    int rc = kc_create(&B->sub);
    if (rc) {
        delete B;
        return h->fail(rc, "plan handle: %s", kc_strerror(rc));
    }
    kc_handle* S = B->sub;
    S->use_graphs = h->use_graphs;
    S->allow_resident = h->allow_resident;
    S->mfma_split = h->mfma_split;
    S->autotune = h->autotune;
    S->tuned = h->tuned;
    S->tune_ms = h->tune_ms;
    S->spin_limit = h->spin_limit;
    S->validate = h->validate;
    S->resident_cap = h->resident_cap;
    S->graph_cap = 0;   // a plan keeps every graph it captures
    B->probs.assign(probs, probs + count);
    B->offsets.resize(count);
    for (int i = 0; i < count; ++i)
        if (probs[i].algo == KC_ALGO_MRG) {
            B->offsets[i].assign(probs[i].offsets, probs[i].offsets + probs[i].m + 1);
            B->probs[i].offsets = B->offsets[i].data();
        }
    batch_layout(S, B->probs.data(), count, B->layout);
    *plan = B;
    return KC_OK;
}

extern "C" int kcenter_batch_run(kc_handle* h, kc_batch_plan* plan, void* stream)
{
    if (!h) return KC_EINVAL;
    if (!plan) return h->fail(KC_EINVAL, "plan NULL");
    kc_handle* S = plan->sub;
    hipStream_t s = (hipStream_t)stream;
    const kc_problem* probs = plan->probs.data();
    const KcBatchLayout& L = plan->layout;
    int rc = KC_OK;
    for (const kc_problem& p : plan->probs) kc_validate_points(S, &p.pts, s);
    if (!plan->prepared) {
        plan->groups.resize(L.groups.size());
        for (size_t g = 0; g < L.groups.size() && !rc; ++g)
            rc = group_prepare(S, probs, L.groups[g].second, L.groups[g].first, L.tags[g], s,
                               plan->groups[g]);
        if (rc) {
            plan->groups.clear();
            return h->fail(rc, "%s", S->last_error.c_str());
        }
        plan->prepared = true;
    }
    for (size_t g = 0; g < plan->groups.size() && !rc; ++g)
        rc = group_execute(S, probs, plan->groups[g], s);
    if (!rc) rc = run_eim_group(S, probs, L.eim, s);
    for (size_t q = 0; q < L.single.size() && !rc; ++q)
        rc = run_single(S, probs[L.single[q]], L.single[q], s);
    // the plan's device status joins the caller's handle
    hipLaunchKernelGGL(k_status_fold, dim3(1), dim3(64), 0, s, h->status_word, S->status_word);
    if (rc) return h->fail(rc, "%s", S->last_error.c_str());
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
}

extern "C" void kcenter_batch_free(kc_batch_plan* plan)
{
    if (!plan) return;
    kc_destroy(plan->sub);   // synchronises the device first
    delete plan;
}
