// kc_api.hip -- host side of libkcenter: the C ABI declared in
// include/kcenter.h, argument checks, workspace, launch planning and HIP
// graph capture of the per-step launch sequences.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "../../include/kcenter.h"
#include "kc_internal.h"
#include "kc_host.h"

// ---------------------------------------------------------------------------
// handle

kc_handle::~kc_handle()
{
    clear_graphs();
    for (auto& kv : spans)
        for (auto& sp : kv.second) {
            (void)hipEventDestroy(sp.a);
            (void)hipEventDestroy(sp.b);
        }
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    for (auto& kv : staging) {
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
        if (kv.second.p) (void)hipHostFree(kv.second.p);
    }
    for (auto& kv : bufs) (void)hipFree(kv.second.p);
    if (status_word) (void)hipFree(status_word);
}

hipEvent_t kc_handle::span_begin(hipStream_t s)
{
    if (!timing) return nullptr;
    hipEvent_t e = nullptr;
    if (!event_pool.empty()) {
        e = event_pool.back();
        event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipEventRecord(e, s) != hipSuccess) {   // no span; the event goes back
        (void)hipGetLastError();
        event_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void kc_handle::span_end(const char* name, hipEvent_t a, int64_t launches, hipStream_t s)
{
    if (!timing || !a) return;
    hipEvent_t b = nullptr;
    if (!event_pool.empty()) {
        b = event_pool.back();
        event_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
        (void)hipGetLastError();
        event_pool.push_back(a);
        return;
    }
    if (hipEventRecord(b, s) != hipSuccess) {   // the span is dropped
        (void)hipGetLastError();
        event_pool.push_back(a);
        event_pool.push_back(b);
        return;
    }
    spans[name].push_back(TimedSpan{a, b, launches});
}

void kc_handle::clear_graphs()
{
    for (auto& kv : graphs) {
        (void)hipGraphExecDestroy(kv.second.exec);
        (void)hipGraphDestroy(kv.second.graph);
    }
    graphs.clear();
}

int kc_handle::fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error = buf;
    return code;
}

void* kc_handle::ws(const std::string& name, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = bufs.find(name);
    if (it != bufs.end() && it->second.bytes >= bytes) return it->second.p;
    if (it != bufs.end()) {
        // growing invalidates every captured graph (they embed the old address);
        // the old buffer is freed only once no queued work can still use it
        if (hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        clear_graphs();
        (void)hipFree(it->second.p);
        bufs.erase(it);
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    bufs[name] = DevBuf{p, bytes};
    return p;
}

// Upload a host table to a named workspace buffer.  The copy is ordered on
// stream s after the work already queued there (which may still read the
// buffer's previous contents): it reads a pinned host staging buffer of the
// same name, and the staging bytes are rewritten only once the previous copy
// from them has completed.  The copy is skipped when the same bytes were
// uploaded last time, so repeated identical calls stay free of host waits.
void* kc_handle::upload(const std::string& name, const void* src, size_t bytes, hipStream_t s)
{
    void* p = ws(name, bytes);
    if (!p) return nullptr;
    auto& shadow = shadows[name];
    if (shadow.size() == bytes && bytes > 0 && memcmp(shadow.data(), src, bytes) == 0 &&
        shadow_ptr[name] == p)
        return p;
    if (bytes > 0) {
        Staging& st = staging[name];
        if (st.done && hipEventSynchronize(st.done) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (st.cap < bytes) {
            if (st.p) (void)hipHostFree(st.p);
            st.p = nullptr;
            st.cap = 0;
            const size_t cap = (bytes + 4095) & ~(size_t)4095;
            if (hipHostMalloc(&st.p, cap, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                st.p = nullptr;
                return nullptr;
            }
            st.cap = cap;
        }
        if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            st.done = nullptr;
            return nullptr;
        }
        memcpy(st.p, src, bytes);
        if (hipMemcpyAsync(p, st.p, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(st.done, s) != hipSuccess) {
            (void)hipGetLastError();
            shadow.clear();
            return nullptr;
        }
    }
    shadow.assign((const char*)src, (const char*)src + bytes);
    shadow_ptr[name] = p;
    return p;
}

// Run `enqueue` on `stream`, through a cached HIP graph when graphs are on and
// the stream is not already being captured by the caller.
int kc_handle::run_graph(const std::string& key, hipStream_t stream,
                         const std::function<void(hipStream_t)>& enqueue)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusNone;
    }
    if (!use_graphs || cs != hipStreamCaptureStatusNone || stream == nullptr) {
        enqueue(stream);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? KC_OK : fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
    }
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        if (graph_cap && graphs.size() >= graph_cap) clear_graphs();
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail(KC_EHIP, "begin capture: %s", hipGetErrorString(e));
        enqueue(stream);
        e = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess) return fail(KC_EHIP, "end capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(KC_EHIP, "instantiate: %s", hipGetErrorString(e));
        }
        it = graphs.emplace(key, GraphEntry{g, ex}).first;
    }
    hipError_t e = hipGraphLaunch(it->second.exec, stream);
    return e == hipSuccess ? KC_OK : fail(KC_EHIP, "graph launch: %s", hipGetErrorString(e));
}

int kc_handle::tune(const std::string& key, int nvar, const bool* feasible, hipStream_t s,
                    const std::function<int(int)>& run)
{
    int first = -1, nfeas = 0;
    for (int v = 0; v < nvar; ++v)
        if (feasible[v]) {
            if (first < 0) first = v;
            ++nfeas;
        }
    if (first < 0) return fail(KC_EUNSUPPORTED, "no feasible variant for %s", key.c_str());
    if (tune_force >= 0) return run(tune_force < nvar && feasible[tune_force] ? tune_force : first);
    auto it = tuned.find(key);
    if (it != tuned.end() && feasible[it->second]) return run(it->second);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusActive;
    }
    if (!autotune || nfeas == 1 || cs != hipStreamCaptureStatusNone) return run(first);
    hipEvent_t ea = nullptr, eb = nullptr;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        (void)hipGetLastError();
        if (ea) (void)hipEventDestroy(ea);
        return run(first);
    }
    std::vector<float> ms(nvar, -1.f);
    int best = first, rc = KC_OK;
    const bool timing_was = timing;   // measured runs stay out of the spans
    timing = false;
    for (int v = 0; v < nvar && rc == KC_OK; ++v) {
        if (!feasible[v]) continue;
        rc = run(v);   // warm: caches, captured graphs
        if (rc) break;
        (void)hipEventRecord(ea, s);   // a failed record shows as a failed elapsed time
        rc = run(v);
        (void)hipEventRecord(eb, s);
        if (rc) break;
        float t = 0.f;
        if (hipEventSynchronize(eb) != hipSuccess || hipEventElapsedTime(&t, ea, eb) != hipSuccess) {
            (void)hipGetLastError();
            t = 1e30f;
        }
        ms[v] = t;
        if (ms[best] < 0.f || t < ms[best]) best = v;
    }
    timing = timing_was;
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (rc) return rc;
    tuned[key] = best;
    tune_ms[key] = ms;
    return run(best);   // the call's results and spans: the chosen variant's
}

int kc_handle::choice(const std::string& key, int nvar, const bool* feasible, hipStream_t s,
                      bool* measure)
{
    *measure = false;
    int first = -1, nfeas = 0;
    for (int v = 0; v < nvar; ++v)
        if (feasible[v]) {
            if (first < 0) first = v;
            ++nfeas;
        }
    if (first < 0) return -1;
    if (tune_force >= 0) return tune_force < nvar && feasible[tune_force] ? tune_force : first;
    auto it = tuned.find(key);
    if (it != tuned.end() && feasible[it->second]) return it->second;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusActive;
    }
    *measure = autotune && nfeas > 1 && cs == hipStreamCaptureStatusNone;
    return first;
}

void* kc_handle::pinned(const std::string& name, size_t bytes)
{
    Staging& st = staging["pinned:" + name];
    if (st.cap >= bytes && st.p) return st.p;
    if (st.p) {
        if (hipDeviceSynchronize() != hipSuccess) {   // a queued copy may still target it
            (void)hipGetLastError();
            return nullptr;
        }
        (void)hipHostFree(st.p);
    }
    st.p = nullptr;
    st.cap = 0;
    const size_t cap = (bytes + 4095) & ~(size_t)4095;
    if (hipHostMalloc(&st.p, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        st.p = nullptr;
        return nullptr;
    }
    st.cap = cap;
    return st.p;
}

// ---------------------------------------------------------------------------
// argument checks

int kc_check_points(kc_handle* h, const kc_points* p, bool need_bf16_if_asked)
{
    if (!p) return h->fail(KC_EINVAL, "points: NULL");
    if (!p->f32) return h->fail(KC_EINVAL, "points: f32 is NULL");
    if (p->n < 1 || p->n >= (int64_t)0xFFFFFFFFll)
        return h->fail(KC_EINVAL, "points: n=%lld out of range", (long long)p->n);
    if (p->d < 1 || p->d > KC_MAXD)
        return h->fail(KC_EINVAL, "points: d=%d out of range [1,%d]", p->d, KC_MAXD);
    if (p->ld < p->d) return h->fail(KC_EINVAL, "points: ld < d");
    if (p->prec != KC_FP32 && p->prec != KC_BF16_RESCORE)
        return h->fail(KC_EINVAL, "points: unknown precision %d", p->prec);
    if (need_bf16_if_asked && p->prec == KC_BF16_RESCORE && !p->bf16)
        return h->fail(KC_EINVAL, "points: BF16 precision needs a bf16 copy");
    return KC_OK;
}

// ---------------------------------------------------------------------------
// batched Gonzalez planning

int kc_plan_gon(kc_handle* h, const std::string& pre, int d, uint32_t tile,
                const std::vector<KcGonJob>& jobs, KcGonRun& R, KcGonHost& H, hipStream_t s)
{
    const int nseg = (int)jobs.size();
    H.segs.assign(nseg, KcSeg{});
    H.blk_seg.clear();
    H.blk_start.clear();
    H.pairs_seg.clear();
    H.pairs_t.clear();
    uint64_t base = 0, keyoff = 0, total = 0;
    uint32_t kmax = 0;
    for (int s = 0; s < nseg; ++s) {
        const KcGonJob& j = jobs[s];
        KcSeg& sg = H.segs[s];
        sg.src = j.row0;
        sg.base = base;
        sg.len = j.len;
        sg.first = j.first;
        sg.ksteps = j.len == 0 ? 0 : j.k;
        sg.keyoff = (uint32_t)keyoff;
        for (uint32_t st = 0; st < j.len; st += tile) {
            H.blk_seg.push_back((uint32_t)s);
            H.blk_start.push_back(st);
        }
        for (uint32_t t = 0; t < sg.ksteps; ++t) {
            H.pairs_seg.push_back((uint32_t)s);
            H.pairs_t.push_back(t);
        }
        base += kc_pad64(j.len);
        keyoff += j.k;
        total += j.len;
        kmax = std::max(kmax, sg.ksteps);
    }
    if (keyoff >= 0xFFFFFFFFull) return h->fail(KC_EINVAL, "too many centers in one batch");
    const uint64_t stride = std::max<uint64_t>(base, 64);
    R.d = d;
    R.nseg = nseg;
    R.kmax = kmax;
    R.stride = stride;
    R.nblk = (uint32_t)H.blk_seg.size();
    R.tile = tile;
    R.npairs = (uint32_t)H.pairs_seg.size();
    R.band = 2.0 * kc_gamma32(d) + 4.0 * 5.9604644775390625e-8;
    R.cand_cap = (uint32_t)std::max<uint64_t>(total, 1);
    float* xs = (float*)h->ws(pre + "xs", sizeof(float) * (size_t)d * stride);
    R.xs = xs;
    R.mind = (float*)h->ws(pre + "mind", sizeof(float) * stride);
    R.keys = (u64*)h->ws(pre + "keys", sizeof(u64) * std::max<uint64_t>(keyoff, 1));
    R.part = (u64*)h->ws(pre + "part", sizeof(u64) * KC_PARTS * KC_PSTRIDE *
                                           std::max<uint64_t>(keyoff, 1));
    R.ccoord = (float*)h->ws(pre + "ccoord", sizeof(float) * (size_t)d * std::max<uint64_t>(keyoff, 1));
    R.radius2 = (double*)h->ws(pre + "radius2", sizeof(double) * nseg);
    R.cand = (u64*)h->ws(pre + "cand", sizeof(u64) * R.cand_cap);
    R.ncand = (uint32_t*)h->ws(pre + "ncand", 2 * sizeof(uint32_t));
    R.ticket = R.ncand ? R.ncand + 1 : nullptr;
    if (!R.xs || !R.mind || !R.keys || !R.part || !R.ccoord || !R.radius2 || !R.cand ||
        !R.ncand)
        return h->fail(KC_ENOMEM, "workspace allocation failed");
    R.segs = (KcSeg*)h->upload(pre + "segs", H.segs.data(), sizeof(KcSeg) * nseg, s);
    R.blk_seg = (uint32_t*)h->upload(pre + "blk_seg", H.blk_seg.data(), 4 * H.blk_seg.size(), s);
    R.blk_start = (uint32_t*)h->upload(pre + "blk_start", H.blk_start.data(), 4 * H.blk_start.size(), s);
    R.pairs_seg = (uint32_t*)h->upload(pre + "pairs_seg", H.pairs_seg.data(), 4 * H.pairs_seg.size(), s);
    R.pairs_t = (uint32_t*)h->upload(pre + "pairs_t", H.pairs_t.data(), 4 * H.pairs_t.size(), s);
    if (!R.segs || !R.blk_seg || !R.blk_start || !R.pairs_seg || !R.pairs_t)
        return h->fail(KC_ENOMEM, "plan upload failed");
    R.keysum = keyoff;
    // with segments in descending order of k, the tiles still active at step
    // t form a prefix of the tile list: launch only those
    bool desc = true;
    uint32_t prev = 0xFFFFFFFFu;
    for (int q = 0; q < nseg; ++q) {
        if (H.segs[q].len == 0) continue;   // no tiles
        if (H.segs[q].ksteps > prev) desc = false;
        prev = H.segs[q].ksteps;
    }
    H.nblk_at.clear();
    R.nblk_at = nullptr;
    if (desc && nseg > 1) {
        H.nblk_at.assign(kmax, 0);
        uint32_t b = (uint32_t)H.blk_seg.size();
        for (uint32_t t = 0; t < kmax; ++t) {
            while (b > 0 && H.segs[H.blk_seg[b - 1]].ksteps <= t) --b;
            H.nblk_at[t] = b;
        }
        R.nblk_at = H.nblk_at.data();
    }
    // Segments reading different arrays stage from a table of their sources
    // (one launch for all of them)
    R.srcs = nullptr;
    bool shared = true;
    for (const KcGonJob& j : jobs)
        if (j.X != jobs[0].X || j.Xb != jobs[0].Xb || j.ld != jobs[0].ld) shared = false;
    if (!shared && nseg > 1) {
        std::vector<KcSrc> src(nseg);
        for (int q = 0; q < nseg; ++q) src[q] = KcSrc{jobs[q].X, jobs[q].Xb, jobs[q].ld, 0};
        R.srcs = (const KcSrc*)h->upload(pre + "srcs", src.data(), sizeof(KcSrc) * nseg, s);
        if (!R.srcs) return h->fail(KC_ENOMEM, "plan upload failed");
    }
    // Graphs captured from this plan embed its grids and loop counts (tiles,
    // steps, active tiles per step): their keys carry this signature.
    uint64_t hsh = kc_hash_bytes(&d, sizeof d);
    hsh = kc_hash_bytes(&tile, sizeof tile, hsh);
    hsh = kc_hash_vec(H.segs, hsh);
    hsh = kc_hash_vec(H.nblk_at, hsh);
    R.plan_hash = hsh;
    return KC_OK;
}

// Enqueue the staging of every job with source rows (FP32 SoA copy, plus the
// BF16 copy and rounding radii when xb is given): one launch when all of them
// read the same arrays, else one per job.
void kc_enqueue_stage(const KcGonRun& R, const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                      hipStream_t s, uint16_t* xb, float* ex)
{
    if (R.srcs) {   // segments with their own arrays: one launch from the table
        kc_stage_rows_src(R.srcs, xb != nullptr, R.d, R.segs, R.blk_seg, R.blk_start, R.nblk,
                          R.tile, (float*)R.xs, xb, ex, R.stride, s);
        return;
    }
    bool shared = jobs.size() > 1 && jobs[0].X != nullptr;
    for (const KcGonJob& j : jobs)
        if (j.X != jobs[0].X || j.Xb != jobs[0].Xb || j.ld != jobs[0].ld) shared = false;
    if (shared) {
        kc_stage_rows_batch(jobs[0].X, xb ? jobs[0].Xb : nullptr, jobs[0].ld, R.d, R.segs,
                            R.blk_seg, R.blk_start, R.nblk, R.tile, (float*)R.xs, xb, ex,
                            R.stride, s);
        return;
    }
    for (size_t q = 0; q < jobs.size(); ++q)
        if (jobs[q].X)
            kc_stage_rows(jobs[q].X, xb ? jobs[q].Xb : nullptr, jobs[q].ld, R.d, jobs[q].row0,
                          jobs[q].len, (float*)R.xs, xb, ex, R.stride, H.segs[q].base, s);
}

// Enqueue staging + init of a planned run (streaming engine).
void kc_enqueue_gon_prep(const KcGonRun& R, const KcGonHost& H,
                         const std::vector<KcGonJob>& jobs, hipStream_t s)
{
    kc_enqueue_stage(R, H, jobs, s);
    kc_fill_u32((uint32_t*)R.mind, 0x7F800000u, R.stride, s);   // +inf
    kc_fill_u64(R.part, 0ull, R.keysum * KC_PARTS * KC_PSTRIDE, s);
}

// Enqueue all step launches of a planned run (streaming engine).
void kc_enqueue_gon_steps(const KcGonRun& R, hipStream_t s)
{
    for (uint32_t t = 0; t < R.kmax; ++t) {
        const uint32_t nb = R.nblk_at ? R.nblk_at[t] : R.nblk;
        if (nb > 0)
            kc_gon_step(R.xs, R.stride, R.d, R.mind, R.part, R.segs, R.blk_seg, R.blk_start,
                        nb, (int)t, s);
    }
    kc_part_collect(R.part, R.keys, R.keysum, s);
}

// Prep, steps and finish of a streaming run as three cached graphs; the
// steps graph is bracketed by a timing span called `span`.
int kc_run_gon_stream(kc_handle* h, const std::string& key0, const KcGonRun& R,
                      const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                      const char* span, hipStream_t s,
                      const std::function<void(hipStream_t)>& finish)
{
    const std::string key = key0 + kc_hash_str(R.plan_hash);
    int rc = h->run_graph(key + ":prep", s,
                          [&](hipStream_t st) { kc_enqueue_gon_prep(R, H, jobs, st); });
    if (rc) return rc;
    hipEvent_t ev = h->span_begin(s);
    rc = h->run_graph(key + ":steps", s, [&](hipStream_t st) { kc_enqueue_gon_steps(R, st); });
    h->span_end(span, ev, R.kmax, s);
    if (rc) return rc;
    return h->run_graph(key + ":finish", s, finish);
}

// A planned FP32 run on the resident engine when every segment fits a
// co-resident grid (option "resident"), else on the streaming engine; then
// `finish`.
int kc_run_gon(kc_handle* h, const std::string& key, const KcGonRun& R, const KcGonHost& H,
               const std::vector<KcGonJob>& jobs, const char* span, hipStream_t s,
               const std::function<void(hipStream_t)>& finish)
{
    bool done = false;
    if (h->allow_resident) {
        const int rc = kc_run_gon_resident_batch(h, key, R, H, jobs, span, s, &done);
        if (rc) return rc;
    }
    if (done) return h->run_graph(key + kc_hash_str(R.plan_hash) + ":rfinish", s, finish);
    return kc_run_gon_stream(h, key, R, H, jobs, span, s, finish);
}

int kc_run_gon_resident_batch(kc_handle* h, const std::string& key0, const KcGonRun& R,
                              const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                              const char* span, hipStream_t s, bool* done)
{
    *done = false;
    const std::string key = key0 + kc_hash_str(R.plan_hash);
    const int d = R.d;
    // Two packings: every segment on the first variant whose grid for it is
    // co-resident, or every segment on the large variant (fewer blocks, so
    // fewer launches, at more arithmetic per step).  The one with the lower
    // estimated duration runs.
    struct Launch {
        int v;
        uint32_t G;
        std::vector<uint32_t> segs;
    };
    auto pack = [&](bool large, std::vector<Launch>& out) -> bool {
        struct Item {
            uint32_t seg, G;
        };
        std::vector<Item> items[2];
        out.clear();
        for (size_t q = 0; q < H.segs.size(); ++q) {
            const KcSeg& sg = H.segs[q];
            if (sg.len == 0 || sg.ksteps == 0) continue;   // nothing to choose
            int v = 1;
            uint32_t G = kc_resident_blocks_for(d, 1, sg.len);
            if (!large && !h->resident_fit(d, sg.len, &v, &G)) return false;
            if (large && (G == 0 || (int64_t)G > (int64_t)h->resident_max(d, 1))) return false;
            items[v].push_back({(uint32_t)q, G});
        }
        // first-fit decreasing into launches of at most gmax blocks; the
        // blocks of a segment are consecutive in its launch
        for (int v = 0; v < 2; ++v) {
            const uint32_t gmax = items[v].empty() ? 0u : (uint32_t)h->resident_max(d, v);
            std::stable_sort(items[v].begin(), items[v].end(),
                             [](const Item& a, const Item& b) { return a.G > b.G; });
            const size_t l0 = out.size();
            for (const Item& it : items[v]) {
                size_t l = l0;
                while (l < out.size() && out[l].G + it.G > gmax) ++l;
                if (l == out.size()) out.push_back({v, 0, {}});
                out[l].G += it.G;
                out[l].segs.push_back(it.seg);
            }
        }
        return true;
    };
    auto cost = [&](const std::vector<Launch>& L) {
        double c = 0;
        for (const Launch& x : L) c += kc_resident_launch_cycles(d, x.v, R.kmax);
        return c;
    };
    std::vector<Launch> launches, alt;
    const bool fit = pack(false, launches);
    if (pack(true, alt) && (!fit || cost(alt) < cost(launches))) launches.swap(alt);
    else if (!fit) return KC_OK;
    if (launches.empty()) return KC_OK;
    std::vector<uint4> tab;
    std::vector<size_t> off;
    for (const Launch& L : launches) {
        off.push_back(tab.size());
        uint32_t b0 = 0;
        for (uint32_t q : L.segs) {
            const uint32_t gs = kc_resident_blocks_for(d, L.v, H.segs[q].len);
            for (uint32_t b = 0; b < gs; ++b) tab.push_back(make_uint4(q, b, gs, b0));
            b0 += gs;
        }
    }
    const uint4* blks =
        (const uint4*)h->upload(key0 + ":rblk", tab.data(), sizeof(uint4) * tab.size(), s);
    // per launch: its exchange words, then its abort flag (one fill clears all)
    const uint64_t bw = kc_resident_slot_words(0, 0) + 8;
    u64* bar = (u64*)h->ws(key0 + ":rbar", sizeof(u64) * bw * launches.size());
    if (!blks || !bar) return h->fail(KC_ENOMEM, "workspace allocation failed");
    // the candidate gathers read the caller's rows when every segment has them
    const float* xa = jobs.empty() ? nullptr : jobs[0].X;
    for (const KcGonJob& j : jobs)
        if (j.X != xa || j.ld != jobs[0].ld) xa = nullptr;
    const int64_t lda = xa ? jobs[0].ld : 0;
    // The points load straight from those rows, with no staging copy, when
    // the caller's finishing pass reads them there too (R.xa) and the
    // kernel's row loads allow them.
    uint64_t rspan = 0;
    for (const KcSeg& sg : H.segs) rspan = std::max<uint64_t>(rspan, sg.len);
    const int rows = xa && R.xa == xa && R.lda == lda && kc_resident_rows_ok(d, xa, lda, rspan);
    int rc = h->run_graph(key + ":rprep", s, [&](hipStream_t st) {
        if (!rows) kc_enqueue_stage(R, H, jobs, st);
        kc_fill_u64(bar, 0ull, bw * launches.size(), st);
    });
    if (rc) return rc;
    hipEvent_t ev = h->span_begin(s);
    for (size_t l = 0; l < launches.size(); ++l) {
        const Launch& L = launches[l];
        u64* slots = bar + bw * l;
        uint32_t* abort_flag = (uint32_t*)(slots + (bw - 8));
        hipError_t e = kc_gon_resident(d, L.v, L.G, R.xs, R.stride, 0, 0, nullptr, 0, 0, R.mind,
                                       R.keys, slots, abort_flag, h->spin_limit, xa, lda, rows,
                                       h->status_word, R.segs, blks + off[l], s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (l == 0) {   // refused before any work: the caller streams
                if (ev) h->event_pool.push_back(ev);
                return KC_OK;
            }
            return h->fail(KC_EHIP, "resident launch %zu: %s", l, hipGetErrorString(e));
        }
    }
    h->span_end(span, ev, (int64_t)launches.size(), s);
    *done = true;
    return KC_OK;
}

// ---------------------------------------------------------------------------
// public entry points

// Option "validate": any non-finite coordinate of the n x d points (FP32,
// and the BF16 copy when one is given) sets KC_STATUS_NONFINITE in the
// device status word.  Rows are walked with a grid stride; a contiguous
// array is read in memory order.
__global__ __launch_bounds__(256) void k_check_finite(const float* __restrict__ X,
                                                      const uint16_t* __restrict__ Xb,
                                                      int64_t ld, int d, uint64_t n,
                                                      uint32_t* __restrict__ status)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    if (ld == d) {
        const uint64_t total = n * (uint64_t)d;
        for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total; e += stride) {
            bad |= (__float_as_uint(X[e]) & 0x7F800000u) == 0x7F800000u;
            if (Xb) bad |= (Xb[e] & 0x7F80u) == 0x7F80u;
        }
    } else {
        for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride)
            for (int j = 0; j < d; ++j) {
                const uint64_t at = i * (uint64_t)ld + j;
                bad |= (__float_as_uint(X[at]) & 0x7F800000u) == 0x7F800000u;
                if (Xb) bad |= (Xb[at] & 0x7F80u) == 0x7F80u;
            }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, KC_STATUS_NONFINITE);
}

void kc_validate_points(kc_handle* h, const kc_points* p, hipStream_t s)
{
    if (!h->validate) return;
    const uint64_t work = p->ld == p->d ? (uint64_t)p->n * p->d : (uint64_t)p->n;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(2048, (work + 255) / 256);
    hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, s, p->f32,
                       p->prec == KC_BF16_RESCORE ? p->bf16 : nullptr, p->ld, p->d,
                       (uint64_t)p->n, h->status_word);
}

extern "C" {

int kc_create(kc_handle** out)
{
    if (!out) return KC_EINVAL;
    *out = nullptr;
    kc_handle* h = new (std::nothrow) kc_handle();
    if (!h) return KC_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device) !=
            hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return KC_EHIP;
    }
    if (hipMalloc(&h->status_word, 256) != hipSuccess ||
        hipMemset(h->status_word, 0, 256) != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return KC_ENOMEM;
    }
    // the no-allocation entry point's array on this device
    if (kc_noalloc_setup(h->device, &h->scratch) != hipSuccess) {
        delete h;
        return KC_EHIP;
    }
    *out = h;
    return KC_OK;
}

void kc_destroy(kc_handle* h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();   // nothing queued may still use its buffers
    delete h;
}

const char* kc_strerror(int status)
{
    switch (status) {
    case KC_OK: return "ok";
    case KC_EINVAL: return "invalid argument";
    case KC_ENOMEM: return "out of device memory";
    case KC_EHIP: return "HIP runtime error";
    case KC_ENOCONV: return "EIM did not converge within max_iters";
    case KC_EUNSUPPORTED: return "unsupported request";
    case KC_EDEVICE: return "device-side check failed";
    default: return "unknown status";
    }
}

const char* kc_last_error(const kc_handle* h)
{
    return h ? h->last_error.c_str() : "NULL handle";
}

int kc_set_option(kc_handle* h, const char* name, int64_t value)
{
    if (!h || !name) return KC_EINVAL;
    if (!strcmp(name, "graphs")) {
        h->use_graphs = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "resident")) {
        h->allow_resident = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "mfma_split")) {
        h->mfma_split = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "autotune")) {
        h->autotune = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "validate")) {
        if (value != 0 && value != 1) return h->fail(KC_EINVAL, "validate must be 0 or 1");
        h->validate = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "tune_force")) {
        if (value < -1 || value > 63) return h->fail(KC_EINVAL, "tune_force range");
        h->tune_force = (int)value;
        return KC_OK;
    }
    if (!strcmp(name, "timing")) {
        h->timing = value != 0;
        return KC_OK;
    }
    if (!strcmp(name, "resident_blocks")) {
        if (value < 0 || value > 0x7FFFFFFF) return h->fail(KC_EINVAL, "resident_blocks range");
        h->resident_cap = (int)value;
        return KC_OK;
    }
    if (!strcmp(name, "spin_limit")) {
        if (value < 1 || value > 0x7FFFFFFF) return h->fail(KC_EINVAL, "spin_limit range");
        h->spin_limit = (uint32_t)value;
        return KC_OK;
    }
    return h->fail(KC_EINVAL, "unknown option '%s'", name);
}

int kc_tune_report(kc_handle* h, char* buf, int64_t cap, int64_t* need)
{
    if (!h || !need || cap < 0 || (cap > 0 && !buf)) return KC_EINVAL;
    std::string out;
    char num[32];
    for (auto& kv : h->tuned) {
        out += kv.first;
        snprintf(num, sizeof num, " %d", kv.second);
        out += num;
        auto it = h->tune_ms.find(kv.first);
        if (it != h->tune_ms.end())
            for (float t : it->second) {
                snprintf(num, sizeof num, " %.4f", (double)t);
                out += num;
            }
        out += '\n';
    }
    *need = (int64_t)out.size() + 1;
    if (cap == 0) return KC_OK;   // a size query
    if (cap < *need) return h->fail(KC_EINVAL, "tune report needs %lld bytes", (long long)*need);
    memcpy(buf, out.c_str(), out.size() + 1);
    return KC_OK;
}

int kc_timing_read(kc_handle* h, const char* name, double* ms, int64_t* launches,
                   int64_t* intervals)
{
    if (!h || !name || !ms || !launches || !intervals) return KC_EINVAL;
    *ms = 0.0;
    *launches = 0;
    *intervals = 0;
    auto it = h->spans.find(name);
    if (it == h->spans.end()) return KC_OK;
    if (hipDeviceSynchronize() != hipSuccess) {
        hipError_t e = hipGetLastError();
        return h->fail(KC_EHIP, "timing sync: %s", hipGetErrorString(e));
    }
    for (auto& sp : it->second) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, sp.a, sp.b) == hipSuccess) {
            *ms += t;
            *launches += sp.launches;
            *intervals += 1;
        } else {
            (void)hipGetLastError();
        }
        h->event_pool.push_back(sp.a);
        h->event_pool.push_back(sp.b);
    }
    h->spans.erase(it);
    return KC_OK;
}

int kc_counter_read(kc_handle* h, const char* name, int64_t* value)
{
    if (!h || !name || !value) return KC_EINVAL;
    const uint32_t* src = nullptr;
    size_t words = h->last_bf16_kmax, every = 1;
    if (!strcmp(name, "bf16_listed")) {
        src = h->last_bf16_listcnt;   // [kmax][KC_PARTS][32]: one count per line
        words *= KC_PARTS * 32;
        every = 32;
    } else if (!strcmp(name, "bf16_rescored")) {
        src = h->last_bf16_nresc;
    } else if (!strcmp(name, "eim_exact")) {
        *value = h->eim_exact;
        return KC_OK;
    } else if (!strcmp(name, "eim_refined")) {
        *value = h->eim_refined;
        return KC_OK;
    } else if (!strcmp(name, "resident_integer")) {
        src = h->status_word + 2;   // counted by the resident kernels
        words = 1;
    } else if (!strcmp(name, "assign_rescored")) {
        src = h->last_assign_nlist;   // one count
        words = 1;
    } else {
        return h->fail(KC_EINVAL, "unknown counter '%s'", name);
    }
    *value = 0;
    if (!src || words == 0) return KC_OK;
    std::vector<uint32_t> v(words);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(v.data(), src, 4 * v.size(), hipMemcpyDeviceToHost) != hipSuccess) {
        hipError_t e = hipGetLastError();
        return h->fail(KC_EHIP, "counter read: %s", hipGetErrorString(e));
    }
    for (size_t i = 0; i < words; i += every) *value += v[i];
    return KC_OK;
}

int kc_device_status(kc_handle* h, void* stream, uint32_t* status)
{
    if (!h || !status) return KC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    uint32_t w[2] = {0, 0};
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(w, h->status_word, 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(h->status_word, 0, 256) != hipSuccess) {
        hipError_t e = hipGetLastError();
        return h->fail(KC_EHIP, "status: %s", hipGetErrorString(e));
    }
    *status = w[0] | w[1];
    return *status ? h->fail(KC_EDEVICE, "device status 0x%x", *status) : KC_OK;
}

int kcenter_gonzalez(kc_handle* h, const kc_points* pts, int64_t k, int64_t first,
                     int64_t* centers, double* radius_trace, int64_t* n_chosen, void* stream)
{
    if (!h) return KC_EINVAL;
    int rc = kc_check_points(h, pts, true);
    if (rc) return rc;
    if (k < 1 || k >= (int64_t)0x7FFFFFFF) return h->fail(KC_EINVAL, "k=%lld", (long long)k);
    if (first < 0 || first >= pts->n) return h->fail(KC_EINVAL, "first out of range");
    if (!centers || !n_chosen) return h->fail(KC_EINVAL, "centers/n_chosen NULL");
    hipStream_t s = (hipStream_t)stream;
    kc_validate_points(h, pts, s);
    if (pts->prec == KC_BF16_RESCORE)
        return kc_gonzalez_bf16(h, pts, k, first, centers, radius_trace, n_chosen, s);

    std::vector<KcGonJob> jobs(1);
    jobs[0] = KcGonJob{pts->f32, pts->ld, 0, (uint32_t)pts->n, (uint32_t)first, (uint32_t)k};
    KcGonRun R;
    KcGonHost H;
    rc = kc_plan_gon(h, "g.", pts->d, 1024, jobs, R, H, s);
    if (rc) return rc;

    // Engines: the register-resident persistent kernel in either variant
    // when the points fit its co-resident grid, the streaming steps, or one
    // workgroup when the points fit its lanes; the autotuner measures the
    // feasible ones once per shape bucket.
    char key[256];
    snprintf(key, sizeof key, "gon:%p:%lld:%d:%lld:%lld:%lld:%p:%p:%p", (const void*)pts->f32,
             (long long)pts->n, pts->d, (long long)pts->ld, (long long)k, (long long)first,
             (void*)centers, (void*)radius_trace, (void*)n_chosen);
    auto stream_run = [&]() {
        return kc_run_gon_stream(h, key, R, H, jobs, "gon_step", s, [&](hipStream_t st) {
            kc_gon_finish(R, centers, n_chosen, radius_trace, nullptr, nullptr, nullptr, st);
        });
    };
    const int rows = kc_resident_rows_ok(pts->d, pts->f32, pts->ld, (uint64_t)pts->n);
    auto run = [&](int var) -> int {
        if (var == 2) return stream_run();
        if (var == 3) {   // one workgroup: small inputs
            R.xa = pts->f32;
            R.lda = pts->ld;
            hipEvent_t ev = h->span_begin(s);
            hipError_t e = kc_gon_block(pts->d, pts->f32, pts->ld, (uint32_t)pts->n,
                                        (uint32_t)first, (int)k, R.mind, R.keys, s);
            h->span_end("gon_block", ev, 1, s);
            if (e != hipSuccess)
                return h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
            kc_gon_finish(R, centers, n_chosen, radius_trace, nullptr, nullptr, nullptr, s);
            e = hipGetLastError();
            return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
        }
        const uint32_t G = kc_resident_blocks_for(pts->d, var, (uint64_t)pts->n);
        // exchange words, then the abort flag: one fill clears both.  The
        // kernel writes every min-distance and every key (zeros past an early
        // stop); candidate and center gathers read the caller's rows.
        const uint64_t bw = kc_resident_slot_words((int)k, G);
        u64* bar = (u64*)h->ws("g.bar", sizeof(u64) * (bw + 8));
        if (!bar) return h->fail(KC_ENOMEM, "workspace allocation failed");
        uint32_t* abort_flag = (uint32_t*)(bar + bw);
        // points straight from the caller's rows when the kernel's row loads
        // allow them, else from the SoA staging copy
        if (!rows)
            kc_stage_soa(pts->f32, pts->ld, pts->d, 0, (uint32_t)pts->n, (float*)R.xs, R.stride,
                         0, s);
        kc_fill_u64(bar, 0ull, bw + 1, s);
        R.xa = pts->f32;
        R.lda = pts->ld;
        hipEvent_t ev = h->span_begin(s);
        hipError_t e = kc_gon_resident(pts->d, var, G, R.xs, R.stride, 0, (uint32_t)pts->n,
                                       nullptr, (uint32_t)first, (int)k, R.mind, R.keys, bar,
                                       abort_flag, h->spin_limit, pts->f32, pts->ld, rows,
                                       h->status_word, nullptr, nullptr, s);
        h->span_end("gon_resident", ev, 1, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();   // not co-resident: stream instead
            return stream_run();
        }
        kc_gon_finish(R, centers, n_chosen, radius_trace, nullptr, nullptr, nullptr, s);
        e = hipGetLastError();
        return e == hipSuccess ? KC_OK : h->fail(KC_EHIP, "launch: %s", hipGetErrorString(e));
    };
    // (the one-workgroup engine is register-resident too: option resident)
    bool feas[4] = {false, false, true,
                    h->allow_resident && kc_gon_block_fits(pts->d, (uint64_t)pts->n)};
    for (int v = 0; v < 2; ++v) {
        const uint32_t G = kc_resident_blocks_for(pts->d, v, (uint64_t)pts->n);
        feas[v] = h->allow_resident && G > 0 && (int64_t)G <= (int64_t)h->resident_max(pts->d, v);
    }
    char tkey[96];
    snprintf(tkey, sizeof tkey, "gon/%d/%d/%d/%d", pts->d, (int)floor(2.0 * log2((double)pts->n)),
             (int)floor(2.0 * log2((double)k)), rows);
    return h->tune(tkey, 4, feas, s, run);
}

}  // extern "C"

int kc_handle::resident_max(int d, int v)
{
    const int key = d * 2 + v;
    int g;
    auto it = resident_cache.find(key);
    if (it != resident_cache.end()) {
        g = it->second;
    } else {
        g = kc_resident_max_blocks(d, v);
        resident_cache[key] = g;
    }
    return resident_cap > 0 ? std::min(g, resident_cap) : g;
}

bool kc_handle::resident_fit(int d, uint64_t len, int* v, uint32_t* G)
{
    for (int q = 0; q < 2; ++q) {
        const uint32_t g = kc_resident_blocks_for(d, q, len);
        if (g > 0 && (int64_t)g <= (int64_t)resident_max(d, q)) {
            *v = q;
            *G = g;
            return true;
        }
    }
    return false;
}
