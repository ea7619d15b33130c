// kc_host.h -- host-side types of libkcenter (handle, workspace, plans).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdio.h>

#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/kcenter.h"
#include "kc_internal.h"

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Pinned host staging of one uploaded table: the bytes a stream-ordered copy
// reads, and an event recorded after that copy (the staging bytes are not
// rewritten before it has completed).
struct Staging {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

// FNV-1a over bytes, chained through `h` (plan signatures in graph keys).
static inline uint64_t kc_hash_bytes(const void* p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}
template <class T>
static inline uint64_t kc_hash_vec(const std::vector<T>& v, uint64_t h)
{
    const uint64_t n = v.size();
    h = kc_hash_bytes(&n, sizeof n, h);
    return v.empty() ? h : kc_hash_bytes(v.data(), sizeof(T) * v.size(), h);
}
static inline std::string kc_hash_str(uint64_t h)
{
    char b[24];
    snprintf(b, sizeof b, ":#%016llx", (unsigned long long)h);
    return b;
}

struct kc_handle {
    int device = 0;
    int num_cu = 0;
    bool use_graphs = true;
    bool allow_resident = true;
    bool mfma_split = true;           // FP32 distance passes on split BF16 MFMAs
    bool autotune = true;             // measured choice of engine variants
    int tune_force = -1;              // >= 0: always that variant where feasible
    bool validate = false;            // scan inputs for non-finite values
    std::map<std::string, int> tuned;  // key -> chosen variant
    std::map<std::string, std::vector<float>> tune_ms;   // key -> measured ms per variant
    uint32_t spin_limit = 1u << 20;   // polls before a barrier wait gives up
    uint32_t* status_word = nullptr;  // device, see kc_device_status
    void* scratch = nullptr;          // device address of the no-allocation array
    std::string last_error;
    std::map<std::string, DevBuf> bufs;
    std::map<std::string, std::vector<char>> shadows;
    std::map<std::string, void*> shadow_ptr;
    std::map<std::string, Staging> staging;
    std::map<std::string, GraphEntry> graphs;
    size_t graph_cap = 512;           // cached graphs before the cache is cleared (0: no limit)
    std::map<int, int> resident_cache;
    int resident_cap = 0;             // blocks per resident launch, 0: no cap
    bool timing = false;
    struct TimedSpan {
        hipEvent_t a, b;
        int64_t launches;
    };
    std::map<std::string, std::vector<TimedSpan>> spans;
    std::vector<hipEvent_t> event_pool;
    // per-step counters of the most recent BF16 run (device, [kmax])
    const uint32_t* last_bf16_listcnt = nullptr;
    const uint32_t* last_bf16_nresc = nullptr;
    uint32_t last_bf16_kmax = 0;
    // candidates decided by the exact FP64 pass in the most recent EIM call
    int64_t eim_exact = 0;
    // candidates refined in canonical FP32 after an MFMA pass (same call)
    int64_t eim_refined = 0;
    // list count (device) of the most recent assignment's FP64 rescoring
    const uint32_t* last_assign_nlist = nullptr;

    ~kc_handle();
    // Record the opening event of a timed span (no-op unless timing is on).
    hipEvent_t span_begin(hipStream_t s);
    void span_end(const char* name, hipEvent_t a, int64_t launches, hipStream_t s);
    void clear_graphs();
    int fail(int code, const char* fmt, ...);
    void* ws(const std::string& name, size_t bytes);
    // Copy a host table into a named workspace buffer, ordered on stream s
    // after the work already queued there (see kc_api.hip).
    void* upload(const std::string& name, const void* src, size_t bytes, hipStream_t s);
    int run_graph(const std::string& key, hipStream_t stream,
                  const std::function<void(hipStream_t)>& enqueue);
    // Measured choice among variants 0..nvar-1 of one operation that all
    // give the same result (feasible[v] says which may run).  With autotune
    // on and `key` not yet seen, every feasible variant runs twice on `s`,
    // the second run timed between events (the host waits for them), with
    // the timing spans off; the fastest is cached for `key` and runs once
    // more, which gives the call's results and spans.  Otherwise the cached
    // choice runs (or, untuned, the first feasible variant).  Returns
    // run()'s status.
    int tune(const std::string& key, int nvar, const bool* feasible, hipStream_t s,
             const std::function<int(int)>& run);
    // The variant tune() would run for `key` without measuring anything
    // (forced, cached or first feasible; -1 if none is feasible); *measure is
    // set when tune() would measure the variants first.
    int choice(const std::string& key, int nvar, const bool* feasible, hipStream_t s,
               bool* measure);
    // Pinned host memory of at least `bytes` under `name` (hipHostMalloc),
    // for readbacks that several queued copies fill before one wait.
    // Growing it waits for the device first.  NULL on failure.
    void* pinned(const std::string& name, size_t bytes);
    // Co-resident blocks of resident variant v for dimension d (0: none),
    // lowered to resident_cap when that is set.
    int resident_max(int d, int v);
    // The first resident variant whose grid for `len` points is co-resident:
    // sets *v and *G and returns true, or returns false.
    bool resident_fit(int d, uint64_t len, int* v, uint32_t* G);
};

// One segment of a batched Gonzalez run, as the host describes it.
struct KcGonJob {
    const float* X = nullptr;  // source rows (NULL: xs already filled)
    int64_t ld = 0;
    uint64_t row0 = 0;         // first source row
    uint32_t len = 0;
    uint32_t first = 0;        // local index of the first center
    uint32_t k = 0;
    const uint16_t* Xb = nullptr;  // BF16 source rows (BF16 mode)
};

// Host copies of a run's tables.
struct KcGonHost {
    std::vector<KcSeg> segs;
    std::vector<uint32_t> blk_seg, blk_start, pairs_seg, pairs_t;
    std::vector<uint32_t> nblk_at;   // see KcGonRun::nblk_at
};

int kc_check_points(kc_handle* h, const kc_points* p, bool need_bf16_if_asked);
// Device address of the no-allocation scratch array on `device` (current),
// looked up once per device (kc_noalloc.hip).
hipError_t kc_noalloc_setup(int device, void** out);
// Plans a batched run: workspace, and the segment / tile / step tables
// uploaded in order on stream s.  R.plan_hash identifies the plan's geometry
// (every graph key built from a plan includes it).
int kc_plan_gon(kc_handle* h, const std::string& pre, int d, uint32_t tile,
                const std::vector<KcGonJob>& jobs, KcGonRun& R, KcGonHost& H, hipStream_t s);
void kc_enqueue_stage(const KcGonRun& R, const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                      hipStream_t s, uint16_t* xb = nullptr, float* ex = nullptr);
void kc_enqueue_gon_prep(const KcGonRun& R, const KcGonHost& H,
                         const std::vector<KcGonJob>& jobs, hipStream_t s);
void kc_enqueue_gon_steps(const KcGonRun& R, hipStream_t s);
int kc_run_gon_stream(kc_handle* h, const std::string& key, const KcGonRun& R,
                      const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                      const char* span, hipStream_t s,
                      const std::function<void(hipStream_t)>& finish);
// The steps of a planned FP32 run on the resident engine, several segments
// per cooperative launch.  Sets *done when the keys and min-distances are
// enqueued; leaves it false, having enqueued nothing that the streaming
// engine's prep does not redo, when some segment fits no resident grid or
// a launch is refused.
int kc_run_gon(kc_handle* h, const std::string& key, const KcGonRun& R, const KcGonHost& H,
               const std::vector<KcGonJob>& jobs, const char* span, hipStream_t s,
               const std::function<void(hipStream_t)>& finish);
int kc_run_gon_resident_batch(kc_handle* h, const std::string& key, const KcGonRun& R,
                              const KcGonHost& H, const std::vector<KcGonJob>& jobs,
                              const char* span, hipStream_t s, bool* done);
// BF16 stream engine (kc_bf16.hip)
void kc_enqueue_bf16_prep(const KcGonRun& R, const KcBf16Run& B, const KcGonHost& H,
                          const std::vector<KcGonJob>& jobs, hipStream_t s);
void kc_enqueue_bf16_steps(const KcGonRun& R, const KcBf16Run& B, hipStream_t s);
void kc_bf16_finish(const KcGonRun& R, const KcBf16Run& B, int64_t* centers,
                    int64_t* n_chosen, double* trace, double* radius_out,
                    const int64_t* report_base, hipStream_t s);
int kc_bf16_alloc(kc_handle* h, const std::string& pre, const KcGonRun& R, KcBf16Run& B);
int kc_run_bf16(kc_handle* h, const std::string& key, const KcGonRun& R, const KcBf16Run& B,
                const KcGonHost& H, const std::vector<KcGonJob>& jobs, const char* span,
                hipStream_t s, const std::function<void(hipStream_t)>& finish);
int kc_assign_run(kc_handle* h, const kc_points* pts, const int64_t* centers, uint32_t k,
                  const int64_t* k_dev, int32_t* labels, double* radius, hipStream_t s,
                  const std::string& pre);

int kc_gonzalez_bf16(kc_handle* h, const kc_points* pts, int64_t k, int64_t first,
                     int64_t* centers, double* radius_trace, int64_t* n_chosen,
                     hipStream_t s);

// EIM's sampling loops (Algorithm 2 with Select) of the problems probs[ids[q]]
// (arguments checked by the caller), in lockstep: one wait per phase for all
// of them.  On return C[q] (device, in the handle's workspace until its next
// EIM call) holds problem q's sample C = S u R in ascending order and nc[q]
// its size; the handle's eim_exact / eim_refined count over all of them.
// Option "validate": enqueue the non-finite scan of the points (kc_api.hip).
void kc_validate_points(kc_handle* h, const kc_points* p, hipStream_t s);

int kc_eim_sample_many(kc_handle* h, const kc_problem* probs, const std::vector<int>& ids,
                       std::vector<const uint32_t*>& C, std::vector<uint32_t>& nc,
                       hipStream_t s);

// Gonzalez in one workgroup (kc_block.hip): whether d has an instantiation
// and n points fit its lanes; the launch (keys and min-distances as the
// resident engine writes them).
bool kc_gon_block_fits(int d, uint64_t n);
hipError_t kc_gon_block(int d, const float* X, int64_t ld, uint32_t n, uint32_t first, int k,
                        float* mind, u64* keys, hipStream_t s);
