/*
 * kc_oracle.c -- plain, slow FP64 reference for the k-center hot path of
 * McClintock & Wirth, "Efficient Parallel Algorithms for k-Center Clustering"
 * (arXiv 1604.03228).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library, and the library never calls it.
 *
 * Every point arrives as FP32 and is promoted exactly to FP64.  All
 * arithmetic is FP64.  The squared distance is
 *     D(i, j) = sum_{t = 0 .. d-1} (x_it - x_jt)^2
 * summed in ascending t, each square and each addition rounded separately
 * (build with -ffp-contract=off).  Comparisons are made on squared
 * distances; sqrt is taken only for reported radii (Section 7.2: Euclidean
 * distance computed from coordinates as needed).  Ties between equally far
 * points go to the lowest point index; ties between equally near centers go
 * to the lowest center position.
 *
 * Functions and the passages they follow:
 *   orc_gon          Gonzalez's farthest-first traversal, Section 3.1.
 *   orc_gon_replay   the same traversal, forced along a given sequence,
 *                    checking each forced choice is a farthest point up to a
 *                    relative band (used to accept certified FP32 ties).
 *   orc_gon_resume   the traversal with its first p centers given (a saved
 *                    prefix), continued by farthest points to k centers;
 *                    Section 3.1's traversal adds one center per step from
 *                    the current set alone, so a prefix of a run extends to
 *                    the longer run.
 *   orc_assign       nearest-center assignment and covering radius, the
 *                    k-center definition in Section 1.1.
 *   orc_mrg          two-round MRG, Algorithm 1 with one pass of its loop.
 *   orc_mrg_rounds   Algorithm 1 with its while loop (Lemma 3, Eq. 1).
 *   orc_eim          EIM-MapReduce-Sample (Algorithm 2) with Select
 *                    (Algorithm 3) and the Section 4.1 changes, then Gonzalez
 *                    on the sample.
 *   orc_philox4x64_10  counter-based generator (Salmon et al., SC'11) that
 *                    draws EIM's Bernoulli samples.
 *   orc_opt_bruteforce exact optimum radius by enumeration (tiny inputs).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

/* Threads used by the per-point loops (the arithmetic per point does not
 * depend on it).  Returns the count actually in force. */
int orc_set_threads(int t)
{
    if (t < 1) t = 1;
#ifdef _OPENMP
    g_threads = t;
#else
    g_threads = 1;
#endif
    return g_threads;
}

/* Squared Euclidean distance between rows a and b of two FP32 arrays. */
static double dist2(const float *a, const float *b, int d)
{
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = (double)a[t] - (double)b[t];
        double sq = diff * diff;
        s = s + sq;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Gonzalez (Section 3.1): the first center is given; every later center is
 * a point farthest from the centers chosen so far.  mind[i] holds the squared
 * distance of point i to its nearest chosen center.
 *
 * X        [n][ld] FP32, row-major; only the first d columns are read.
 * centers  out [k]: chosen point indices in selection order (-1 padded).
 * trace    out [k]: trace[t] = covering radius with centers c_0..c_t
 *          (Euclidean); 0 after an early stop.
 * mind_out optional out [n]: final squared distance to the nearest center.
 * Returns the number of centers chosen: k, or fewer when every point already
 * coincides with a center (the problem asks for at most k centers). */
int64_t orc_gon(const float *X, int64_t n, int d, int64_t ld, int64_t k,
                int64_t first, int64_t *centers, double *trace,
                double *mind_out)
{
    double *mind = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!mind) return -1;
    for (int64_t i = 0; i < n; ++i) mind[i] = INFINITY;
    for (int64_t t = 0; t < k; ++t) { centers[t] = -1; trace[t] = 0.0; }

    int64_t c = first;
    int64_t chosen = 0;
    for (int64_t t = 0; t < k; ++t) {
        centers[t] = c;
        chosen = t + 1;
        const float *xc = X + c * ld;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double dd = dist2(X + i * ld, xc, d);
            if (dd < mind[i]) mind[i] = dd;
        }
        double M = -1.0;
        int64_t a = -1;
        for (int64_t i = 0; i < n; ++i)
            if (mind[i] > M) { M = mind[i]; a = i; }
        trace[t] = sqrt(M);
        if (M == 0.0) break;   /* every point is a center already */
        c = a;
    }
    if (mind_out) memcpy(mind_out, mind, sizeof(double) * (size_t)n);
    free(mind);
    return chosen;
}

/* Gonzalez forced along seq[0..nseq-1] (seq[0] is the first center).
 * At each step t < nseq-1 the forced next center g = seq[t+1] must satisfy
 *     band == 0:  g is the farthest point with the lowest index, exactly;
 *     band  > 0:  mind[g] >= M * (1 - band), M the FP64 maximum.
 * The run also checks the stopping rule: the sequence must end exactly when
 * the maximum reaches 0, or at length k.
 * trace out [nseq]: the oracle's covering radius after each step.
 * Returns -1 if the whole sequence is accepted, else the first bad step
 * (nseq if the stopping rule is violated).  *n_ties counts accepted steps
 * where g differs from the oracle's own lowest-index farthest point. */
int64_t orc_gon_replay(const float *X, int64_t n, int d, int64_t ld,
                       int64_t k, const int64_t *seq, int64_t nseq,
                       double band, double *trace, int64_t *n_ties)
{
    *n_ties = 0;
    if (nseq < 1 || nseq > k) return 0;
    for (int64_t t = 0; t < nseq; ++t)
        if (seq[t] < 0 || seq[t] >= n) return t;
    double *mind = (double *)malloc(sizeof(double) * (size_t)n);
    if (!mind) return 0;
    for (int64_t i = 0; i < n; ++i) mind[i] = INFINITY;

    int64_t bad = -1;
    for (int64_t t = 0; t < nseq; ++t) {
        const float *xc = X + seq[t] * ld;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double dd = dist2(X + i * ld, xc, d);
            if (dd < mind[i]) mind[i] = dd;
        }
        double M = -1.0;
        int64_t a = -1;
        for (int64_t i = 0; i < n; ++i)
            if (mind[i] > M) { M = mind[i]; a = i; }
        trace[t] = sqrt(M);
        if (t == nseq - 1) {
            /* sequence ended: legal at length k or when the radius is 0 */
            if (!(nseq == k || M == 0.0)) bad = nseq;
            break;
        }
        if (M == 0.0) { bad = nseq; break; }   /* should have stopped */
        int64_t g = seq[t + 1];
        if (band == 0.0) {
            if (g != a) { bad = t + 1; break; }
        } else {
            if (!(mind[g] > 0.0 && mind[g] >= M * (1.0 - band))) {
                bad = t + 1;
                break;
            }
            if (g != a) ++*n_ties;
        }
    }
    free(mind);
    return bad;
}

/* Gonzalez with a forced prefix (Section 3.1).  Centers c_0..c_{p-1} are
 * prefix[0..p-1]; every later center is a farthest point (lowest index on
 * ties) from the centers so far.  Step t applies c_t to every point's squared
 * min-distance m_i and picks the next center (the forced one while t+1 < p).
 * The forced centers are all kept (a saved prefix is taken as given); the
 * traversal ends after k centers, or at a step t >= p-1 whose farthest
 * point is already at distance 0 from c_0..c_t (every point is covered).
 * trace out [k]: for a step t that is followed by another center,
 *   sqrt(m of that center), its distance to c_0..c_t; for the last chosen
 *   step, sqrt(max_i m_i), the covering radius of all chosen centers; 0
 *   after the end.  Along a free step both readings are the same value.
 * centers out [k] (-1 padded).  Returns the number of centers chosen, or -1
 * when the prefix is invalid (p < 1, p > k, an index out of range). */
int64_t orc_gon_resume(const float *X, int64_t n, int d, int64_t ld, int64_t k,
                       const int64_t *prefix, int64_t p, int64_t *centers,
                       double *trace)
{
    if (p < 1 || p > k) return -1;
    for (int64_t t = 0; t < p; ++t)
        if (prefix[t] < 0 || prefix[t] >= n) return -1;
    double *mind = (double *)malloc(sizeof(double) * (size_t)n);
    if (!mind) return -1;
    for (int64_t i = 0; i < n; ++i) mind[i] = INFINITY;
    for (int64_t t = 0; t < k; ++t) { centers[t] = -1; trace[t] = 0.0; }

    int64_t c = prefix[0];
    int64_t chosen = 0;
    for (int64_t t = 0; t < k; ++t) {
        centers[t] = c;
        chosen = t + 1;
        const float *xc = X + c * ld;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double dd = dist2(X + i * ld, xc, d);
            if (dd < mind[i]) mind[i] = dd;
        }
        double M = -1.0;
        int64_t a = -1;
        for (int64_t i = 0; i < n; ++i)
            if (mind[i] > M) { M = mind[i]; a = i; }
        int64_t next = (t + 1 < p) ? prefix[t + 1] : a;
        if (t == k - 1 || (t + 1 >= p && mind[next] == 0.0)) {
            trace[t] = sqrt(M);   /* covering radius of the chosen centers */
            break;
        }
        trace[t] = sqrt(mind[next]);
        c = next;
    }
    free(mind);
    return chosen;
}

/* ------------------------------------------------------------------------ */
/* Assignment (Section 1.1): every point goes to its nearest center; the
 * solution value is the largest such distance (the covering radius).
 * centers [k] are point indices.  labels out [n]: position j in centers
 * (lowest j among equally near centers).  mind_out optional [n] squared.
 * Returns the Euclidean covering radius. */
double orc_assign(const float *X, int64_t n, int d, int64_t ld,
                  const int64_t *centers, int64_t k, int32_t *labels,
                  double *mind_out)
{
    double R = 0.0;
#pragma omp parallel for num_threads(g_threads) schedule(static) reduction(max : R)
    for (int64_t i = 0; i < n; ++i) {
        double best = INFINITY;
        int32_t bj = -1;
        for (int64_t j = 0; j < k; ++j) {
            double dd = dist2(X + i * ld, X + centers[j] * ld, d);
            if (dd < best) { best = dd; bj = (int32_t)j; }
        }
        if (labels) labels[i] = bj;
        if (mind_out) mind_out[i] = best;
        if (best > R) R = best;
    }
    return sqrt(R);
}

/* Gonzalez on the subset listed (ascending global indices) in idx[0..m-1],
 * first center idx[0].  Centers are returned as global indices.  The subset
 * is gathered into a compact array so that lowest local index means lowest
 * global index. */
static int64_t gon_subset(const float *X, int d, int64_t ld,
                          const int64_t *idx, int64_t m, int64_t k,
                          int64_t *centers, double *trace)
{
    float *Y = (float *)malloc(sizeof(float) * (size_t)(m * d));
    int64_t *loc = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!Y || !loc) { free(Y); free(loc); return -1; }
    for (int64_t i = 0; i < m; ++i)
        memcpy(Y + i * d, X + idx[i] * ld, sizeof(float) * (size_t)d);
    int64_t got = orc_gon(Y, m, d, d, k, 0, loc, trace, NULL);
    for (int64_t t = 0; t < k; ++t)
        centers[t] = (t < got) ? idx[loc[t]] : -1;
    free(Y);
    free(loc);
    return got;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Two-round MRG (Algorithm 1, one pass of its loop; Lemma 2).
 * offsets [m+1]: partition p is the contiguous range [offsets[p],
 *   offsets[p+1]) of X (empty partitions are skipped).
 * Round 1: Gonzalez(k) on each partition, first center = its first point.
 * Union U = ascending global indices of all round-1 centers.
 * Round 2: Gonzalez(k) on U, first center = U[0].
 * Outputs: centers [k] (global, -1 padded), *n_centers; round1 [m*k]
 *   (partition p's centers at p*k, -1 padded), r1 [m] (round-1 covering
 *   radius of each partition, 0 if empty), uni [m*k] and *n_union (U),
 *   *r2 (round-2 radius over U).  Returns the covering radius over all of X
 *   (assignment of every point to its nearest final center). */
double orc_mrg(const float *X, int64_t n, int d, int64_t ld,
               const int64_t *offsets, int m, int64_t k, int64_t *centers,
               int64_t *n_centers, int64_t *round1, double *r1, int64_t *uni,
               int64_t *n_union, double *r2)
{
    double *tr = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t nu = 0;
    for (int p = 0; p < m; ++p) {
        int64_t lo = offsets[p], hi = offsets[p + 1];
        for (int64_t t = 0; t < k; ++t) round1[(int64_t)p * k + t] = -1;
        r1[p] = 0.0;
        if (hi <= lo) continue;
        int64_t got = orc_gon(X + lo * ld, hi - lo, d, ld, k, 0,
                              round1 + (int64_t)p * k, tr, NULL);
        r1[p] = tr[got - 1];
        for (int64_t t = 0; t < got; ++t) {
            round1[(int64_t)p * k + t] += lo;   /* local -> global index */
            uni[nu++] = round1[(int64_t)p * k + t];
        }
    }
    qsort(uni, (size_t)nu, sizeof(int64_t), cmp_i64);
    *n_union = nu;
    int64_t got = gon_subset(X, d, ld, uni, nu, k, centers, tr);
    *n_centers = got;
    *r2 = tr[got - 1];
    free(tr);
    (void)n;
    return orc_assign(X, n, d, ld, centers, got, NULL, NULL);
}

/* Multi-round MRG (Algorithm 1 with its loop; Lemma 3).  While the current
 * sample S holds more than c points, S is split into m_i = ceil(|S| / c)
 * contiguous blocks of its ascending index order (block sizes differ by at
 * most one, so every block fits in capacity c) and Gonzalez(k) runs on each
 * block; S becomes the union of their centers.  Then one machine runs
 * Gonzalez(k) on S (first center = smallest index).
 * *rounds counts all rounds including the last (i+1 in Lemma 3's terms).
 * s_out (optional, [n]) and *n_s_out receive the sample S the last round
 * runs on (ascending).
 * Returns the covering radius over X, or -1 if the loop cannot shrink S
 * (when every block already has at most k points). */
double orc_mrg_rounds(const float *X, int64_t n, int d, int64_t ld,
                      int64_t k, int64_t c, int64_t *centers,
                      int64_t *n_centers, int *rounds, int64_t *s_out,
                      int64_t *n_s_out)
{
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *loc = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    double *tr = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t ns = n;
    for (int64_t i = 0; i < n; ++i) S[i] = i;
    *rounds = 0;
    double result = -1.0;
    while (ns > c) {
        int64_t mi = (ns + c - 1) / c;
        int64_t nt = 0;
        for (int64_t p = 0; p < mi; ++p) {
            int64_t lo = p * ns / mi, hi = (p + 1) * ns / mi;
            int64_t got = gon_subset(X, d, ld, S + lo, hi - lo, k, loc, tr);
            for (int64_t t = 0; t < got; ++t) T[nt++] = loc[t];
        }
        ++*rounds;
        if (nt >= ns) goto done;   /* no progress: k too close to c */
        qsort(T, (size_t)nt, sizeof(int64_t), cmp_i64);
        memcpy(S, T, sizeof(int64_t) * (size_t)nt);
        ns = nt;
    }
    {
        if (s_out) memcpy(s_out, S, sizeof(int64_t) * (size_t)ns);
        if (n_s_out) *n_s_out = ns;
        int64_t got = gon_subset(X, d, ld, S, ns, k, centers, tr);
        *n_centers = got;
        ++*rounds;
        result = orc_assign(X, n, d, ld, centers, got, NULL, NULL);
    }
done:
    free(S); free(T); free(loc); free(tr);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds. */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, &hi0, &lo0);
        mul128(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* EIM's two uniforms for point x in iteration it: one Philox block with
 * key (seed, 0) and counter (x, it, 0, 0); word 0 drives the draw into S,
 * word 1 the draw into H; each uniform is the top 53 bits times 2^-53. */
static void eim_uniforms(uint64_t seed, int64_t x, int it, double *uS,
                         double *uH)
{
    uint64_t ctr[4] = {(uint64_t)x, (uint64_t)it, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t o[4];
    orc_philox4x64_10(ctr, key, o);
    *uS = (double)(o[0] >> 11) * 0x1.0p-53;
    *uH = (double)(o[1] >> 11) * 0x1.0p-53;
}

/* Per-iteration statistics of orc_eim. */
typedef struct {
    int64_t r_size;    /* |R| at the start of the iteration */
    int64_t ds_size;   /* points drawn into S this iteration */
    int64_t h_size;    /* |H| */
    int64_t s_size;    /* |S| after the draw */
    double tau;        /* squared threshold d(v,S)^2; -inf if none */
    double p_s, p_h;   /* sampling probabilities */
} orc_eim_iter;

static int cmp_desc_f64(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}

/* EIM-MapReduce-Sample (Algorithm 2) with Select (Algorithm 3) and the
 * termination changes of Section 4.1, followed by Gonzalez on the sample.
 *   L = ln n; A_S = 9 k n^eps L; A_H = 4 n^eps L; thr = (4/eps) k n^eps L;
 *   r = ceil(phi L).
 *   while |R| > thr (at most max_iters times):
 *     each x in R joins S with probability min(1, A_S/|R|) and H with
 *     probability min(1, A_H/|R|), independently;
 *     if S is empty nothing is removed;
 *     tau = the min(r,|H|)-th largest d(h,S)^2 over h in H (-inf if H empty);
 *     R keeps x iff x is not in S and d(x,S)^2 > tau (points at distance
 *     equal to d(v,S) leave, and sampled points always leave: Section 4.1).
 *   C = S u R ascending; Gonzalez(C, k) from C[0]; radius over all of X.
 * The mappers' partitions do not affect the result (each draw and each
 * removal decision is per point), so they are not modelled.
 * Outputs: centers [k], *n_centers, sample [n] (C ascending) and *n_sample,
 * the final S and R ([n] each, ascending) with their sizes, iters
 * [max_iters], *n_iters.  Returns the covering radius over X, or -1
 * if R is still above the threshold after max_iters iterations. */
double orc_eim(const float *X, int64_t n, int d, int64_t ld, int64_t k,
               double eps, double phi, uint64_t seed, int max_iters,
               int64_t *centers, int64_t *n_centers, int64_t *sample,
               int64_t *n_sample, int64_t *s_out, int64_t *n_s_out,
               int64_t *r_out, int64_t *n_r_out, orc_eim_iter *iters,
               int *n_iters)
{
    double L = log((double)n);
    double ne = pow((double)n, eps);
    double A_S = 9.0 * (double)k * ne * L;
    double A_H = 4.0 * ne * L;
    double thr = (4.0 / eps) * (double)k * ne * L;
    int64_t r = (int64_t)ceil(phi * L);
    if (r < 1) r = 1;

    int64_t *R = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *H = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    char *inS = (char *)calloc((size_t)n, 1);
    double *dH = (double *)malloc(sizeof(double) * (size_t)n);
    double *tr = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t nr = n, ns = 0;
    for (int64_t i = 0; i < n; ++i) R[i] = i;

    int it = 0;
    double result = -1.0;
    while ((double)nr > thr) {
        if (it >= max_iters) goto done;
        double pS = A_S / (double)nr; if (pS > 1.0) pS = 1.0;
        double pH = A_H / (double)nr; if (pH > 1.0) pH = 1.0;
        int64_t nh = 0, nds = 0;
        for (int64_t j = 0; j < nr; ++j) {
            double uS, uH;
            eim_uniforms(seed, R[j], it, &uS, &uH);
            if (uS < pS) { S[ns++] = R[j]; inS[R[j]] = 1; ++nds; }
            if (uH < pH) H[nh++] = R[j];
        }
        orc_eim_iter *st = &iters[it];
        st->r_size = nr; st->ds_size = nds; st->h_size = nh; st->s_size = ns;
        st->p_s = pS; st->p_h = pH; st->tau = -INFINITY;
        if (ns > 0) {
            /* Select (Algorithm 3): distance of every h in H to S */
            for (int64_t j = 0; j < nh; ++j) {
                double best = INFINITY;
                for (int64_t s = 0; s < ns; ++s) {
                    double dd = dist2(X + H[j] * ld, X + S[s] * ld, d);
                    if (dd < best) best = dd;
                }
                dH[j] = best;
            }
            double tau = -INFINITY;
            if (nh > 0) {
                qsort(dH, (size_t)nh, sizeof(double), cmp_desc_f64);
                int64_t pos = r < nh ? r : nh;
                tau = dH[pos - 1];
            }
            st->tau = tau;
            /* threshold pass (Algorithm 2, removal step) */
            int64_t keep = 0;
            for (int64_t j = 0; j < nr; ++j) {
                int64_t x = R[j];
                if (inS[x]) continue;
                double best = INFINITY;
                for (int64_t s = 0; s < ns; ++s) {
                    double dd = dist2(X + x * ld, X + S[s] * ld, d);
                    if (dd < best) best = dd;
                }
                if (best > tau) R[keep++] = x;
            }
            nr = keep;
        }
        ++it;
    }
    {
        int64_t nc = 0;
        qsort(S, (size_t)ns, sizeof(int64_t), cmp_i64);
        memcpy(s_out, S, sizeof(int64_t) * (size_t)ns);
        memcpy(r_out, R, sizeof(int64_t) * (size_t)nr);
        *n_s_out = ns;
        *n_r_out = nr;
        for (int64_t s = 0; s < ns; ++s) sample[nc++] = S[s];
        for (int64_t j = 0; j < nr; ++j) sample[nc++] = R[j];
        qsort(sample, (size_t)nc, sizeof(int64_t), cmp_i64);
        *n_sample = nc;
        int64_t got = gon_subset(X, d, ld, sample, nc, k, centers, tr);
        *n_centers = got;
        result = orc_assign(X, n, d, ld, centers, got, NULL, NULL);
    }
done:
    *n_iters = it;
    free(R); free(S); free(H); free(inS); free(dH); free(tr);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Exact optimum covering radius (Euclidean) over all center sets of size
 * min(k, n) drawn from the points: enumeration, for n <= 20 only.  A larger
 * set never has a larger radius, so sets of exactly min(k, n) suffice. */
double orc_opt_bruteforce(const float *X, int64_t n, int d, int64_t ld,
                          int64_t k)
{
    if (n < 1 || n > 20 || k < 1) return -1.0;
    int64_t kk = k < n ? k : n;
    int idx[20];
    for (int i = 0; i < kk; ++i) idx[i] = i;
    double best = INFINITY;
    for (;;) {
        double R = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double m = INFINITY;
            for (int j = 0; j < kk; ++j) {
                double dd = dist2(X + i * ld, X + (int64_t)idx[j] * ld, d);
                if (dd < m) m = dd;
            }
            if (m > R) R = m;
        }
        if (R < best) best = R;
        /* next combination in lexicographic order */
        int j = (int)kk - 1;
        while (j >= 0 && idx[j] == (int)(n - kk + j)) --j;
        if (j < 0) break;
        ++idx[j];
        for (int t = j + 1; t < kk; ++t) idx[t] = idx[t - 1] + 1;
    }
    return sqrt(best);
}

/* ------------------------------------------------------------------------ */
/* Single decisions, for checking large runs one output at a time. */

/* EIM's two uniforms for point x in iteration it (see orc_eim). */
void orc_eim_uniform_pair(uint64_t seed, int64_t x, int it, double out[2])
{
    eim_uniforms(seed, x, it, &out[0], &out[1]);
}

/* EIM's draws of one iteration for the listed points R[0..nr-1]: flags[j]
 * bit 0 when R[j] joins S (u_S < pS), bit 1 when it joins H (u_H < pH),
 * with the uniforms of orc_eim_uniform_pair.  Returns the number drawn
 * into S. */
int64_t orc_eim_draw_flags(uint64_t seed, int it, const int64_t *R, int64_t nr,
                           double pS, double pH, uint8_t *flags)
{
    int64_t ns = 0;
    for (int64_t j = 0; j < nr; ++j) {
        double uS, uH;
        eim_uniforms(seed, R[j], it, &uS, &uH);
        flags[j] = (uint8_t)((uS < pS ? 1 : 0) | (uH < pH ? 2 : 0));
        ns += uS < pS;
    }
    return ns;
}

/* min over the listed points s of D(x, s) (squared, FP64) and the lowest
 * list position attaining it; +inf and -1 for an empty list. */
double orc_min_dist2_to_set(const float *X, int d, int64_t ld, int64_t x,
                            const int64_t *set, int64_t nset, int64_t *arg)
{
    double best = INFINITY;
    int64_t a = -1;
    for (int64_t j = 0; j < nset; ++j) {
        double dd = dist2(X + x * ld, X + set[j] * ld, d);
        if (dd < best) { best = dd; a = j; }
    }
    if (arg) *arg = a;
    return best;
}
