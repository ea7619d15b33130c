// kc_assign.hip -- nearest-center distances on MFMA with certified results.
//
// k_mindist_mfma computes, for every point x and a set of "centers" c_i,
//     v_i = |c_i|^2 - 2 x.c_i        (the dot products on MFMA)
// and keeps per point the smallest v (with its lowest center index) and the
// second smallest; |x|^2 is added afterwards.  The contraction is
//     C (16 centers x K) * X^T (K x 16 points)  -> 16 x 16 accumulators,
// so every lane ends up holding one point and four centers of each tile, and
// the per-point minimum needs one merge over the four lanes sharing a point.
// FP32 inputs use v_mfma_f32_16x16x4f32 (K = 4 per instruction), BF16 inputs
// v_mfma_f32_16x16x32_bf16 (K = 32), both accumulating in FP32.  Centers are
// staged through LDS in chunks; points stream from the caller's array.
//
// Certification (used by the assignment, the covering radius and EIM's
// distance pass), per pair of a point x and a center c, with a = |x| and
// b = |c| of the values fed to the MFMA:
//     |(|x|^2 + v) - D^| <= g (a + b)^2,   g = (6d + 40) u
// where D^ is their exact squared distance, and for BF16 inputs the exact
// distance D of the FP32 points satisfies |sqrt(D) - sqrt(D^)| <= E = e_x +
// e_c (their rounding radii), hence
//     D >= |x|^2 + v - g (a + b)^2 - 2 E (a + b).
// This lower bound is linear in per-center constants, so the kernel keeps,
// per point, the best v with its lowest center index and the smallest lower
// bound over every other center (three FMAs per pair).  A point whose
// smallest other lower bound exceeds the best center's upper bound has a
// certified nearest center; every other point is rescored exactly in FP64.
// Bounds per pair, not through the largest center norm: Gonzalez's centers
// include the data's outliers, whose norms would otherwise swamp the bound
// of every ordinary point.
#include "kc_device.h"
#include "kc_internal.h"

typedef float kc_v4f __attribute__((ext_vector_type(4)));
typedef __bf16 kc_v8bf __attribute__((ext_vector_type(8)));

// Per point and lane: the best v with its center index, the lower-bound
// term w of that center, and the smallest w over every other center (LAB),
// or over all centers (without LAB).
struct KcBest {
    float m1;
    int a1;
    float wb;
    float l2;
};

// Labels pass: push center idx with its v and w.
__device__ __forceinline__ void kc_best_push(KcBest& b, float v, float w, int idx)
{
    // centers arrive in ascending index order per lane: strict < keeps the
    // lower index on ties, and a tied center's w (below its v) then stays in
    // l2, leaving the point uncertified
    if (v < b.m1) {
        b.l2 = fminf(b.l2, b.wb);
        b.m1 = v;
        b.a1 = idx;
        b.wb = w;
    } else {
        b.l2 = fminf(b.l2, w);
    }
}

__device__ __forceinline__ KcBest kc_best_merge(KcBest a, KcBest o)
{
    const bool take_o = (o.m1 < a.m1) || (o.m1 == a.m1 && o.a1 < a.a1);
    KcBest r = take_o ? o : a;
    const float lw = take_o ? a.wb : o.wb;
    r.l2 = fminf(fminf(a.l2, o.l2), lw);
    return r;
}

__device__ __forceinline__ KcBest kc_best_xor(KcBest b, int mask)
{
    KcBest o;
    o.m1 = __shfl_xor(b.m1, mask, 64);
    o.a1 = __shfl_xor(b.a1, mask, 64);
    o.wb = __shfl_xor(b.wb, mask, 64);
    o.l2 = __shfl_xor(b.l2, mask, 64);
    return kc_best_merge(b, o);
}

__device__ __forceinline__ float kc_bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// Waves per block of the distance pass: 4, or 8 (twice the points share
// each LDS copy of a center chunk; for large n).
// Input modes of the distance pass: FP32 on v_mfma_f32_16x16x4f32; BF16
// inputs (the caller's BF16 copy) on v_mfma_f32_16x16x32_bf16; FP32 inputs
// split into BF16 high and low parts, x = h + l + r with h = bf16(x),
// l = bf16(x - h), |r| <= 2^-18 |x|, on three BF16 MFMAs (h.h' + h.l' + l.h').
// The split's products are exact in the FP32 accumulator and the dropped
// terms (l.l', and the r's) are below 3.01 * 2^-18 |x| |c|, so its error
// bound is the FP32 one plus 3.1 * 2^-18 (a + b)^2, at 3/16 of the FP32
// MFMA's issue cost.
// Where 3d is well below 3 * 32 * ceil(d/32), the packed split lays the
// three products along one K range instead: points [h | h | l], centers
// [h' | l' | h'] (each part d long, zero padding after), one MFMA chain of
// ceil(3d/32) K-steps; the products and their count are the split's, so is
// the bound.
#define KC_MD_F32 0
#define KC_MD_BF16 1
#define KC_MD_SPLIT 2
#define KC_MD_SPLITP 3
// Point tiles (16 points each) per wave: four where the B operand is small
// (more independent MFMA chains per center tile, fewer A reads per point),
// two where it would crowd the VGPRs.
__host__ __device__ constexpr int kc_md_pt(int mode, int ks)
{
    return (mode == KC_MD_F32 && ks <= 8) || (mode == KC_MD_SPLITP && ks <= 4) ||
                   (mode != KC_MD_F32 && ks <= 2)
               ? 4
               : 2;
}
// LDS row pitch of a staged center, in elements: the padded K plus 16
// bytes, so the 16 rows one A-operand read touches start in distinct banks.
__host__ __device__ constexpr int kc_md_pitch(int mode, int dp)
{
    return mode == KC_MD_F32 ? dp + 4 : dp + 8;
}

__device__ __forceinline__ float kc_max3(float a, float b, float c)
{
    return fmaxf(fmaxf(a, b), c);
}

__device__ __forceinline__ uint16_t kc_f32_to_bf16_rne(float t)
{
    const uint32_t b = __float_as_uint(t);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// MODE: KC_MD_F32, KC_MD_BF16, KC_MD_SPLIT or KC_MD_SPLITP.  KS: MFMA K-steps (K = 4*KS
// for FP32, 32*KS otherwise).  LAB: labels pass, per point the best center's
// index (arg), its v (m1), its lower-bound term (lob) and the smallest one of
// the other centers (lo2).  Without LAB (a covering radius, a distance to a
// set): with FP32 inputs, bounds of min_j |x|^2 + v_j taken per LDS chunk of
// centers with that chunk's largest |c| -- the smallest v of the chunk
// plus (m1) and minus (lo2) g (a + b_chunk)^2 -- so centers ordered by norm
// give nearly per-center bounds at no cost per pair; with BF16 inputs the
// smallest v (m1).  Always |x|^2 of the values fed to the MFMA (nx; of the
// FP32 values in the split mode).  FP32 inputs with a local origin C.mu have
// it subtracted as they load; the centers come translated.  The passes
// without labels start each MFMA chain from -|c|^2/2 and keep the largest
// -|c|^2/2 + x.c, which is -v/2 (scaling by 2 is exact), so their epilogue
// is one max per output.
template <int MODE, int KS, bool LAB, int W>
__global__ __launch_bounds__(W * 64) void k_mindist_mfma(
    const float* __restrict__ X, const uint16_t* __restrict__ Xb, const float* __restrict__ ex,
    int64_t ld, uint32_t n, int d, float gm, KcCenters C, uint32_t chunk, KcMinOut O,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ n_dev)
{
    constexpr bool BF = MODE != KC_MD_F32;     // BF16 MFMA instructions
    constexpr bool SP = MODE == KC_MD_SPLIT;   // high and low parts
    constexpr bool RB = MODE == KC_MD_BF16;    // inputs carry rounding radii
    constexpr int DP = BF ? KS * 32 : KS * 4;  // padded K
    constexpr int KC_MD_PT = kc_md_pt(MODE, KS);
    constexpr bool CB = !LAB && !RB;            // per-chunk bounds
    constexpr int PITCH = kc_md_pitch(MODE, DP);
    __shared__ float s_bmax;
    extern __shared__ __align__(16) unsigned char kc_smem[];
    float* s_norm = (float*)kc_smem;                          // [chunk] cn
    float* s_cnl = s_norm + chunk;                            // [chunk] cnl
    float* s_len = s_cnl + chunk;                             // [chunk] |c|
    float* s_cer = s_len + chunk;                             // [chunk] e_c (BF16)
    void* s_c = (void*)(s_cer + (RB ? chunk : 0));            // [chunk][DP]
    uint16_t* s_cl = (uint16_t*)s_c + (SP ? (size_t)chunk * PITCH : 0);   // low parts
    const float* __restrict__ Cf = C.mu ? C.Ct : C.Cf;
    const uint16_t* __restrict__ Cb = C.Cb;
    const uint32_t kpad = C.kpad;

    if (n_dev) {   // a device-side count (a pass over listed rows)
        const uint32_t nd = *n_dev;
        n = nd < n ? nd : n;
        if ((uint64_t)blockIdx.x * W * 16 * KC_MD_PT >= n) return;   // the whole block
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const uint64_t p0 =
        ((uint64_t)blockIdx.x * W + wave) * (16 * KC_MD_PT);

    // B operand (points) for all point tiles and K-steps, kept in registers
    float bf[KC_MD_PT][BF ? 1 : KS];
    kc_v8bf bb[KC_MD_PT][BF ? KS : 1];
    kc_v8bf bl[KC_MD_PT][SP ? KS : 1];
    float nxp[KC_MD_PT];
#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        const uint64_t p0r = p0 + pt * 16 + col;
        const bool ok = p0r < n;
        const uint64_t p = (rows && ok) ? (uint64_t)rows[p0r] : p0r;   // the row read
        nxp[pt] = 0.f;
        if (MODE == KC_MD_F32) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int kk = ks * 4 + grp;
                float v = (ok && kk < d) ? X[p * ld + kk] : 0.f;
                if (C.mu && kk < d) v = ok ? v - C.mu[kk] : 0.f;
                bf[pt][BF ? 0 : ks] = v;
                nxp[pt] = __builtin_fmaf(v, v, nxp[pt]);
            }
        } else if (MODE == KC_MD_BF16) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kc_v8bf w;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = ks * 32 + grp * 8 + e;
                    const uint16_t h = (ok && kk < d) ? Xb[p * ld + kk] : (uint16_t)0;
                    const float f = kc_bf16_to_f32(h);
                    w[e] = (__bf16)f;
                    nxp[pt] = __builtin_fmaf(f, f, nxp[pt]);
                }
                bb[pt][BF ? ks : 0] = w;
            }
        } else if (MODE == KC_MD_SPLITP) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kc_v8bf w;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    // packed K position: part 0 and 1 take h, part 2 takes l
                    const int kk = ks * 32 + grp * 8 + e;
                    const int part = kk < d ? 0 : kk < 2 * d ? 1 : kk < 3 * d ? 2 : 3;
                    const int j = kk - part * d;
                    float v = (ok && part < 3) ? X[p * ld + j] : 0.f;
                    if (C.mu && part < 3) v = ok ? v - C.mu[j] : 0.f;
                    if (part == 0) nxp[pt] = __builtin_fmaf(v, v, nxp[pt]);
                    const float fh = kc_bf16_to_f32(kc_f32_to_bf16_rne(v));
                    const float fl = kc_bf16_to_f32(kc_f32_to_bf16_rne(v - fh));
                    w[e] = (__bf16)(part == 2 ? fl : fh);
                }
                bb[pt][ks] = w;
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                kc_v8bf wh, wl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = ks * 32 + grp * 8 + e;
                    float v = (ok && kk < d) ? X[p * ld + kk] : 0.f;
                    if (C.mu && kk < d) v = ok ? v - C.mu[kk] : 0.f;
                    nxp[pt] = __builtin_fmaf(v, v, nxp[pt]);
                    const float fh = kc_bf16_to_f32(kc_f32_to_bf16_rne(v));
                    const float fl = kc_bf16_to_f32(kc_f32_to_bf16_rne(v - fh));
                    wh[e] = (__bf16)fh;   // exact: both are BF16 values
                    wl[e] = (__bf16)fl;
                }
                bb[pt][BF ? ks : 0] = wh;
                bl[pt][SP ? ks : 0] = wl;
            }
        }
    }

    // |x|^2 over the four lane groups, then the point's coefficients of the
    // per-pair lower bound: P1 multiplies |c|, P2 multiplies e_c
    float P1[KC_MD_PT], P2[KC_MD_PT], ap[KC_MD_PT];
    float wt[KC_MD_PT], ut[KC_MD_PT];   // per-chunk bounds: lower and upper terms
#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        float nx = nxp[pt];
        nx += __shfl_xor(nx, 16, 64);
        nx += __shfl_xor(nx, 32, 64);
        nxp[pt] = nx;
        ap[pt] = sqrtf(nx) * (1.f + (float)(d + 4) * 5.9604645e-8f) * (1.f + 1e-6f);
        wt[pt] = __builtin_inff();
        ut[pt] = __builtin_inff();
        if (LAB) {
            const uint64_t p = p0 + pt * 16 + col;
            const float e = (RB && ex && p < n) ? ex[rows ? (uint64_t)rows[p] : p] : 0.f;
            P1[pt] = (2.f * gm * ap[pt] + 2.f * e) * (1.f + 1e-6f);
            P2[pt] = 2.f * ap[pt] * (1.f + 1e-6f);
        }
    }

    KcBest best[KC_MD_PT];
#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        best[pt].m1 = LAB ? __builtin_inff() : -__builtin_inff();
        best[pt].a1 = 0x7FFFFFFF;
        best[pt].wb = __builtin_inff();
        best[pt].l2 = __builtin_inff();
    }

    for (uint32_t c0 = 0; c0 < kpad; c0 += chunk) {
        const uint32_t cn = min(chunk, kpad - c0);
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < cn; q += blockDim.x) {
            s_norm[q] = LAB ? C.cn[c0 + q] : -0.5f * C.cn[c0 + q];
            if (LAB || CB) s_len[q] = C.clen[c0 + q];
            if (LAB) {
                s_cnl[q] = C.cnl[c0 + q];
                if (RB) s_cer[q] = C.cerr[c0 + q];
            }
        }
        if (!BF) {
            const float4* src = (const float4*)(Cf + (uint64_t)c0 * DP);
            float4* dst = (float4*)s_c;
            for (uint32_t q = threadIdx.x; q < cn * DP / 4; q += blockDim.x) {
                const uint32_t r = q / (DP / 4), w = q - r * (DP / 4);
                dst[r * (PITCH / 4) + w] = src[q];
            }
        } else {
            const uint4* src = (const uint4*)(Cb + (uint64_t)c0 * DP);
            uint4* dst = (uint4*)s_c;
            const uint4* srl = (const uint4*)(C.Cbl + (uint64_t)c0 * DP);
            uint4* dsl = (uint4*)s_cl;
            for (uint32_t q = threadIdx.x; q < cn * DP / 8; q += blockDim.x) {
                const uint32_t r = q / (DP / 8), w = q - r * (DP / 8);
                dst[r * (PITCH / 8) + w] = src[q];
                if (SP) dsl[r * (PITCH / 8) + w] = srl[q];
            }
        }
        __syncthreads();
        if (CB) {
            // the chunk's largest |c| (wave 0; read after the next barrier)
            if (wave == 0) {
                float bm = 0.f;
                for (uint32_t q = lane; q < cn; q += 64) bm = fmaxf(bm, s_len[q]);
                for (int off = 32; off >= 1; off >>= 1) bm = fmaxf(bm, __shfl_xor(bm, off, 64));
                if (lane == 0) s_bmax = bm;
            }
            __syncthreads();
        }

        // A operand: centers ct + col, K slice of this lane group.  Two sets
        // of registers take turns: the next tile's operands load into one
        // while the other's MFMAs run (no copies between them)
        float afA[BF ? 1 : KS], afB[BF ? 1 : KS];
        kc_v8bf abA[BF ? KS : 1], abB[BF ? KS : 1];
        kc_v8bf alA[SP ? KS : 1], alB[SP ? KS : 1];
        float4 ncA, ncB;
        auto load_a = [&](uint32_t ct, float* af, kc_v8bf* ab, kc_v8bf* al, float4& nc) {
            if (!BF) {
                const float* cs = (const float*)s_c + (uint64_t)(ct + col) * PITCH;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) af[BF ? 0 : ks] = cs[ks * 4 + grp];
            } else {
                const uint16_t* cs = (const uint16_t*)s_c + (uint64_t)(ct + col) * PITCH;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    ab[BF ? ks : 0] = *(const kc_v8bf*)(cs + ks * 32 + grp * 8);
                if (SP) {
                    const uint16_t* cl = s_cl + (uint64_t)(ct + col) * PITCH;
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks)
                        al[SP ? ks : 0] = *(const kc_v8bf*)(cl + ks * 32 + grp * 8);
                }
            }
            nc = *(const float4*)(s_norm + ct + grp * 4);
        };
        auto tile = [&](uint32_t ct, const float* af, const kc_v8bf* ab, const kc_v8bf* al,
                        const float4 nc4) {
            float4 nl4 = make_float4(0.f, 0.f, 0.f, 0.f), cb4 = nl4, ce4 = nl4;
            if (LAB) {
                nl4 = *(const float4*)(s_cnl + ct + grp * 4);
                cb4 = *(const float4*)(s_len + ct + grp * 4);
                if (RB) ce4 = *(const float4*)(s_cer + ct + grp * 4);
            }
#pragma unroll
            for (int pt = 0; pt < KC_MD_PT; ++pt) {
                kc_v4f acc = {0.f, 0.f, 0.f, 0.f};
                if (!LAB) acc = kc_v4f{nc4.x, nc4.y, nc4.z, nc4.w};   // -|c|^2/2
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    if (!BF) {
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[BF ? 0 : ks],
                                                                   bf[pt][BF ? 0 : ks], acc,
                                                                   0, 0, 0);
                    } else {
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[BF ? ks : 0],
                                                                      bb[pt][BF ? ks : 0],
                                                                      acc, 0, 0, 0);
                        if (SP) {
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                ab[BF ? ks : 0], bl[pt][SP ? ks : 0], acc, 0, 0, 0);
                            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                al[SP ? ks : 0], bb[pt][BF ? ks : 0], acc, 0, 0, 0);
                        }
                    }
                }
                // v = |c|^2 - 2 x.c; labels: w = v - (g b^2 + 2 e_c b) - P1 b
                // - P2 e_c (padding centers have cn = cnl = +inf, so they
                // never count)
                if (LAB) {
                    const int ib = (int)(c0 + ct) + grp * 4;
                    const float q1 = P1[pt], q2 = P2[pt];
                    auto pair = [&](float a, float cnv, float cnlv, float bv, float ev, int idx) {
                        const float v = __builtin_fmaf(-2.f, a, cnv);
                        float w = __builtin_fmaf(-2.f, a, cnlv);
                        w = __builtin_fmaf(-q1, bv, w);
                        if (RB) w = __builtin_fmaf(-q2, ev, w);
                        kc_best_push(best[pt], v, w, idx);
                    };
                    pair(acc[0], nc4.x, nl4.x, cb4.x, ce4.x, ib + 0);
                    pair(acc[1], nc4.y, nl4.y, cb4.y, ce4.y, ib + 1);
                    pair(acc[2], nc4.z, nl4.z, cb4.z, ce4.z, ib + 2);
                    pair(acc[3], nc4.w, nl4.w, cb4.w, ce4.w, ib + 3);
                } else {   // m1 holds the largest -v/2 here
                    best[pt].m1 = kc_max3(kc_max3(best[pt].m1, acc[0], acc[1]), acc[2], acc[3]);
                }
            }
        };
        load_a(0, afA, abA, alA, ncA);
        for (uint32_t ct = 0; ct < cn; ct += 32) {
            if (ct + 16 < cn) load_a(ct + 16, afB, abB, alB, ncB);
            tile(ct, afA, abA, alA, ncA);
            if (ct + 16 >= cn) break;
            if (ct + 32 < cn) load_a(ct + 32, afA, abA, alA, ncA);
            tile(ct + 16, afB, abB, alB, ncB);
        }
        if (CB) {
            // this chunk's bounds: its smallest v -/+ g (a + b_chunk)^2
            const float bc = s_bmax;
#pragma unroll
            for (int pt = 0; pt < KC_MD_PT; ++pt) {
                const float sb = ap[pt] + bc;
                const float e = gm * sb * sb * (1.f + 1e-6f);
                const float m1 = -2.f * best[pt].m1;   // the chunk's smallest v
                wt[pt] = fminf(wt[pt], m1 - e);
                ut[pt] = fminf(ut[pt], m1 + e);
                best[pt].m1 = -__builtin_inff();
            }
        }
    }

#pragma unroll
    for (int pt = 0; pt < KC_MD_PT; ++pt) {
        KcBest b = best[pt];
        if (LAB) {
            b = kc_best_xor(b, 16);
            b = kc_best_xor(b, 32);
        } else if (CB) {
            b.m1 = fminf(ut[pt], __shfl_xor(ut[pt], 16, 64));
            b.m1 = fminf(b.m1, __shfl_xor(b.m1, 32, 64));
            b.l2 = fminf(wt[pt], __shfl_xor(wt[pt], 16, 64));
            b.l2 = fminf(b.l2, __shfl_xor(b.l2, 32, 64));
        } else {
            b.m1 = fmaxf(b.m1, __shfl_xor(b.m1, 16, 64));
            b.m1 = -2.f * fmaxf(b.m1, __shfl_xor(b.m1, 32, 64));
        }
        const uint64_t p = p0 + pt * 16 + col;
        if (grp == 0 && p < n) {
            if (LAB) {
                O.arg[p] = b.a1;
                O.lo2[p] = b.l2;
                O.lob[p] = b.wb;
            }
            if (CB) O.lo2[p] = b.l2;
            O.m1[p] = b.m1;
            O.nx[p] = nxp[pt];
        }
    }
}

// ---------------------------------------------------------------------------
// center staging: compact FP32 / BF16 rows [kpad][DP], norms (+inf padding),
// and the maxima |c| and e_c used by the error bound.

// One thread per center: for many centers (an EIM pass stages its samples),
// where a wave per center would spend most of its time on the reductions.
__global__ void k_stage_centers_thread(const float* __restrict__ X,
                                       const uint16_t* __restrict__ Xb, int64_t ld, int d,
                                       uint32_t n, const int64_t* __restrict__ idx,
                                       const uint32_t* __restrict__ idx32, uint32_t k,
                                       const int64_t* __restrict__ k_dev, KcCenters C,
                                       uint32_t* __restrict__ status)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t kpad = C.kpad;
    const int dp = C.dp;
    if (i >= kpad) return;
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    int64_t ri = 0;
    if (i < k) {
        ri = idx ? idx[i] : (int64_t)idx32[i];
        if (ri < 0 || ri >= (int64_t)n) {   // invalid index: report, stay in bounds
            atomicOr(status, 4u);
            ri = 0;
        }
    }
    if (i >= k) {
        for (int j = 0; j < dp; ++j) {
            if (C.Cf) C.Cf[(uint64_t)i * dp + j] = 0.f;
            if (C.Ct) C.Ct[(uint64_t)i * dp + j] = 0.f;
            if (C.Cb) C.Cb[(uint64_t)i * dp + j] = 0;
            if (C.Cbl) C.Cbl[(uint64_t)i * dp + j] = 0;
        }
        C.cn[i] = __builtin_inff();
        C.cnl[i] = __builtin_inff();
        C.clen[i] = 0.f;
        if (C.cerr) C.cerr[i] = 0.f;
        return;
    }
    const uint64_t r = (uint64_t)ri;
    double nn = 0.0, ee = 0.0, nb = 0.0;
    float nf = 0.f;
    const bool split = C.Cbl != nullptr || C.pk;
    for (int j = 0; j < dp; ++j) {
        const float v = j < d ? X[r * ld + j] : 0.f;
        if (C.Cf) C.Cf[(uint64_t)i * dp + j] = v;
        if (C.Ct) C.Ct[(uint64_t)i * dp + j] = (C.mu && j < d) ? v - C.mu[j] : v;
        if (C.pk) {
            // packed row [h | l | h | 0]: position j takes part j / d of
            // coordinate j mod d
            const int part = j < d ? 0 : j < 2 * d ? 1 : j < 3 * d ? 2 : 3;
            const int jj = j - part * d;
            const float u = part < 3 ? X[r * ld + jj] : 0.f;
            const float t = (C.mu && part < 3) ? u - C.mu[jj] : u;
            const uint16_t hh = kc_f32_to_bf16_rne(t);
            C.Cb[(uint64_t)i * dp + j] =
                part == 1 ? kc_f32_to_bf16_rne(t - kc_bf16_to_f32(hh)) : hh;
            if (part == 0) {
                nf = __builtin_fmaf(t, t, nf);
                nn += (double)t * (double)t;
            }
        } else if (split) {
            // high and low BF16 parts of the translated value
            const float t = (C.mu && j < d) ? v - C.mu[j] : v;
            const uint16_t hh = kc_f32_to_bf16_rne(t);
            C.Cb[(uint64_t)i * dp + j] = hh;
            C.Cbl[(uint64_t)i * dp + j] = kc_f32_to_bf16_rne(t - kc_bf16_to_f32(hh));
            nf = __builtin_fmaf(t, t, nf);
            nn += (double)t * (double)t;
        } else if (C.Cb) {
            const uint16_t h = j < d ? Xb[r * ld + j] : (uint16_t)0;
            C.Cb[(uint64_t)i * dp + j] = h;
            const float f = kc_bf16_to_f32(h);
            nf = __builtin_fmaf(f, f, nf);
            nb += (double)f * (double)f;
            const double e = (double)f - (double)v;
            ee += e * e;
        } else {
            // the value the MFMA pass loads: translated to the local origin
            const float t = (C.mu && j < d) ? v - C.mu[j] : v;
            nf = __builtin_fmaf(t, t, nf);
            nn += (double)t * (double)t;
        }
    }
    // the norm used in v: of the values fed to the MFMA, in FP32 as the
    // kernel's error bound assumes; |c| and e_c rounded up
    const bool bf_in = C.Cb && !split;
    const double b = sqrt(bf_in ? nb : nn) * (1.0 + 1e-6);
    const double e = bf_in ? sqrt(ee) * (1.0 + 1e-6) : 0.0;
    const double g = kc_md_gamma(d, split);
    C.cn[i] = nf;
    C.cnl[i] = (float)((double)nf - (g * b * b + 2.0 * e * b));
    C.clen[i] = (float)b * (1.f + 1e-6f);
    if (C.cerr) C.cerr[i] = (float)e * (1.f + 1e-6f);
    kc_atomic_max_f32_nonneg(&C.cmax[0], (float)b * (1.f + 1e-6f));
    if (bf_in) kc_atomic_max_f32_nonneg(&C.cmax[1], (float)e * (1.f + 1e-6f));
}

// One wave per center: lanes over the row's K positions, the norms reduced
// over the wave (any order: the bounds cover FP32 sums in any order); for
// few centers (an assignment's), where one thread per center would leave
// the launch a handful of long serial loops.
__global__ __launch_bounds__(256) void k_stage_centers(
    const float* __restrict__ X, const uint16_t* __restrict__ Xb, int64_t ld, int d, uint32_t n,
    const int64_t* __restrict__ idx, const uint32_t* __restrict__ idx32, uint32_t k,
    const int64_t* __restrict__ k_dev, KcCenters C, uint32_t* __restrict__ status)
{
    const uint32_t i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t kpad = C.kpad;
    const int dp = C.dp;
    if (i >= kpad) return;   // the whole wave
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    const uint64_t row = (uint64_t)i * dp;
    if (i >= k) {
        for (int j = lane; j < dp; j += 64) {
            if (C.Cf) C.Cf[row + j] = 0.f;
            if (C.Ct) C.Ct[row + j] = 0.f;
            if (C.Cb) C.Cb[row + j] = 0;
            if (C.Cbl) C.Cbl[row + j] = 0;
        }
        if (lane == 0) {
            C.cn[i] = __builtin_inff();
            C.cnl[i] = __builtin_inff();
            C.clen[i] = 0.f;
            if (C.cerr) C.cerr[i] = 0.f;
        }
        return;
    }
    int64_t ri = idx ? idx[i] : (int64_t)idx32[i];
    if (ri < 0 || ri >= (int64_t)n) {   // invalid index: report, stay in bounds
        if (lane == 0) atomicOr(status, 4u);
        ri = 0;
    }
    const uint64_t r = (uint64_t)ri;
    double nn = 0.0, ee = 0.0, nb = 0.0;
    float nf = 0.f;
    const bool split = C.Cbl != nullptr || C.pk;
    for (int j = lane; j < dp; j += 64) {
        const float v = j < d ? X[r * ld + j] : 0.f;
        if (C.Cf) C.Cf[row + j] = v;
        if (C.Ct) C.Ct[row + j] = (C.mu && j < d) ? v - C.mu[j] : v;
        if (C.pk) {
            // packed row [h | l | h | 0]: position j takes part j / d of
            // coordinate j mod d
            const int part = j < d ? 0 : j < 2 * d ? 1 : j < 3 * d ? 2 : 3;
            const int jj = j - part * d;
            const float u = part < 3 ? X[r * ld + jj] : 0.f;
            const float t = (C.mu && part < 3) ? u - C.mu[jj] : u;
            const uint16_t hh = kc_f32_to_bf16_rne(t);
            C.Cb[row + j] = part == 1 ? kc_f32_to_bf16_rne(t - kc_bf16_to_f32(hh)) : hh;
            if (part == 0) {
                nf = __builtin_fmaf(t, t, nf);
                nn += (double)t * (double)t;
            }
        } else if (split) {
            // high and low BF16 parts of the translated value
            const float t = (C.mu && j < d) ? v - C.mu[j] : v;
            const uint16_t hh = kc_f32_to_bf16_rne(t);
            C.Cb[row + j] = hh;
            C.Cbl[row + j] = kc_f32_to_bf16_rne(t - kc_bf16_to_f32(hh));
            nf = __builtin_fmaf(t, t, nf);
            nn += (double)t * (double)t;
        } else if (C.Cb) {
            const uint16_t h = j < d ? Xb[r * ld + j] : (uint16_t)0;
            C.Cb[row + j] = h;
            const float f = kc_bf16_to_f32(h);
            nf = __builtin_fmaf(f, f, nf);
            nb += (double)f * (double)f;
            const double e = (double)f - (double)v;
            ee += e * e;
        } else {
            // the value the MFMA pass loads: translated to the local origin
            const float t = (C.mu && j < d) ? v - C.mu[j] : v;
            nf = __builtin_fmaf(t, t, nf);
            nn += (double)t * (double)t;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        nf += __shfl_xor(nf, off, 64);
        nn += __shfl_xor(nn, off, 64);
        nb += __shfl_xor(nb, off, 64);
        ee += __shfl_xor(ee, off, 64);
    }
    if (lane != 0) return;
    // the norm used in v: of the values fed to the MFMA, in FP32 as the
    // kernel's error bound assumes; |c| and e_c rounded up
    const bool bf_in = C.Cb && !split;
    const double b = sqrt(bf_in ? nb : nn) * (1.0 + 1e-6);
    const double e = bf_in ? sqrt(ee) * (1.0 + 1e-6) : 0.0;
    const double g = kc_md_gamma(d, split);
    C.cn[i] = nf;
    C.cnl[i] = (float)((double)nf - (g * b * b + 2.0 * e * b));
    C.clen[i] = (float)b * (1.f + 1e-6f);
    if (C.cerr) C.cerr[i] = (float)e * (1.f + 1e-6f);
    kc_atomic_max_f32_nonneg(&C.cmax[0], (float)b * (1.f + 1e-6f));
    if (bf_in) kc_atomic_max_f32_nonneg(&C.cmax[1], (float)e * (1.f + 1e-6f));
}

// mu[j] = the median (the lower middle value) of coordinate j over m points
// spread evenly over the n rows: block j ranks its m values by counting.
#define KC_LO_SAMPLE 256
__global__ __launch_bounds__(256) void k_local_origin(const float* __restrict__ X, int64_t ld,
                                                      uint32_t n, float* __restrict__ mu)
{
    __shared__ float sv[KC_LO_SAMPLE];
    const int j = blockIdx.x;
    const uint32_t m = n < KC_LO_SAMPLE ? n : KC_LO_SAMPLE;
    const uint32_t want = (m - 1) / 2;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x)
        sv[i] = X[((uint64_t)i * n / m) * (uint64_t)ld + j];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const float v = sv[i];
        uint32_t below = 0, equal = 0;
        for (uint32_t q = 0; q < m; ++q) {
            below += sv[q] < v;
            equal += sv[q] == v;
        }
        if (below <= want && want < below + equal) mu[j] = v;   // all writers agree
    }
}

// Per-point BF16 rounding radius e_x = |bf16(x) - x| (FP64, rounded up).  A
// block takes 64 points, reads their rows through LDS (consecutive threads
// on consecutive elements, so the reads coalesce), 64 coordinates per pass,
// and thread i sums point i's squared differences in coordinate order.
__global__ __launch_bounds__(256) void k_bf16_err(const float* __restrict__ X,
                                                  const uint16_t* __restrict__ Xb, int64_t ld,
                                                  int d, uint32_t n, float* __restrict__ ex)
{
    __shared__ double se[64][65];
    const uint32_t p0 = blockIdx.x * 64u;
    double acc = 0.0;
    for (int j0 = 0; j0 < d; j0 += 64) {
        const uint32_t w = (uint32_t)min(64, d - j0);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < 64u * w; e += blockDim.x) {
            const uint32_t i = e / w, j = e - i * w;
            double v = 0.0;
            if (p0 + i < n) {
                const uint64_t at = (uint64_t)(p0 + i) * (uint64_t)ld + (uint64_t)(j0 + j);
                v = (double)kc_bf16_to_f32(Xb[at]) - (double)X[at];
                v = v * v;
            }
            se[i][j] = v;
        }
        __syncthreads();
        if (threadIdx.x < 64)
            for (uint32_t j = 0; j < w; ++j) acc += se[threadIdx.x][j];
    }
    if (threadIdx.x < 64 && p0 + threadIdx.x < n)
        ex[p0 + threadIdx.x] = (float)(sqrt(acc) * (1.0 + 1e-12)) * (1.f + 1e-6f);
}

// The same radius for dense rows (ld == d, at most KC_ERR_DENSE_D
// coordinates): a block's 64 rows are one contiguous span of 64 d elements,
// streamed with 16-byte FP32 and 8-byte BF16 loads of 4 elements each (no
// index arithmetic per element).  The squared differences go to LDS in
// element order; then four threads per point sum fixed quarters of its row
// and combine them in a fixed pairing, so the value does not depend on
// scheduling.  The FP64 sum of d <= 96 non-negative terms is within
// 96 * 2^-53 of exact, far inside the 1e-12 rounding-up margin.
#define KC_ERR_DENSE_D 96
__global__ __launch_bounds__(256) void k_bf16_err_dense(const float* __restrict__ X,
                                                        const uint16_t* __restrict__ Xb, int d,
                                                        uint32_t n, float* __restrict__ ex)
{
    extern __shared__ double se_d[];   // 64 * d squared differences, element order
    const uint32_t p0 = blockIdx.x * 64u;
    const uint32_t np = min(64u, n - p0);
    const uint64_t e0 = (uint64_t)p0 * (uint64_t)d;
    const uint32_t ne = np * (uint32_t)d;
    for (uint32_t c = threadIdx.x; c * 4u < ne; c += blockDim.x) {
        const uint32_t e = c * 4u;
        float xv[4];
        uint32_t bv[4];
        if (e + 4u <= ne) {
            const float4 x4 = *(const float4*)(X + e0 + e);
            const uint2 b2 = *(const uint2*)(Xb + e0 + e);
            xv[0] = x4.x;
            xv[1] = x4.y;
            xv[2] = x4.z;
            xv[3] = x4.w;
            bv[0] = b2.x & 0xFFFFu;
            bv[1] = b2.x >> 16;
            bv[2] = b2.y & 0xFFFFu;
            bv[3] = b2.y >> 16;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool in = e + (uint32_t)u < ne;
                xv[u] = in ? X[e0 + e + u] : 0.f;
                bv[u] = in ? (uint32_t)Xb[e0 + e + u] : 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e + (uint32_t)u < ne) {
                const double v = (double)kc_bf16_to_f32((uint16_t)bv[u]) - (double)xv[u];
                se_d[e + u] = v * v;
            }
    }
    __syncthreads();
    const uint32_t i = threadIdx.x >> 2, q = threadIdx.x & 3u;
    const int per = (d + 3) / 4;
    double acc = 0.0;
    if (i < np) {
        const int j0 = (int)q * per, j1 = min(d, j0 + per);
        for (int j = j0; j < j1; ++j) acc += se_d[i * (uint32_t)d + (uint32_t)j];
    }
    acc += __shfl_xor(acc, 1, 64);   // (q0 + q1) and (q2 + q3), the same in both lanes
    acc += __shfl_xor(acc, 2, 64);   // their sum, the same in all four
    if (q == 0 && i < np) ex[p0 + i] = (float)(sqrt(acc) * (1.0 + 1e-12)) * (1.f + 1e-6f);
}

// ---------------------------------------------------------------------------
// assignment epilogue: certify, collect ambiguous points, radius lower bound

// Append `val` to list for every thread whose `pred` holds, one atomic per
// block (hundreds of thousands of appends from every wave of the grid would
// otherwise queue at one word).  Every thread of the block must call it.
__device__ __forceinline__ void kc_block_append(bool pred, uint32_t val, uint32_t* list,
                                                uint32_t* nlist)
{
    __shared__ uint32_t s_cnt[16];
    __shared__ uint32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 b = __ballot(pred);
    if (lane == 0) s_cnt[wave] = (uint32_t)__builtin_popcountll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_cnt[w];
        s_base = tot ? atomicAdd(nlist, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = s_base;
    for (int w = 0; w < wave; ++w) off += s_cnt[w];
    if (pred) list[off + (uint32_t)__builtin_popcountll(b & ((1ull << lane) - 1ull))] = val;
}

// kc_block_append for PP values per thread: one atomic per block for all of
// them.  Every thread of the block must call it.
template <int PP>
__device__ __forceinline__ void kc_block_append_pp(const bool (&pred)[PP],
                                                   const uint32_t (&val)[PP], uint32_t* list,
                                                   uint32_t* nlist)
{
    __shared__ uint32_t s_cnt[PP][16];
    __shared__ uint32_t s_base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    u64 b[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        b[q] = __ballot(pred[q]);
        if (lane == 0) s_cnt[q][wave] = (uint32_t)__builtin_popcountll(b[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int q = 0; q < PP; ++q)
            for (int w = 0; w < nw; ++w) tot += s_cnt[q][w];
        s_base = tot ? atomicAdd(nlist, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = s_base;   // values in order (q, wave, lane)
#pragma unroll
    for (int q = 0; q < PP; ++q) {
        uint32_t o = off;
        for (int w = 0; w < nw; ++w) {
            if (w < wave) o += s_cnt[q][w];
            off += s_cnt[q][w];
        }
        if (pred[q]) list[o + (uint32_t)__builtin_popcountll(b[q] & ((1ull << lane) - 1ull))] = val[q];
    }
}

// With labels == NULL only the radius is wanted: an ambiguous point matters
// only if its upper bound reaches the largest lower bound, and
// k_radius_candidates lists exactly those, so ambiguity lists nothing.
#define KC_EPI_PP 4
__global__ __launch_bounds__(256) void k_assign_epilogue(uint32_t n, int d, KcMinOut O,
                                                         const float* __restrict__ ex,
                                  KcCenters C, int32_t* __restrict__ labels,
                                  float* __restrict__ hi_out, uint32_t* __restrict__ list,
                                  uint32_t* __restrict__ nlist, float* __restrict__ lo_max)
{
    // KC_EPI_PP points per thread, so that a block appends its ambiguous
    // points with one atomic for KC_EPI_PP * 256 points (hundreds of
    // thousands of them in a BF16 pass queue at that one word)
    bool amb[KC_EPI_PP];
    uint32_t pv[KC_EPI_PP];
    float lo_f = 0.f;
#pragma unroll
    for (int q = 0; q < KC_EPI_PP; ++q) {
        const uint32_t p = (blockIdx.x * KC_EPI_PP + q) * blockDim.x + threadIdx.x;
        amb[q] = false;
        pv[q] = p;
        if (p < n) {
            const KcMdBounds B = kc_md_bounds(O, p, ex, C, d, labels != nullptr);
            if (labels) {
                amb[q] = !(B.lo_other > B.hi);
                labels[p] = amb[q] ? -1 : O.arg[p];
            }
            hi_out[p] = (float)B.hi * (1.f + 1e-6f);
            lo_f = fmaxf(lo_f, (float)B.lo_min * (1.f - 1e-6f));
        }
    }
    kc_block_append_pp<KC_EPI_PP>(amb, pv, list, nlist);
    // block max of the lower bounds, one atomic per block
    __shared__ float red[4];
    float v = lo_f;
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
        // tens of thousands of blocks meet at one word: skip the atomic when
        // the word already holds as much (a stale read is never larger)
        const float cur = __uint_as_float(__hip_atomic_load(
            (const uint32_t*)lo_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (r > cur) kc_atomic_max_f32_nonneg(lo_max, r);
    }
}

// points whose upper bound reaches the largest lower bound may attain the
// covering radius: rescore them too
__global__ void k_radius_candidates(uint32_t n, const float* __restrict__ hi,
                                    const float* __restrict__ lo_max,
                                    uint32_t* __restrict__ list, uint32_t* __restrict__ nlist)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const float L = *lo_max;
    kc_block_append(p < n && hi[p] >= L, p, list, nlist);
}

// Second pass of an assignment on BF16 inputs, over the points the first
// one listed (entry q: row list[q]): the MFMA pass on their FP32 rows (O2,
// C2) bounds them again, without the BF16 rounding radii.  A label it
// certifies is written; an uncertain one lists the row for FP64.  Its lower
// bounds raise lo_max (still a lower bound of the radius).
__global__ void k_assign_refine_epilogue(const uint32_t* __restrict__ list,
                                         const uint32_t* __restrict__ nlist, uint32_t cap, int d,
                                         KcMinOut O2, KcCenters C2, int32_t* __restrict__ labels,
                                         float* __restrict__ hi2, uint32_t* __restrict__ list2,
                                         uint32_t* __restrict__ nlist2, float* __restrict__ lo_max)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nq = min(*nlist, cap);
    if ((uint64_t)blockIdx.x * blockDim.x >= nq) return;   // the whole block
    float lo_f = 0.f;
    bool need = false;
    uint32_t p = 0;
    if (q < nq) {
        p = list[q];
        const KcMdBounds B = kc_md_bounds(O2, q, nullptr, C2, d, labels != nullptr);
        if (labels) {
            if (B.lo_other > B.hi) labels[p] = O2.arg[q];
            else need = true;
        }
        hi2[q] = (float)B.hi * (1.f + 1e-6f);
        lo_f = (float)B.lo_min * (1.f - 1e-6f);
    }
    kc_block_append(need, p, list2, nlist2);
    __shared__ float red[4];
    float v = lo_f;
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
        const float cur = __uint_as_float(__hip_atomic_load(
            (const uint32_t*)lo_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (r > cur) kc_atomic_max_f32_nonneg(lo_max, r);
    }
}

// listed rows whose second-pass upper bound reaches the raised lower bound
// may attain the radius: FP64 for them; every point not listed by the first
// pass already has an upper bound below it
__global__ void k_assign_refine_radius(const uint32_t* __restrict__ list,
                                       const uint32_t* __restrict__ nlist, uint32_t cap,
                                       const float* __restrict__ hi2,
                                       const float* __restrict__ lo_max,
                                       uint32_t* __restrict__ list2, uint32_t* __restrict__ nlist2)
{
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nq = min(*nlist, cap);
    if ((uint64_t)blockIdx.x * blockDim.x >= nq) return;
    const float L = *lo_max;
    kc_block_append(q < nq && hi2[q] >= L, q < nq ? list[q] : 0u, list2, nlist2);
}

// Exact FP64 nearest center (lowest position on ties) of every listed point,
// with its label and radius^2 (as bits of a double).  A block takes 16 listed
// points at a time (four per wave, one after another, each held in VGPRs)
// and streams the k centers through LDS, rows at an odd pitch so the 64 lanes of a
// wave, each on its own center, read distinct banks; a wave reduces its lanes' minima
// per point, and the per-point minima carry over LDS chunks.  The distance
// sums separately rounded squares in coordinate order, as the FP64
// reference does.
#define KC_RS_FLOATS 12288   // 48 KiB of center coordinates per LDS chunk
#define KC_RS_PTS 16         // listed points per block pass
template <int D>
__global__ __launch_bounds__(256) void k_rescore_f64(const float* __restrict__ X, int64_t ld,
                                                     int d_rt, const float* __restrict__ Cf,
                                                     int dp, uint32_t k,
                                                     const int64_t* __restrict__ k_dev,
                                                     const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ nlist,
                                                     uint32_t cap, int32_t* __restrict__ labels,
                                                     double* __restrict__ radius2)
{
    const int d = D > 0 ? D : d_rt;
    const uint32_t pitch = (uint32_t)d | 1u;
    __shared__ float sC[KC_RS_FLOATS];
    __shared__ float sP[KC_RS_PTS][KC_MAXD];
    __shared__ double sBest[KC_RS_PTS];
    __shared__ int sArg[KC_RS_PTS];
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    uint32_t nl = *nlist;
    if (nl > cap) nl = cap;
    const uint32_t per = KC_RS_FLOATS / pitch;   // centers per chunk
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t b0 = blockIdx.x * KC_RS_PTS; b0 < nl; b0 += gridDim.x * KC_RS_PTS) {
        const uint32_t np = min((uint32_t)KC_RS_PTS, nl - b0);
        __syncthreads();
        for (uint32_t e = threadIdx.x; e < np * (uint32_t)d; e += blockDim.x) {
            const uint32_t q = e / (uint32_t)d, u = e - q * (uint32_t)d;
            sP[q][u] = X[(uint64_t)list[b0 + q] * (uint64_t)ld + u];
        }
        if (threadIdx.x < KC_RS_PTS) {
            sBest[threadIdx.x] = __builtin_inf();
            sArg[threadIdx.x] = 0x7FFFFFFF;
        }
        for (uint32_t c0 = 0; c0 < k; c0 += per) {
            const uint32_t cn = min(per, k - c0);
            __syncthreads();
            for (uint32_t e = threadIdx.x; e < cn * (uint32_t)d; e += blockDim.x) {
                const uint32_t c = e / (uint32_t)d, u = e - c * (uint32_t)d;
                sC[c * pitch + u] = Cf[(uint64_t)(c0 + c) * dp + u];
            }
            __syncthreads();
            for (uint32_t q = wave; q < np; q += blockDim.x >> 6) {
                const float* P = sP[q];
                float xr[D > 0 ? D : 1];   // the point, as FP32 (exact) in VGPRs
                if constexpr (D > 0) {
#pragma unroll
                    for (int u = 0; u < D; ++u) xr[u] = P[u];
                }
                double best = __builtin_inf();
                int bj = 0x7FFFFFFF;
                for (uint32_t c = lane; c < cn; c += 64) {
                    const float* cc = sC + c * pitch;
                    double a = 0.0;
                    if constexpr (D > 0) {
#pragma unroll
                        for (int u = 0; u < D; ++u)
                            a = kc_d64_step(a, (double)xr[u], (double)cc[u]);
                    } else {
                        for (int u = 0; u < d; ++u) a = kc_d64_step(a, (double)P[u], (double)cc[u]);
                    }
                    if (a < best) {   // a lane's centers ascend: ties keep the lowest
                        best = a;
                        bj = (int)(c0 + c);
                    }
                }
                for (int off = 32; off >= 1; off >>= 1) {
                    const double ob = __shfl_xor(best, off, 64);
                    const int oj = __shfl_xor(bj, off, 64);
                    if (ob < best || (ob == best && oj < bj)) {
                        best = ob;
                        bj = oj;
                    }
                }
                if (lane == 0 && best < sBest[q]) {   // later chunks hold higher positions
                    sBest[q] = best;
                    sArg[q] = bj;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < np) {
            const uint32_t q = threadIdx.x;
            if (labels) labels[list[b0 + q]] = sArg[q];
            kc_atomic_max_f64_nonneg(radius2, sBest[q]);
        }
    }
}

static void kc_rescore_f64(const float* X, int64_t ld, int d, const float* Cf, int dp,
                           uint32_t k, const int64_t* k_dev, const uint32_t* list,
                           const uint32_t* nlist, uint32_t cap, int32_t* labels,
                           double* radius2, hipStream_t s)
{
    const dim3 g(2048), b(256);
    switch (d) {
#define KC_RS_CASE(DD)                                                                      \
    case DD:                                                                                \
        hipLaunchKernelGGL(k_rescore_f64<DD>, g, b, 0, s, X, ld, d, Cf, dp, k, k_dev, list,  \
                           nlist, cap, labels, radius2);                                    \
        break;
        KC_RS_CASE(2)
        KC_RS_CASE(3)
        KC_RS_CASE(8)
        KC_RS_CASE(10)
        KC_RS_CASE(16)
        KC_RS_CASE(32)
        KC_RS_CASE(41)
#undef KC_RS_CASE
    default:
        hipLaunchKernelGGL(k_rescore_f64<0>, g, b, 0, s, X, ld, d, Cf, dp, k, k_dev, list, nlist,
                           cap, labels, radius2);
    }
}

// Covering radius only, small d: the canonical FP32 distance to every
// center (one lane per point, coordinates in VGPRs, the centers streamed
// through LDS).  Its relative error is at most g = gamma_{d+2}, so the
// exact min-distance lies in [m / (1 + g), m / (1 - g)] around the smallest
// FP32 value m (widened for rounding and for squares that underflow): far
// tighter than the MFMA bound, whose error scales with the norms, so only
// a handful of points reach the largest lower bound and go to the exact
// FP64 pass.  Writes hi_out[p] and the maximum lower bound into lo_max.
#define KC_RD_MAXD 8
#define KC_RD_CHUNK 1024
template <int D>
__global__ __launch_bounds__(256) void k_radius_direct(const float* __restrict__ X, int64_t ld,
                                                       uint32_t n, const float* __restrict__ Cf,
                                                       int dp, uint32_t k,
                                                       const int64_t* __restrict__ k_dev,
                                                       double g, float* __restrict__ hi_out,
                                                       float* __restrict__ lo_max)
{
    __shared__ float sC[KC_RD_CHUNK * D];
    __shared__ float red[4];
    if (k_dev && (int64_t)k > *k_dev) k = (uint32_t)(*k_dev < 0 ? 0 : *k_dev);
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = p < n;
    float xc[D];
#pragma unroll
    for (int u = 0; u < D; ++u) xc[u] = live ? X[(uint64_t)p * ld + u] : 0.f;
    float m = __builtin_inff();
    for (uint32_t j0 = 0; j0 < k; j0 += KC_RD_CHUNK) {
        const uint32_t cnt = min((uint32_t)KC_RD_CHUNK, k - j0);
        __syncthreads();
        for (uint32_t e0 = threadIdx.x; e0 < cnt * D; e0 += 8 * blockDim.x) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t e = e0 + q * blockDim.x, r = e / D, u = e - r * D;
                v[q] = e < cnt * D ? Cf[(uint64_t)(j0 + r) * dp + u] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t e = e0 + q * blockDim.x;
                if (e < cnt * D) sC[e] = v[q];
            }
        }
        __syncthreads();
        for (uint32_t r = 0; r < cnt; ++r) {
            const float a = kc_d32_dist<D>(xc, sC + r * D);
            m = fminf(m, a);
        }
    }
    float lo_f = 0.f;
    if (live) {
        const double mv = (double)m;
        double l = mv / (1.0 + g) - 1e-37 * D;
        if (l < 0.0) l = 0.0;
        const double u = mv / (1.0 - g) + 1e-37 * D;
        hi_out[p] = (float)u * (1.f + 1e-6f);
        lo_f = (float)l * (1.f - 1e-6f);
    }
    float v = lo_f;
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmaxf(r, red[w]);
        const float cur = __uint_as_float(__hip_atomic_load(
            (const uint32_t*)lo_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (r > cur) kc_atomic_max_f32_nonneg(lo_max, r);
    }
}

__global__ void k_sqrt_out(const double* __restrict__ r2, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = kc_sqrt_rn(*r2);
}

// ---------------------------------------------------------------------------
// host launchers

#define KC_MD_CASES_F32(X) X(1) X(2) X(3) X(4) X(8) X(11) X(16) X(32) X(64)
#define KC_MD_CASES_BF16(X) X(1) X(2) X(4) X(8)
#define KC_MD_CASES_PK(X) X(1) X(2) X(4) X(5)

int kc_mindist_ksteps(int d, bool bf)
{
    if (bf) {
        const int ks = (d + 31) / 32;
        if (ks <= 1) return 1;
        if (ks <= 2) return 2;
        if (ks <= 4) return 4;
        return 8;
    }
    const int ks = (d + 3) / 4;
    const int opts[] = {1, 2, 3, 4, 8, 11, 16, 32, 64};
    for (int o : opts)
        if (ks <= o) return o;
    return 64;
}

int kc_mindist_dpad(int d, bool bf)
{
    return bf ? kc_mindist_ksteps(d, true) * 32 : kc_mindist_ksteps(d, false) * 4;
}

int kc_split_packed_ksteps(int d)
{
    const int ks = (3 * d + 31) / 32;
    const int opts[] = {1, 2, 4, 5};   // d <= 53 (longer rows spill at 8 waves)
    for (int o : opts)
        if (ks <= o) return o < 3 * kc_mindist_ksteps(d, true) ? o : 0;
    return 0;
}

bool kc_split_use_packed(int d, uint32_t kpad)
{
    // the packed operands cost a point about 3d scattered loads and roundings
    // up front, which fewer MFMAs repay only over many centers
    return kpad >= 2048 && kc_split_packed_ksteps(d) > 0;
}

int kc_mindist_dpad_split(int d, uint32_t kpad)
{
    return kc_split_use_packed(d, kpad) ? kc_split_packed_ksteps(d) * 32
                                        : kc_mindist_dpad(d, true);
}

// Bytes per staged center element in LDS (the split keeps two parts).
static uint32_t kc_md_elem_bytes(int mode)
{
    return mode == KC_MD_BF16 || mode == KC_MD_SPLITP ? 2 : 4;
}

// Largest center chunk (multiple of 16) whose LDS copy fits in `kib` KiB
// (dp: the staged rows' padded K).
static uint32_t kc_mindist_chunk(int dp_rows, int mode, uint32_t kpad, uint32_t kib)
{
    const uint32_t dp = (uint32_t)kc_md_pitch(mode, dp_rows);
    const uint32_t per = dp * kc_md_elem_bytes(mode) + (mode == KC_MD_BF16 ? 16 : 12);
    uint32_t c = (kib * 1024u / per) & ~15u;
    if (c < 16) c = 16;
    return c < kpad ? c : kpad;
}

void kc_mindist(const float* X, const uint16_t* Xb, const float* ex, int64_t ld, uint32_t n,
                int d, const KcCenters& C, const KcMinOut& O, bool lab, hipStream_t s, int waves,
                int lds_kib, const uint32_t* rows, const uint32_t* n_dev)
{
    if (lds_kib != 32) lds_kib = 64;
    if (waves != 8) waves = 4;
    const int mode = Xb     ? KC_MD_BF16
                     : C.pk  ? KC_MD_SPLITP
                     : C.Cbl ? KC_MD_SPLIT
                             : KC_MD_F32;
    const bool bf = mode != KC_MD_F32;
    const int klen = mode == KC_MD_SPLITP ? C.dp : kc_mindist_dpad(d, bf);   // staged row
    const int ks = mode == KC_MD_SPLITP ? C.dp / 32 : kc_mindist_ksteps(d, bf);
    const uint32_t chunk = kc_mindist_chunk(klen, mode, C.kpad, (uint32_t)lds_kib);
    const int dp = kc_md_pitch(mode, klen);
    const size_t smem = (size_t)chunk * (mode == KC_MD_BF16 ? 16 : 12) +
                        (size_t)chunk * dp * kc_md_elem_bytes(mode);
    const uint32_t per_block = (uint32_t)waves * 16 * kc_md_pt(mode, ks);
    const dim3 grid((n + per_block - 1) / per_block), block(waves * 64);
    const float gm = (float)kc_md_gamma(d, mode == KC_MD_SPLIT || mode == KC_MD_SPLITP);
#define KC_LAUNCH_W(M, K, WW)                                                              \
    if (lab)                                                                               \
        hipLaunchKernelGGL((k_mindist_mfma<M, K, true, WW>), grid, block, smem, s, X, Xb, ex, \
                           ld, n, d, gm, C, chunk, O, rows, n_dev);                        \
    else                                                                                   \
        hipLaunchKernelGGL((k_mindist_mfma<M, K, false, WW>), grid, block, smem, s, X, Xb,  \
                           ex, ld, n, d, gm, C, chunk, O, rows, n_dev);
#define KC_LAUNCH(M, K)         \
    if (waves == 8) {           \
        KC_LAUNCH_W(M, K, 8)    \
    } else {                    \
        KC_LAUNCH_W(M, K, 4)    \
    }
    if (mode == KC_MD_F32) {
        switch (ks) {
#define KC_CASE(K) \
    case K:        \
        KC_LAUNCH(KC_MD_F32, K) break;
            KC_MD_CASES_F32(KC_CASE)
#undef KC_CASE
        }
    } else if (mode == KC_MD_BF16) {
        switch (ks) {
#define KC_CASE(K) \
    case K:        \
        KC_LAUNCH(KC_MD_BF16, K) break;
            KC_MD_CASES_BF16(KC_CASE)
#undef KC_CASE
        }
    } else if (mode == KC_MD_SPLIT) {
        switch (ks) {
#define KC_CASE(K) \
    case K:        \
        KC_LAUNCH(KC_MD_SPLIT, K) break;
            KC_MD_CASES_BF16(KC_CASE)
#undef KC_CASE
        }
    } else {
        switch (ks) {
#define KC_CASE(K) \
    case K:        \
        KC_LAUNCH(KC_MD_SPLITP, K) break;
            KC_MD_CASES_PK(KC_CASE)
#undef KC_CASE
        }
    }
#undef KC_LAUNCH
#undef KC_LAUNCH_W
}

void kc_stage_centers(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n,
                      const int64_t* idx, const uint32_t* idx32, uint32_t k,
                      const int64_t* k_dev, const KcCenters& C, uint32_t* status, hipStream_t s)
{
    kc_fill_u32((uint32_t*)C.cmax, 0u, 2, s);
    if (C.kpad >= 2048)
        hipLaunchKernelGGL(k_stage_centers_thread, dim3((C.kpad + 255) / 256), dim3(256), 0, s,
                           X, Xb, ld, d, n, idx, idx32, k, k_dev, C, status);
    else
        hipLaunchKernelGGL(k_stage_centers, dim3((C.kpad + 3) / 4), dim3(256), 0, s, X, Xb, ld, d,
                           n, idx, idx32, k, k_dev, C, status);
}

void kc_local_origin(const float* X, int64_t ld, int d, uint32_t n, float* mu, hipStream_t s)
{
    hipLaunchKernelGGL(k_local_origin, dim3(d), dim3(256), 0, s, X, ld, n, mu);
}

void kc_bf16_err(const float* X, const uint16_t* Xb, int64_t ld, int d, uint32_t n, float* ex,
                 hipStream_t s)
{
    if (ld == d && d <= KC_ERR_DENSE_D && (uintptr_t)X % 16 == 0 && (uintptr_t)Xb % 8 == 0)
        hipLaunchKernelGGL(k_bf16_err_dense, dim3((n + 63) / 64), dim3(256),
                           (size_t)64 * (size_t)d * sizeof(double), s, X, Xb, d, n, ex);
    else
        hipLaunchKernelGGL(k_bf16_err, dim3((n + 63) / 64), dim3(256), 0, s, X, Xb, ld, d, n,
                           ex);
}

bool kc_radius_direct(uint32_t n, int d, const float* X, int64_t ld, const float* Cf, int dp,
                      uint32_t k, const int64_t* k_dev, float* hi, uint32_t* list,
                      uint32_t* nlist, float* lo_max, double* radius2, double* radius_out,
                      hipStream_t s)
{
    if (d < 1 || d > KC_RD_MAXD) return false;
    const double u32 = 5.9604644775390625e-8, m = d + 2;
    const double g = m * u32 / (1.0 - m * u32);
    kc_fill_u32(nlist, 0u, 1, s);
    kc_fill_u32((uint32_t*)lo_max, 0u, 1, s);
    kc_fill_u64((u64*)radius2, 0ull, 1, s);
    const dim3 gr((n + 255) / 256);
    switch (d) {
#define KC_RD_CASE(DD)                                                                      \
    case DD:                                                                                \
        hipLaunchKernelGGL(k_radius_direct<DD>, gr, dim3(256), 0, s, X, ld, n, Cf, dp, k,    \
                           k_dev, g, hi, lo_max);                                           \
        break;
        KC_RD_CASE(1)
        KC_RD_CASE(2)
        KC_RD_CASE(3)
        KC_RD_CASE(4)
        KC_RD_CASE(5)
        KC_RD_CASE(6)
        KC_RD_CASE(7)
        KC_RD_CASE(8)
#undef KC_RD_CASE
    }
    hipLaunchKernelGGL(k_radius_candidates, gr, dim3(256), 0, s, n, hi, lo_max, list, nlist);
    kc_rescore_f64(X, ld, d, Cf, dp, k, k_dev, list, nlist, 2 * n, nullptr, radius2, s);
    hipLaunchKernelGGL(k_sqrt_out, dim3(1), dim3(64), 0, s, radius2, radius_out);
    return true;
}

void kc_assign_finish(uint32_t n, int d, const float* X, int64_t ld, const KcCenters& C,
                      uint32_t k, const int64_t* k_dev, const KcMinOut& O, const float* ex,
                      int32_t* labels, float* hi, uint32_t* list, uint32_t* nlist,
                      float* lo_max, double* radius2, double* radius_out, hipStream_t s,
                      const KcAssignRefine* R2)
{
    kc_fill_u32(nlist, 0u, 1, s);
    kc_fill_u32((uint32_t*)lo_max, 0u, 1, s);
    kc_fill_u64((u64*)radius2, 0ull, 1, s);
    const dim3 g((n + 255) / 256);
    hipLaunchKernelGGL(k_assign_epilogue, dim3((n + 256 * KC_EPI_PP - 1) / (256 * KC_EPI_PP)),
                       dim3(256), 0, s, n, d, O, ex, C, labels, hi, list, nlist, lo_max);
    hipLaunchKernelGGL(k_radius_candidates, g, dim3(256), 0, s, n, hi, lo_max, list, nlist);
    if (!R2) {
        kc_rescore_f64(X, ld, d, C.Cf, C.dp, k, k_dev, list, nlist, 2 * n, labels, radius2, s);
    } else {
        // the listed points again, on their FP32 rows (up to 2n entries: a
        // point can be listed as ambiguous and as a radius candidate)
        const uint32_t cap = 2 * n;
        const dim3 g2((cap + 255) / 256);
        kc_fill_u32(R2->nlist, 0u, 1, s);
        kc_mindist(X, nullptr, nullptr, ld, cap, d, R2->C, R2->O, labels != nullptr, s, 4, 64,
                   list, nlist);
        hipLaunchKernelGGL(k_assign_refine_epilogue, g2, dim3(256), 0, s, list, nlist, cap, d,
                           R2->O, R2->C, labels, R2->hi, R2->list, R2->nlist, lo_max);
        hipLaunchKernelGGL(k_assign_refine_radius, g2, dim3(256), 0, s, list, nlist, cap, R2->hi,
                           lo_max, R2->list, R2->nlist);
        kc_rescore_f64(X, ld, d, C.Cf, C.dp, k, k_dev, R2->list, R2->nlist, 2 * cap, labels,
                       radius2, s);
    }
    hipLaunchKernelGGL(k_sqrt_out, dim3(1), dim3(64), 0, s, radius2, radius_out);
}
