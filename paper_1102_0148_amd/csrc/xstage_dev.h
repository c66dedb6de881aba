// X-stage of the FX correlator: for every channel f, the Hermitian rank-T
// update V_f += X_f X_f^H over a time range, upper triangle only, on MFMA.
//
// What is computed (Section 1 of Prasad & Subrahmanya): for each channel and
// every antenna pair a <= b, V[a,b] = sum_t X[t,a] conj(X[t,b]).
//
// How (gfx950): the antennas of one channel form 16-antenna blocks; a
// wavefront owns a region of block pairs (I, J) and keeps both 16x16
// accumulators of every pair in registers over its time range.  With a
// record P = [re x TG | im x TG] of TG spectra and Q = [im x TG | -re x TG]:
//     Re V_IJ = sum P_I P_J^T,     Im V_IJ = sum Q_I P_J^T,
// since sum_k Q_a[k] P_b[k] = sum_t (im_a re_b - re_a im_b).  One 16-byte
// record per lane is exactly one MFMA operand for the fp16 (16x16x32) and
// int8 (16x16x64) forms, and four consecutive operands for fp32 (16x16x4).
// The fp32 form, which is bound by MFMA rate rather than by memory, issues
// fewer products: off the diagonal it uses three real products instead of
// four (P1 = Xr Xr^T, P2 = Xi Xi^T, P3 = (Xr+Xi)(Xr-Xi)^T give Re = P1 + P2
// and Im = P3 - P1 + P2), and on a diagonal block Re = P1 + P2 in one
// accumulator and Im = M - M^T with M = Xi Xr^T (so autos are exactly real).
// Each wave writes its partial sums [split][channel][baseline]; the dump
// kernel adds them into float64 in a fixed order.
#pragma once
#include "corr_internal.h"

namespace corr {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int PREC> struct AccT { typedef f32x4 type; };
template <> struct AccT<kINT8> { typedef i32x4 type; };

// per-byte negation of four int8 values in [-127, 127]
__device__ __forceinline__ uint32_t neg_i8x4(uint32_t b) {
    return (0x80808080u - (b & 0x7F7F7F7Fu)) ^ (~b & 0x80808080u);
}

// Q = [hi half | -(lo half)] of a record
template <int PREC>
__device__ __forceinline__ uint4 make_q(uint4 p) {
    if constexpr (PREC == kFP32) {
        return make_uint4(p.z, p.w, p.x ^ 0x80000000u, p.y ^ 0x80000000u);
    } else if constexpr (PREC == kFP16) {
        return make_uint4(p.z, p.w, p.x ^ 0x80008000u, p.y ^ 0x80008000u);
    } else {
        return make_uint4(p.z, p.w, neg_i8x4(p.x), neg_i8x4(p.y));
    }
}

template <int PREC>
__device__ __forceinline__ void mma(typename AccT<PREC>::type &acc, uint4 a, uint4 b) {
    if constexpr (PREC == kFP32) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), acc, 0, 0, 0);
    } else if constexpr (PREC == kFP16) {
        f16x8 av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
    } else {
        i32x4 av = {(int)a.x, (int)a.y, (int)a.z, (int)a.w};
        i32x4 bv = {(int)b.x, (int)b.y, (int)b.z, (int)b.w};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, acc, 0, 0, 0);
    }
}

template <int PREC>
__device__ __forceinline__ void store_vis(void *partial, int64_t idx, typename AccT<PREC>::type &re,
                                          typename AccT<PREC>::type &im, int v, bool auto_corr) {
    if constexpr (PREC == kINT8) {
        reinterpret_cast<int2 *>(partial)[idx] = make_int2(re[v], auto_corr ? 0 : im[v]);
    } else {
        reinterpret_cast<float2 *>(partial)[idx] = make_float2(re[v], auto_corr ? 0.0f : im[v]);
    }
}

__device__ __forceinline__ f32x4 mf32(float a, float b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}


// One wavefront's share of the X-stage: region `wave % nregions` of channel
// (wave / nregions) % K over time split wave / (nregions K).  `wave` must be
// wave-uniform; tb is this wave's 16 x 17 floats of LDS (fp32 form only).
template <int PREC, int RB, bool DIAG>
__device__ __forceinline__ void x_wave(const XArgs &a, int wave, float *tb) {
    typedef typename AccT<PREC>::type acc_t;
    constexpr bool F3M = PREC == kFP32;   // three-product form
    const int lane = threadIdx.x & 63;
    if (wave >= a.nregions * a.K * a.nsplit) return;
    const int reg = wave % a.nregions;
    const int rest = wave / a.nregions;
    const int f = rest % a.K;
    const int sp = rest / a.K;
    const int I0 = a.regions[reg].x, J0 = a.regions[reg].y;
    const int kb0 = (int)((int64_t)sp * a.nkb / a.nsplit);
    const int kb1 = (int)((int64_t)(sp + 1) * a.nkb / a.nsplit);

    // Q form: accR = Re, accI = Im.  fp32: diagonal pair accR = Re, accI = M;
    // off-diagonal pair accR = P1, accI = P2, acc3 = P3.
    acc_t accR[RB][RB], accI[RB][RB], acc3[RB][RB];
#pragma unroll
    for (int I = 0; I < RB; ++I)
#pragma unroll
        for (int J = 0; J < RB; ++J) {
            accR[I][J] = acc_t{0, 0, 0, 0};
            accI[I][J] = acc_t{0, 0, 0, 0};
            acc3[I][J] = acc_t{0, 0, 0, 0};
        }

    // lane (row r, group g) reads record tq = 4 kb + g of antenna 16 I + r;
    // a k-block is the (kb mod 4)-th quarter of time block kb / 4
    const uint4 *base = a.spec + (int64_t)f * kTQB * a.a_pad + (lane >> 4) * a.a_pad + (lane & 15);
    const int64_t bstride = (int64_t)a.K * kTQB * a.a_pad;

    // two register sets alternate: the records of the next k-block are in
    // flight while the current one is multiplied
    auto load = [&](int kb, uint4 *r, uint4 *c) {
        const uint4 *rec = base + (kb >> 2) * bstride + (kb & 3) * 4 * a.a_pad;
#pragma unroll
        for (int I = 0; I < RB; ++I) r[I] = rec[(I0 + I) * 16];
        if constexpr (!DIAG) {
#pragma unroll
            for (int J = 0; J < RB; ++J) c[J] = rec[(J0 + J) * 16];
        }
    };
    auto compute = [&](const uint4 *pr, const uint4 *pc) {
        if constexpr (F3M) {
            // record = (re t0, re t1, im t0, im t1)
            float sr[RB][2], dc[RB][2];
#pragma unroll
            for (int I = 0; I < RB; ++I) {
                const float4 p = *reinterpret_cast<const float4 *>(&pr[I]);
                sr[I][0] = p.x + p.z;
                sr[I][1] = p.y + p.w;
            }
#pragma unroll
            for (int J = 0; J < RB; ++J) {
                const float4 p = *reinterpret_cast<const float4 *>(DIAG ? &pr[J] : &pc[J]);
                dc[J][0] = p.x - p.z;
                dc[J][1] = p.y - p.w;
            }
#pragma unroll
            for (int I = 0; I < RB; ++I)
#pragma unroll
                for (int J = 0; J < RB; ++J) {
                    if (DIAG && J < I) continue;
                    const float4 x = *reinterpret_cast<const float4 *>(&pr[I]);
                    const float4 y = *reinterpret_cast<const float4 *>(DIAG ? &pr[J] : &pc[J]);
                    if (DIAG && I == J) {
                        accR[I][J] = mf32(x.x, x.x, accR[I][J]);
                        accR[I][J] = mf32(x.y, x.y, accR[I][J]);
                        accR[I][J] = mf32(x.z, x.z, accR[I][J]);
                        accR[I][J] = mf32(x.w, x.w, accR[I][J]);
                        accI[I][J] = mf32(x.z, x.x, accI[I][J]);
                        accI[I][J] = mf32(x.w, x.y, accI[I][J]);
                    } else {
                        accR[I][J] = mf32(x.x, y.x, accR[I][J]);
                        accR[I][J] = mf32(x.y, y.y, accR[I][J]);
                        accI[I][J] = mf32(x.z, y.z, accI[I][J]);
                        accI[I][J] = mf32(x.w, y.w, accI[I][J]);
                        acc3[I][J] = mf32(sr[I][0], dc[J][0], acc3[I][J]);
                        acc3[I][J] = mf32(sr[I][1], dc[J][1], acc3[I][J]);
                    }
                }
        } else {
            uint4 qr[RB];
#pragma unroll
            for (int I = 0; I < RB; ++I) qr[I] = make_q<PREC>(pr[I]);
#pragma unroll
            for (int I = 0; I < RB; ++I)
#pragma unroll
                for (int J = 0; J < RB; ++J) {
                    if (DIAG && J < I) continue;
                    const uint4 b = DIAG ? pr[J] : pc[J];
                    mma<PREC>(accR[I][J], pr[I], b);
                    mma<PREC>(accI[I][J], qr[I], b);
                }
        }
    };
    uint4 ar[RB], ac[RB], br[RB], bc[RB];
    int kb = kb0;
    if (kb < kb1) load(kb, ar, ac);
#pragma unroll 1
    for (; kb + 1 < kb1; kb += 2) {
        load(kb + 1, br, bc);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
        compute(ar, ac);
        load(min(kb + 2, kb1 - 1), ar, ac);
        __builtin_amdgcn_sched_barrier(0);
        compute(br, bc);
    }
    if (kb < kb1) compute(ar, ac);

    if constexpr (F3M) {
        // turn the fp32 accumulators into (Re, Im): off the diagonal Re = P1 + P2,
        // Im = P3 - P1 + P2; on it Im = M - M^T, transposed through LDS
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RB; ++J) {
                if (DIAG && J < I) continue;
                if (DIAG && I == J) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) tb[(4 * (lane >> 4) + v) * 17 + (lane & 15)] = accI[I][J][v];
                    wave_lds_sync();
                    f32x4 mt;
#pragma unroll
                    for (int v = 0; v < 4; ++v) mt[v] = tb[(lane & 15) * 17 + 4 * (lane >> 4) + v];
                    wave_lds_sync();
                    accI[I][J] = accI[I][J] - mt;
                } else {
                    const f32x4 p1 = accR[I][J], p2 = accI[I][J];
                    accR[I][J] = p1 + p2;
                    accI[I][J] = acc3[I][J] - p1 + p2;
                }
            }
    }

    // accumulator element v of lane l is row 4*(l/16)+v, column l%16
    const int64_t obase = ((int64_t)sp * a.K + f) * a.nb;
#pragma unroll
    for (int I = 0; I < RB; ++I)
#pragma unroll
        for (int J = 0; J < RB; ++J) {
            if (DIAG && J < I) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ia = (I0 + I) * 16 + 4 * (lane >> 4) + v;
                const int ib = (J0 + J) * 16 + (lane & 15);
                if (ia < a.N && ib < a.N && ia <= ib) {
                    const int bl = ia * a.N - ia * (ia - 1) / 2 + (ib - ia);
                    store_vis<PREC>(a.partial, obase + bl, accR[I][J], accI[I][J], v, ia == ib);
                }
            }
        }
}

}  // namespace
}  // namespace corr
