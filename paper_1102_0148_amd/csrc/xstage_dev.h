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


// The accumulators of one wavefront's region: RB x RBJ pairs of 16-antenna
// blocks (DIAG: the upper triangle of a square diagonal region) of one
// channel, both
// 16x16 accumulators of every pair in registers.  zero() clears them, run()
// adds a range of k-blocks of a record buffer laid out as rec_index (add()
// one k-block whose records are already in registers), store() turns them
// into (Re, Im) and writes the pairs a <= b < N of a partial row.
template <int PREC, int RB, bool DIAG, int RBJ = RB>
struct XRegion {
    static_assert(!DIAG || RBJ == RB, "a diagonal region is square");
    typedef typename AccT<PREC>::type acc_t;
    static constexpr bool F3M = PREC == kFP32;  // three-product form
    // Q form: accR = Re, accI = Im.  fp32: diagonal pair accR = Re, accI = M;
    // off-diagonal pair accR = P1, accI = P2, acc3 = P3.
    acc_t accR[RB][RBJ], accI[RB][RBJ], acc3[RB][RBJ];

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RBJ; ++J) {
                accR[I][J] = acc_t{0, 0, 0, 0};
                accI[I][J] = acc_t{0, 0, 0, 0};
                acc3[I][J] = acc_t{0, 0, 0, 0};
            }
    }

    // k-blocks [kb0, kb1) of channel f, row blocks I0.., column blocks J0..
    // NBUF register sets rotate: the records of the next NBUF - 1 k-blocks are
    // in flight while one is multiplied (2 where many waves share a SIMD and
    // hide each other's latency; more for a wave that runs alone).
    template <int NBUF = 2>
    __device__ __forceinline__ void run(const uint4 *spec, int K, int a_pad, int f, int I0, int J0, int kb0,
                                        int kb1) {
        const int lane = threadIdx.x & 63;
        // lane (row r, group g) reads record tq = 4 kb + g of antenna 16 I + r;
        // a k-block is the (kb mod 4)-th quarter of time block kb / 4
        const uint4 *base = spec + (int64_t)f * kTQB * a_pad + (lane >> 4) * a_pad + (lane & 15);
        const int64_t bstride = (int64_t)K * kTQB * a_pad;

        // two register sets alternate: the records of the next k-block are in
        // flight while the current one is multiplied
        auto load = [&](int kb, uint4 *r, uint4 *c) {
            const uint4 *rec = base + (kb >> 2) * bstride + (kb & 3) * 4 * a_pad;
#pragma unroll
            for (int I = 0; I < RB; ++I) r[I] = rec[(I0 + I) * 16];
            if constexpr (!DIAG) {
#pragma unroll
                for (int J = 0; J < RBJ; ++J) c[J] = rec[(J0 + J) * 16];
            }
        };
        auto compute = [&](const uint4 *pr, const uint4 *pc) { this->add(pr, pc); };
        // set i holds k-block kb + i at the top of a round; in step i of a round
        // set (i + NBUF - 1) mod NBUF, just freed, is loaded with k-block
        // kb + i + NBUF - 1 (the last one again past the end) and set i is
        // multiplied
        uint4 r[NBUF][RB], c[NBUF][RBJ];
#pragma unroll
        for (int i = 0; i < NBUF - 1; ++i)
            if (kb0 + i < kb1) load(kb0 + i, r[i], c[i]);
        int kb = kb0;
#pragma unroll 1
        for (; kb + NBUF - 1 < kb1; kb += NBUF) {
#pragma unroll
            for (int i = 0; i < NBUF; ++i) {
                load(min(kb + i + NBUF - 1, kb1 - 1), r[(i + NBUF - 1) % NBUF], c[(i + NBUF - 1) % NBUF]);
                __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
                compute(r[i], c[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < NBUF - 1; ++i)
            if (kb + i < kb1) compute(r[i], c[i]);
    }

    // One k-block: the row blocks' records pr[RB] (lane: record tq = 4 kb + g
    // of antenna 16 I + r) and the column blocks' pc[RB] (unused on the
    // diagonal).
    __device__ __forceinline__ void add(const uint4 *pr, const uint4 *pc) {
            if constexpr (F3M) {
                // record = (re t0, re t1, im t0, im t1)
                float sr[RB][2], dc[RBJ][2];
#pragma unroll
                for (int I = 0; I < RB; ++I) {
                    const float4 p = *reinterpret_cast<const float4 *>(&pr[I]);
                    sr[I][0] = p.x + p.z;
                    sr[I][1] = p.y + p.w;
                }
#pragma unroll
                for (int J = 0; J < RBJ; ++J) {
                    const float4 p = *reinterpret_cast<const float4 *>(DIAG ? &pr[J] : &pc[J]);
                    dc[J][0] = p.x - p.z;
                    dc[J][1] = p.y - p.w;
                }
#pragma unroll
                for (int I = 0; I < RB; ++I)
#pragma unroll
                    for (int J = 0; J < RBJ; ++J) {
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
                    for (int J = 0; J < RBJ; ++J) {
                        if (DIAG && J < I) continue;
                        const uint4 b = DIAG ? pr[J] : pc[J];
                        mma<PREC>(accR[I][J], pr[I], b);
                        mma<PREC>(accI[I][J], qr[I], b);
                    }
            }
    }

    // Write the region into partial row obase ([baseline] of one split and
    // channel); tb is this wave's 16 x 17 floats of LDS (fp32 form only).
    // The fp32 accumulators are turned into (Re, Im) in place.
    __device__ __forceinline__ void store(void *partial, int64_t obase, int N, int I0, int J0, float *tb) {
        const int lane = threadIdx.x & 63;
        if constexpr (F3M) {
            // off the diagonal Re = P1 + P2, Im = P3 - P1 + P2; on it
            // Im = M - M^T, transposed through LDS
#pragma unroll
            for (int I = 0; I < RB; ++I)
#pragma unroll
                for (int J = 0; J < RBJ; ++J) {
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
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RBJ; ++J) {
                if (DIAG && J < I) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ia = (I0 + I) * 16 + 4 * (lane >> 4) + v;
                    const int ib = (J0 + J) * 16 + (lane & 15);
                    if (ia < N && ib < N && ia <= ib) {
                        const int bl = ia * N - ia * (ia - 1) / 2 + (ib - ia);
                        store_vis<PREC>(partial, obase + bl, accR[I][J], accI[I][J], v, ia == ib);
                    }
                }
            }
    }
};

// One wavefront's share of the X-stage: region `wave % nregions` of channel
// (wave / nregions) % K over time split wave / (nregions K).  `wave` must be
// wave-uniform; tb is this wave's 16 x 17 floats of LDS (fp32 form only).
template <int PREC, int RB, bool DIAG>
__device__ __forceinline__ void x_wave(const XArgs &a, int wave, float *tb) {
    if (wave >= a.nregions * a.K * a.nsplit) return;
    const int reg = wave % a.nregions;
    const int rest = wave / a.nregions;
    const int f = rest % a.K;
    const int sp = rest / a.K;
    const int I0 = a.regions[reg].x, J0 = a.regions[reg].y;
    const int kb0 = (int)((int64_t)sp * a.nkb / a.nsplit);
    const int kb1 = (int)((int64_t)(sp + 1) * a.nkb / a.nsplit);
    XRegion<PREC, RB, DIAG> x;
    x.zero();
    x.run(a.spec, a.K, a.a_pad, f, I0, J0, kb0, kb1);
    x.store(a.partial, ((int64_t)sp * a.K + f) * a.nb, a.N, I0, J0, tb);
}

// ------------------------------------------------------------ LDS groups
// A stage of the LDS ring: 16 block slots of one k-block, slot s holding
// [record g][antenna r] (16 B each) of block r0 + s (s < 8) or c0 + s - 8.
constexpr int kXSlots = 16;
constexpr int kXStage = kXSlots * 64;  // uint4 per stage (16 KB)
#ifndef X_RING
#define X_RING 3
#endif
constexpr int kXRing = X_RING;  // stages in the ring

// Issue this wave's share of one k-block's blocks as direct global-to-LDS
// loads (16 B per lane; lane l lands at slot base + 16 l, which is the
// [g][r] order, lane = 16 g + r).  NS slots per k-block, NS / 4 per wave.
template <int NS>
__device__ __forceinline__ void xg_issue(const uint4 *spec, int K, int a_pad, int r0, int c0, int f, int kb,
                                         uint4 *stage, int wave) {
    const int lane = threadIdx.x & 63;
    const uint4 *rec = spec + ((int64_t)(kb >> 2) * K + f) * kTQB * a_pad + (kb & 3) * 4 * a_pad +
                       (lane >> 4) * a_pad + (lane & 15);
#pragma unroll
    for (int i = 0; i < NS / 4; ++i) {
        const int s = wave * (NS / 4) + i;
        const int blk = s < 8 ? r0 + s : c0 + (s - 8);
        __builtin_amdgcn_global_load_lds(rec + blk * 16, stage + s * 64, 16, 0, 0);
    }
}

// One k-block of a region from a stage: P/Q products as in x_wave.
template <int PREC, bool DIAG, int NJ = 4>
__device__ __forceinline__ void xg_compute(const uint4 *stage, int rs, int cs,
                                           typename AccT<PREC>::type (&accR)[4][NJ],
                                           typename AccT<PREC>::type (&accI)[4][NJ]) {
    const int lane = threadIdx.x & 63;
    uint4 pr[4], pc[NJ], qr[4];
#pragma unroll
    for (int I = 0; I < 4; ++I) pr[I] = stage[(rs + I) * 64 + lane];
    if constexpr (!DIAG) {
#pragma unroll
        for (int J = 0; J < NJ; ++J) pc[J] = stage[(cs + J) * 64 + lane];
    }
#pragma unroll
    for (int I = 0; I < 4; ++I) qr[I] = make_q<PREC>(pr[I]);
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int J = 0; J < NJ; ++J) {
            if (DIAG && J < I) continue;
            const uint4 b = DIAG ? pr[J] : pc[J];
            mma<PREC>(accR[I][J], pr[I], b);
            mma<PREC>(accI[I][J], qr[I], b);
        }
}

// s_waitcnt vmcnt(n) lgkmcnt(0), expcnt left alone.  The builtin takes an
// immediate only; n is a constant after unrolling and the switch folds away
// (a count above 15 waits for everything, which is never wrong).
__device__ __forceinline__ void wait_vm_lgkm0(int n) {
    switch (n) {
#define X_WAIT_CASE(c) \
    case c: __builtin_amdgcn_s_waitcnt(0x0070 | c); break;
        X_WAIT_CASE(1) X_WAIT_CASE(2) X_WAIT_CASE(3) X_WAIT_CASE(4) X_WAIT_CASE(5) X_WAIT_CASE(6)
        X_WAIT_CASE(7) X_WAIT_CASE(8) X_WAIT_CASE(9) X_WAIT_CASE(10) X_WAIT_CASE(11) X_WAIT_CASE(12)
        X_WAIT_CASE(13) X_WAIT_CASE(14) X_WAIT_CASE(15)
#undef X_WAIT_CASE
        default: __builtin_amdgcn_s_waitcnt(0x0070); break;
    }
}

// The k-block loop of one wave's region over a ring of kXRing stages: the
// loads run kXRing - 1 k-blocks ahead, and one barrier per k-block both
// publishes the stage about to be used and frees the one about to be
// refilled.  Each wave waits only for its own loads of the current k-block
// (vmcnt), then the barrier covers every wave's; lgkmcnt(0) first retires
// this wave's reads of the stage that the loads issued after the barrier
// overwrite.  (A __syncthreads here would wait for every load in flight, the
// prefetch too.)  Whole rounds of kXRing k-blocks come first, so every path
// into a round has the same loads in flight, which keeps the compiler's own
// vmcnt bookkeeping exact; the last k-blocks, fewer than kXRing, already sit
// in the first stages.  Loads past the range repeat the last k-block.
template <int PREC, bool DIAG, int NS>
__device__ __forceinline__ void xg_loop(const uint4 *spec, int K, int a_pad, int r0, int c0, int f, int kb0,
                                        int kb1, int wave, int rs, int cs, bool active,
                                        uint4 *const (&st)[kXRing], typename AccT<PREC>::type (&accR)[4][4],
                                        typename AccT<PREC>::type (&accI)[4][4]) {
    constexpr int kPer = NS / 4;  // loads per wave per k-block
    const int last = kb1 - 1;
#pragma unroll
    for (int s = 0; s + 1 < kXRing; ++s) xg_issue<NS>(spec, K, a_pad, r0, c0, f, min(kb0 + s, last), st[s], wave);
    int kb = kb0;
#pragma unroll 1
    for (; kb + kXRing <= kb1; kb += kXRing) {
#pragma unroll
        for (int s = 0; s < kXRing; ++s) {
            wait_vm_lgkm0((kXRing - 2) * kPer);
            __builtin_amdgcn_s_barrier();
            xg_issue<NS>(spec, K, a_pad, r0, c0, f, min(kb + s + kXRing - 1, last), st[(s + kXRing - 1) % kXRing],
                         wave);
            if (active) xg_compute<PREC, DIAG>(st[s], rs, cs, accR, accI);
        }
    }
#pragma unroll
    for (int s = 0; s + 1 < kXRing; ++s) {
        if (kb + s < kb1) {
            wait_vm_lgkm0((kXRing - 2 - s) * kPer);
            __builtin_amdgcn_s_barrier();
            if (active) xg_compute<PREC, DIAG>(st[s], rs, cs, accR, accI);
        }
    }
    wait_vm_lgkm0(0);  // the ring's last loads have landed
}

// ------------------------------------------------- whole-channel groups
// Sixteen antenna blocks (4 x 4-block regions in 4 region rows): one
// workgroup of eight waves per (channel, split) stages all 16 blocks of a
// k-block in LDS once (slot s = block s; each wave loads two slots), so every
// record of the channel is fetched once per split instead of twice as with
// the three region groups.  The 136 block pairs go to the waves so that
// every SIMD carries 34 (waves are dealt to SIMDs in turn, w and w + 4
// sharing one): wave w < 4 takes the diagonal region at block 4w (10 pairs)
// and half of an off-diagonal one, (0, 4) or (8, 12) split by columns into
// 4 x 2 blocks (8 pairs); waves 4-7 take the off-diagonal regions (0, 8),
// (0, 12), (4, 8) and (4, 12) (16 pairs each).  (Two diagonal regions on
// each of waves 0 and 1 and one off-diagonal region on each other wave left
// the SIMDs 36, 36, 32 and 32 pairs.)  Two waves per SIMD keep 256
// registers.
constexpr int kXChanWaves = 8;

__device__ __forceinline__ void xc_issue(const uint4 *spec, int K, int a_pad, int f, int kb, uint4 *stage, int wave) {
    const int lane = threadIdx.x & 63;
    const uint4 *rec = spec + ((int64_t)(kb >> 2) * K + f) * kTQB * a_pad + (kb & 3) * 4 * a_pad +
                       (lane >> 4) * a_pad + (lane & 15);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int s = 2 * wave + i;
        __builtin_amdgcn_global_load_lds(rec + s * 16, stage + s * 64, 16, 0, 0);
    }
}

// The ring loop of xg_loop over R stages with every wave loading two slots;
// compute(stage) runs the wave's regions on one k-block.
template <int R, typename C>
__device__ __forceinline__ void xc_loop(const uint4 *spec, int K, int a_pad, int f, int kb0, int kb1, int wave,
                                        uint4 *const (&st)[R], C &&compute) {
    constexpr int kPer = 2;
    const int last = kb1 - 1;
#pragma unroll
    for (int s = 0; s + 1 < R; ++s) xc_issue(spec, K, a_pad, f, min(kb0 + s, last), st[s], wave);
    int kb = kb0;
#pragma unroll 1
    for (; kb + R <= kb1; kb += R) {
#pragma unroll
        for (int s = 0; s < R; ++s) {
            wait_vm_lgkm0((R - 2) * kPer);
            __builtin_amdgcn_s_barrier();
            xc_issue(spec, K, a_pad, f, min(kb + s + R - 1, last), st[(s + R - 1) % R], wave);
            compute(st[s]);
        }
    }
#pragma unroll
    for (int s = 0; s + 1 < R; ++s) {
        if (kb + s < kb1) {
            wait_vm_lgkm0((R - 2 - s) * kPer);
            __builtin_amdgcn_s_barrier();
            compute(st[s]);
        }
    }
    wait_vm_lgkm0(0);
}

// Writes one region's accumulators as partials (upper triangle, a <= b < N).
template <int PREC, int NJ = 4>
__device__ __forceinline__ void xc_store(const XArgs &a, int64_t obase, int I0, int J0, bool dreg,
                                         typename AccT<PREC>::type (&accR)[4][NJ],
                                         typename AccT<PREC>::type (&accI)[4][NJ]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int J = 0; J < NJ; ++J) {
            if (dreg && J < I) continue;
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

// The off-diagonal half region of wave w < 4 (its first row and column
// block) and the off-diagonal region of wave w >= 4.
__device__ __forceinline__ int2 xc_half(int w) { return make_int2(w < 2 ? 0 : 8, (w < 2 ? 4 : 12) + 2 * (w & 1)); }
__device__ __forceinline__ int2 xc_off(int w) { return make_int2(w < 6 ? 0 : 4, (w & 1) ? 12 : 8); }

// fp32 (three-product form) whole-channel groups: the same stages and wave
// roles, each wave's regions in XRegion accumulators fed from the stage, so
// every pair is summed in the same order as by the per-wave regions.  The
// off-diagonal 4x4 regions' 48 accumulators need 460 registers with their
// own double-buffered loads (one wave per SIMD); fed from LDS, a wave fits
// in 242, two per SIMD.
template <int R>
__device__ __forceinline__ void x_chan_f32(const XArgs &a, int unit, uint4 *const (&st)[R], float *tb) {
    if (unit >= a.K * a.nsplit) return;  // the whole workgroup
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int f = unit % a.K, sp = unit / a.K;
    const int kb0 = (int)((int64_t)sp * a.nkb / a.nsplit);
    const int kb1 = (int)((int64_t)(sp + 1) * a.nkb / a.nsplit);
    const int64_t obase = ((int64_t)sp * a.K + f) * a.nb;
    float *tbw = tb + wave * 16 * 17;
    if (wave < 4) {
        const int rD = 4 * wave;
        const int2 h = xc_half(wave);
        XRegion<kFP32, 4, true> D;
        XRegion<kFP32, 4, false, 2> H;
        D.zero();
        H.zero();
        if (kb0 < kb1)
            xc_loop(a.spec, a.K, a.a_pad, f, kb0, kb1, wave, st, [&](const uint4 *stg) {
                uint4 p[4], q[2];
#pragma unroll
                for (int I = 0; I < 4; ++I) p[I] = stg[(rD + I) * 64 + lane];
                D.add(p, p);
                // one region's operands at a time
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int I = 0; I < 4; ++I) p[I] = stg[(h.x + I) * 64 + lane];
#pragma unroll
                for (int J = 0; J < 2; ++J) q[J] = stg[(h.y + J) * 64 + lane];
                H.add(p, q);
            });
        D.store(a.partial, obase, a.N, rD, rD, tbw);
        H.store(a.partial, obase, a.N, h.x, h.y, tbw);
    } else {
        const int2 o = xc_off(wave);
        XRegion<kFP32, 4, false> X;
        X.zero();
        if (kb0 < kb1)
            xc_loop(a.spec, a.K, a.a_pad, f, kb0, kb1, wave, st, [&](const uint4 *stg) {
                uint4 pr[4], pc[4];
#pragma unroll
                for (int I = 0; I < 4; ++I) pr[I] = stg[(o.x + I) * 64 + lane];
#pragma unroll
                for (int J = 0; J < 4; ++J) pc[J] = stg[(o.y + J) * 64 + lane];
                X.add(pr, pc);
            });
        X.store(a.partial, obase, a.N, o.x, o.y, tbw);
    }
}

template <int PREC, int R>
__device__ __forceinline__ void x_chan(const XArgs &a, int unit, uint4 *const (&st)[R]) {
    typedef typename AccT<PREC>::type acc_t;
    if (unit >= a.K * a.nsplit) return;  // the whole workgroup
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int f = unit % a.K, sp = unit / a.K;
    const int kb0 = (int)((int64_t)sp * a.nkb / a.nsplit);
    const int kb1 = (int)((int64_t)(sp + 1) * a.nkb / a.nsplit);
    const int64_t obase = ((int64_t)sp * a.K + f) * a.nb;
    const uint4 *spec = a.spec;
    const int K = a.K, a_pad = a.a_pad;
    if (wave < 4) {
        const int rD = 4 * wave;
        const int2 h = xc_half(wave);
        acc_t dR[4][4], dI[4][4], hR[4][2], hI[4][2];
#pragma unroll
        for (int I = 0; I < 4; ++I) {
#pragma unroll
            for (int J = 0; J < 4; ++J) dR[I][J] = dI[I][J] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int J = 0; J < 2; ++J) hR[I][J] = hI[I][J] = acc_t{0, 0, 0, 0};
        }
        if (kb0 < kb1)
            xc_loop(spec, K, a_pad, f, kb0, kb1, wave, st, [&](const uint4 *stg) {
                xg_compute<PREC, true>(stg, rD, rD, dR, dI);
                // one region's operands at a time
                __builtin_amdgcn_sched_barrier(0);
                xg_compute<PREC, false, 2>(stg, h.x, h.y, hR, hI);
            });
        xc_store<PREC>(a, obase, rD, rD, true, dR, dI);
        xc_store<PREC, 2>(a, obase, h.x, h.y, false, hR, hI);
    } else {
        const int2 o = xc_off(wave);
        acc_t aR[4][4], aI[4][4];
#pragma unroll
        for (int I = 0; I < 4; ++I)
#pragma unroll
            for (int J = 0; J < 4; ++J) aR[I][J] = aI[I][J] = acc_t{0, 0, 0, 0};
        if (kb0 < kb1)
            xc_loop(spec, K, a_pad, f, kb0, kb1, wave, st,
                    [&](const uint4 *stg) { xg_compute<PREC, false>(stg, o.x, o.y, aR, aI); });
        xc_store<PREC>(a, obase, o.x, o.y, false, aR, aI);
    }
}

// A workgroup's share of the X-stage with LDS-staged groups: unit = group
// (fastest), channel, split.  Wave w takes the group's region w.  int8 and
// fp16 (P / Q form) only.
template <int PREC>
__device__ __forceinline__ void x_group(const XArgs &a, int unit, uint4 *const (&st)[kXRing]) {
    typedef typename AccT<PREC>::type acc_t;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (unit >= a.ngroups * a.K * a.nsplit) return;  // the whole workgroup
    const XGroup &gr = a.groups[unit % a.ngroups];
    const int rest = unit / a.ngroups;
    const int f = rest % a.K;
    const int sp = rest / a.K;
    const int kb0 = (int)((int64_t)sp * a.nkb / a.nsplit);
    const int kb1 = (int)((int64_t)(sp + 1) * a.nkb / a.nsplit);
    // the group's fields once, into registers (read inside the loop they would
    // be loads the k-block waits would have to cover)
    const int r0 = gr.r0, c0 = gr.c0, gdiag = gr.diag;
    const bool active = wave < gr.nreg;
    const int I0 = active ? gr.reg[wave].x : 0, J0 = active ? gr.reg[wave].y : 0;
    const bool dreg = active && gr.kind[wave];
    const int rs = I0 - r0;
    const int cs = gdiag ? J0 - r0 : 8 + (J0 - c0);
    const uint4 *spec = a.spec;
    const int K = a.K, a_pad = a.a_pad;
    acc_t accR[4][4], accI[4][4];
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int J = 0; J < 4; ++J) accR[I][J] = accI[I][J] = acc_t{0, 0, 0, 0};
    if (kb0 < kb1) {
        if (gdiag) {
            if (dreg)
                xg_loop<PREC, true, 8>(spec, K, a_pad, r0, c0, f, kb0, kb1, wave, rs, cs, active, st, accR, accI);
            else
                xg_loop<PREC, false, 8>(spec, K, a_pad, r0, c0, f, kb0, kb1, wave, rs, cs, active, st, accR, accI);
        } else {
            xg_loop<PREC, false, 16>(spec, K, a_pad, r0, c0, f, kb0, kb1, wave, rs, cs, active, st, accR, accI);
        }
    }
    if (!active) return;
    // accumulator element v of lane l is row 4*(l/16)+v, column l%16
    const int64_t obase = ((int64_t)sp * a.K + f) * a.nb;
#pragma unroll
    for (int I = 0; I < 4; ++I)
#pragma unroll
        for (int J = 0; J < 4; ++J) {
            if (dreg && J < I) continue;
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

// ------------------------------------------------------------------ int16
// The 16-bit form (the paper's short complex type) on the int8 MFMA.  Each
// value is q = 255 h + l with digits h, l in [-127, 127], so
//     sum q_a q_b = 65025 sum h_a h_b + 255 sum (h_a l_b + l_a h_b) + sum l_a l_b,
// every digit sum exact in int32, combined exactly at the end.  A record
// holds 4 spectra as [h re x4][h im x4][l re x4][l im x4]; one MFMA operand
// (16 bytes per lane) takes the digits of two consecutive records, so a step
// covers 8 records (two k-blocks) and lane group g reads records 2g, 2g + 1.
// Digit negation is exact, so Q = [im | -re] is formed digit-wise as for
// int8.  Six accumulators per block pair: Re and Im of (hh, hl + lh, ll).
template <int RB, bool DIAG>
__device__ __forceinline__ void x_wave16(const XArgs &a, int wave) {
    const int lane = threadIdx.x & 63;
    if (wave >= a.nregions * a.K * a.nsplit) return;
    const int reg = wave % a.nregions;
    const int rest = wave / a.nregions;
    const int f = rest % a.K;
    const int sp = rest / a.K;
    const int I0 = a.regions[reg].x, J0 = a.regions[reg].y;
    // steps of two k-blocks (a.nkb is even for this form)
    const int nst = a.nkb / 2;
    const int st0 = (int)((int64_t)sp * nst / a.nsplit);
    const int st1 = (int)((int64_t)(sp + 1) * nst / a.nsplit);
    i32x4 rhh[RB][RB], rx[RB][RB], rll[RB][RB], ihh[RB][RB], ix[RB][RB], ill[RB][RB];
#pragma unroll
    for (int I = 0; I < RB; ++I)
#pragma unroll
        for (int J = 0; J < RB; ++J)
            rhh[I][J] = rx[I][J] = rll[I][J] = ihh[I][J] = ix[I][J] = ill[I][J] = i32x4{0, 0, 0, 0};
    // lane (row r, group g): records tq = 8 step + 2 g and + 1 of antenna 16 I + r
    const uint4 *base = a.spec + (int64_t)f * kTQB * a.a_pad + (2 * (lane >> 4)) * a.a_pad + (lane & 15);
    const int64_t bstride = (int64_t)a.K * kTQB * a.a_pad;
    auto mm = [](i32x4 &acc, uint4 x, uint4 y) {
        const i32x4 av = {(int)x.x, (int)x.y, (int)x.z, (int)x.w};
        const i32x4 bv = {(int)y.x, (int)y.y, (int)y.z, (int)y.w};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv, acc, 0, 0, 0);
    };
    for (int st = st0; st < st1; ++st) {
        // step st: time block st / 2, records 8 (st % 2) .. + 7
        const uint4 *rec = base + (st >> 1) * bstride + (st & 1) * 8 * a.a_pad;
        uint4 ph[RB], pl[RB], qh[RB], ql[RB], ch[RB], cl[RB];
#pragma unroll
        for (int I = 0; I < RB; ++I) {
            const uint4 r0 = rec[(I0 + I) * 16], r1 = rec[(I0 + I) * 16 + a.a_pad];
            ph[I] = make_uint4(r0.x, r0.y, r1.x, r1.y);
            pl[I] = make_uint4(r0.z, r0.w, r1.z, r1.w);
            qh[I] = make_uint4(r0.y, neg_i8x4(r0.x), r1.y, neg_i8x4(r1.x));
            ql[I] = make_uint4(r0.w, neg_i8x4(r0.z), r1.w, neg_i8x4(r1.z));
        }
        if constexpr (!DIAG) {
#pragma unroll
            for (int J = 0; J < RB; ++J) {
                const uint4 r0 = rec[(J0 + J) * 16], r1 = rec[(J0 + J) * 16 + a.a_pad];
                ch[J] = make_uint4(r0.x, r0.y, r1.x, r1.y);
                cl[J] = make_uint4(r0.z, r0.w, r1.z, r1.w);
            }
        }
#pragma unroll
        for (int I = 0; I < RB; ++I)
#pragma unroll
            for (int J = 0; J < RB; ++J) {
                if (DIAG && J < I) continue;
                const uint4 bh = DIAG ? ph[J] : ch[J], bl = DIAG ? pl[J] : cl[J];
                mm(rhh[I][J], ph[I], bh);
                mm(rx[I][J], ph[I], bl);
                mm(rx[I][J], pl[I], bh);
                mm(rll[I][J], pl[I], bl);
                mm(ihh[I][J], qh[I], bh);
                mm(ix[I][J], qh[I], bl);
                mm(ix[I][J], ql[I], bh);
                mm(ill[I][J], ql[I], bl);
            }
    }
    // accumulator element v of lane l is row 4*(l/16)+v, column l%16
    const int64_t obase = ((int64_t)sp * a.K + f) * a.nb;
    double2 *out = reinterpret_cast<double2 *>(a.partial);
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
                    const int64_t re = 65025ll * rhh[I][J][v] + 255ll * rx[I][J][v] + (int64_t)rll[I][J][v];
                    const int64_t im = 65025ll * ihh[I][J][v] + 255ll * ix[I][J][v] + (int64_t)ill[I][J][v];
                    out[obase + bl] = make_double2((double)re, ia == ib ? 0.0 : (double)im);
                }
            }
        }
}

}  // namespace
}  // namespace corr
