// F-stage of the FX correlator: unpack 4-bit samples, 2K-point real FFT,
// corner turn to channel-major records, conversion to the X-stage precision.
//
// What is computed (Section 1, Section 4 of Prasad & Subrahmanya): for each
// spectrum s and antenna a, X[s,a,k] = sum_n x[n] exp(-2 pi i k n / 2K),
// k = 0..K-1, forward and unnormalised, no window.
//
// How (gfx950): the 2K real samples of a block are read as K complex values
// z[m] = x[2m] + i x[2m+1] -- one byte of the frame is exactly one z[m], low
// nibble the real part.  A K-point complex FFT runs as Stockham passes of
// radix 16 (then 8, 4 or 2) over a padded LDS slot, 16 points per lane and
// K/16 lanes per transform, so every exchange inside one transform stays in
// one wavefront.  The real-input spectrum follows from Z[q] and Z[K-q]:
//   X[q] = (Z[q] + conj Z[K-q])/2 - (i/2) W_2K^q (Z[q] - conj Z[K-q]).
// Twiddles come from a host table with exact 0, +-1 and +-sqrt(1/2) entries,
// and the paths to bins 0 and K/2 only ever multiply by 1, so those two bins
// are exact (they are Gaussian integers).  A tile is TS consecutive spectra
// of GA consecutive antennas; its outputs are staged in LDS and written as
// 16-byte records [re x TS][im x TS], GA records (GA*16 bytes) contiguous
// per channel.  Power mode sums |X|^2 over the calibration window instead.
#pragma once
#include <type_traits>
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int kThreads = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kPowerTS = 2;
// antennas per power-mode tile: one round of transforms
constexpr int power_group(int M) { return (kThreads / (M / 16)) / kPowerTS; }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Every product-sum is written with explicit fmaf (the library is built with
// contraction off), so a transform rounds the same way in every kernel that
// inlines it and results do not depend on tile choices.
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(fmaf(a.x, w.x, -(a.y * w.y)), fmaf(a.x, w.y, a.y * w.x));
}
// -i * a
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// exact constants of the 16th roots of unity
constexpr float kC1 = 0.923879532511286756f;  // cos(pi/8)
constexpr float kS1 = 0.382683432365089772f;  // sin(pi/8)
constexpr float kR = 0.707106781186547524f;   // sqrt(1/2)

__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    float2 s13 = cadd(a1, a3), d13 = mul_mi(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}

// 16-point DFT as 4 x 4: x[4 n1 + n2], k = k1 + 4 k2; output in natural order.
__device__ __forceinline__ void dft16(float2 *v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[4 k1 + n2] = A[n2][k1]; multiply by W16^(n2 k1)
    v[5] = make_float2(fmaf(kC1, v[5].x, kS1 * v[5].y), fmaf(kC1, v[5].y, -(kS1 * v[5].x)));      // W^1
    v[6] = make_float2(kR * (v[6].x + v[6].y), kR * (v[6].y - v[6].x));                // W^2
    v[7] = make_float2(fmaf(kS1, v[7].x, kC1 * v[7].y), fmaf(kS1, v[7].y, -(kC1 * v[7].x)));      // W^3
    v[9] = make_float2(kR * (v[9].x + v[9].y), kR * (v[9].y - v[9].x));                // W^2
    v[10] = mul_mi(v[10]);                                                              // W^4
    v[11] = make_float2(kR * (v[11].y - v[11].x), -kR * (v[11].x + v[11].y));          // W^6
    v[13] = make_float2(fmaf(kS1, v[13].x, kC1 * v[13].y), fmaf(kS1, v[13].y, -(kC1 * v[13].x))); // W^3
    v[14] = make_float2(kR * (v[14].y - v[14].x), -kR * (v[14].x + v[14].y));          // W^6
    v[15] = make_float2(fmaf(-kC1, v[15].x, -(kS1 * v[15].y)), fmaf(kS1, v[15].x, -(kC1 * v[15].y))); // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // now v[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4 x 4 index
    float2 t[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] = v[4 * (k & 3) + (k >> 2)];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[k];
}

// 8-point DFT as 2 x 4: x[4 n1 + n2], k = k1 + 2 k2; output in natural order.
__device__ __forceinline__ void dft8(float2 *v) {
    float2 a[4][2];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        a[n2][0] = cadd(v[n2], v[4 + n2]);
        a[n2][1] = csub(v[n2], v[4 + n2]);
    }
    a[1][1] = make_float2(kR * (a[1][1].x + a[1][1].y), kR * (a[1][1].y - a[1][1].x));  // W8^1
    a[2][1] = mul_mi(a[2][1]);                                                            // W8^2
    a[3][1] = make_float2(kR * (a[3][1].y - a[3][1].x), -kR * (a[3][1].x + a[3][1].y));  // W8^3
#pragma unroll
    for (int k1 = 0; k1 < 2; ++k1) {
        dft4(a[0][k1], a[1][k1], a[2][k1], a[3][k1]);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 2 * k2] = a[k2][k1];
    }
}

template <int R>
__device__ __forceinline__ void dft_r(float2 *v) {
    if constexpr (R == 16) dft16(v);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else dft2(v[0], v[1]);
}

// LDS index with one float2 of padding every 16 (bank spreading)
__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }


// Stockham pass of radix R (p = product of the radices before it), in place
// in one transform's LDS slot.  Butterfly i reads z[i + r M/R], multiplies by
// W_{pR}^{r k} (k = i mod p), and writes z[(i - k) R + k + r p].  The lane's
// twiddles come in registers, tw[m (R-1) + r - 1] for its butterfly m.
template <int M, int R>
__device__ __forceinline__ void fft_pass(float2 *z, int j, int p, const float2 *tw) {
    constexpr int L = M / 16;
    constexpr int T = M / R;
    constexpr int NBF = 16 / R;
    float2 v[16];
#pragma unroll
    for (int m = 0; m < NBF; ++m) {
        const int i = j + L * m;
#pragma unroll
        for (int r = 0; r < R; ++r) v[m * R + r] = z[pad(i + r * T)];
    }
    wave_lds_sync();  // every read of this pass precedes every write
#pragma unroll
    for (int m = 0; m < NBF; ++m) {
        const int i = j + L * m;
        const int k = i & (p - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) v[m * R + r] = cmul(v[m * R + r], tw[m * (R - 1) + r - 1]);
        dft_r<R>(&v[m * R]);
        const int base = (i - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) z[pad(base + r * p)] = v[m * R + r];
    }
}

// The twiddles lane j needs in a pass of radix R after p points: W_M^(r k
// M/(pR)) for each of its butterflies m (k = (j + L m) mod p) and r = 1..R-1.
template <int M, int R>
__device__ __forceinline__ void pass_twiddles(int j, int p, const float2 *twM, float2 *out) {
    constexpr int L = M / 16;
#pragma unroll
    for (int m = 0; m < 16 / R; ++m) {
        const int k = (j + L * m) & (p - 1);
        const int step = k * (M / (p * R));
#pragma unroll
        for (int r = 1; r < R; ++r) out[m * (R - 1) + r - 1] = twM[(r * step) & (M - 1)];
    }
}

// A lane's twiddles for every pass after the first: radix 16 (8 for M = 128)
// after 16 points, then radix 2 (M = 512) or 4 (M = 1024) after 256.  They
// depend only on the lane, so a workgroup loads them once.  (M = 256 runs on
// the matrix cores and holds their operands instead.)
template <int M>
struct PassTw {
    static constexpr int R2 = M == 128 ? 8 : 16;
    static constexpr int R3 = M == 512 ? 2 : (M == 1024 ? 4 : 1);
    static constexpr int N2 = (16 / R2) * (R2 - 1);
    static constexpr int N3 = R3 > 1 ? (16 / R3) * (R3 - 1) : 1;
    float2 w2[N2];
    float2 w3[N3];
    __device__ __forceinline__ void load(int j, const float2 *twM) {
        pass_twiddles<M, R2>(j, 16, twM, w2);
        if constexpr (R3 > 1) pass_twiddles<M, R3>(j, 256, twM, w3);
    }
};

// The 256-point transform on the matrix cores.  With z[16 s + f] (s, f < 16)
//   Y[f][c]     = sum_s W16^(s c) z[16 s + f],
//   Y'[f][c]    = W256^(f c) Y[f][c],
//   Z[c + 16 d] = sum_f W16^(f d) Y'[f][c],
// both 16-point DFTs are real 16 x 32 by 32 x 16 products, one transform per
// wavefront at a time, on v_mfma_f32_16x16x32_f16: lane (j = lane mod 16,
// g = lane / 16) holds row j of the left operand and column j of the right
// one over contraction positions 8g .. 8g + 7, i.e. the real parts of points
// 4g .. 4g + 3, then their imaginary parts, and gets rows 4g + i of column j
// of the result.  The real form of
// W16 in that layout is the same register set in both products: the right
// operand of the first (contraction s, column c = j) and the left operand of
// the second (row d = j, contraction f).  Each DFT is summed from f16 halves,
// W16 = hi + lo and Y' = hi + lo, with the products of halves exact in the
// f32 accumulator; the dropped lo * lo terms and the rounding of the lo
// halves are of order 2^-21 of the result.  The 4-bit samples are exact in
// f16.  Bins 0 and 128 see only the entries +-1 and 0 (hi exact, lo zero) and
// stay exact.  The first product's result is already the second one's right
// operand in the same lanes: no exchange between the passes.
//
// The 512-point transform is one radix-2 step (decimation in time) after two
// such transforms of the even and the odd samples, E and O:
//   Z[q] = E[q] + W512^q O[q],  Z[q + 256] = E[q] - W512^q O[q],  q < 256,
// where lane (j, g) already holds E and O at the same q = j + 16 (4g + i).
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// The matrix-core transform serves the reduced-precision records at 256 and
// 512 points, where the F-stage is bound by vector work.  The float32 records
// (bound by their HBM writes, where it measured a few percent slower) and the
// calibration power sums keep the vector transform.
template <int M, int PREC> constexpr bool mfma_fft() { return (M == 256 || M == 512) && PREC != kFP32; }

template <int M>
struct MfmaFft {
    static constexpr int P = M / 256;  // 256-point transforms per block
    h8_t dh[2], dl[2];  // W16, real form: [0] real outputs, [1] imaginary outputs
    float2 w[4];        // W256^(f c), f = 4g + i, c = j
    float2 w2[P == 2 ? 4 : 1];  // W512^q, q = j + 16 (4g + i)
    uint32_t sel01[P], sel23[P];
    // -1, opaque to the optimizer: a known -1 turns the product of the
    // split's fma into a subtraction, which has no mixed-precision form
    float m1;
    __device__ __forceinline__ void load(int, const float2 *twM) {
        const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
        m1 = -1.0f;
        asm volatile("" : "+v"(m1));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = 4 * g + i;
            // twM[e] = exp(-2 pi i e / M) = (cos t, -sin t); the real form of
            // multiplication by it is [cos t, sin t] -> re, [-sin t, cos t] -> im
            const float2 t = twM[((s * j) & 15) * (M / 16)];
            const float v[2][2] = {{t.x, -t.y}, {t.y, t.x}};
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const _Float16 h = (_Float16)v[b][c];
                    dh[b][4 * c + i] = h;
                    dl[b][4 * c + i] = (_Float16)(v[b][c] - (float)h);
                }
            w[i] = twM[((s * j) & 255) * (M / 256)];
            if constexpr (P == 2) w2[i] = twM[j + 16 * s];
        }
        // byte b of four dwords -> one dword: b = j mod 4 (256 points), or
        // 2 (j mod 2) + p for the even (p = 0) and odd (p = 1) samples
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t b = P == 1 ? (j & 3) : 2 * (j & 1) + p;
            sel01[p] = b | (b + 4) << 8 | 0x0c0c0000u;
            sel23[p] = 0x0c0cu | b << 16 | (b + 4) << 24;
        }
    }
};

__device__ __forceinline__ f4_t mfma_h(h8_t a, h8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// 256 points, the lane's four samples z[16 (4g + i) + j] packed one per byte
// of p, to the lane's four outputs Z[j + 16 (4g + i)] (zr, zi).
template <int M>
__device__ __forceinline__ void dft256_mfma(uint32_t p, const MfmaFft<M> &k, f4_t &zr, f4_t &zi) {
    // offset nibbles u = n + 8 as 1024 + u in f16 (byte u under the exponent
    // byte 0x64), then minus 1032: exact.  Real parts are the low nibbles.
    const uint32_t t = p ^ 0x88888888u;
    const uint32_t lo = t & 0x0f0f0f0fu, hi = (t >> 4) & 0x0f0f0f0fu;
    const uint32_t bits[4] = {__builtin_amdgcn_perm(0x64646464u, lo, 0x04010400u),
                              __builtin_amdgcn_perm(0x64646464u, lo, 0x04030402u),
                              __builtin_amdgcn_perm(0x64646464u, hi, 0x04010400u),
                              __builtin_amdgcn_perm(0x64646464u, hi, 0x04030402u)};
    h8_t a;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const h2_t v = __builtin_bit_cast(h2_t, bits[w]) - h2_t{(_Float16)1032.0f, (_Float16)1032.0f};
        a[2 * w] = v[0];
        a[2 * w + 1] = v[1];
    }
    const f4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f4_t yr = mfma_h(a, k.dl[0], zero), yi = mfma_h(a, k.dl[1], zero);
    yr = mfma_h(a, k.dh[0], yr);
    yi = mfma_h(a, k.dh[1], yi);
    float2 y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = cmul(make_float2(yr[i], yi[i]), k.w[i]);
    // hi: y rounded toward zero to f16, i.e. cut to 11 significant bits
    // (below 2^-14 the cut is coarser, by at most 2^-24), lo = y - hi, exact
    // in the f32 arithmetic of the mixed-precision fma, rounded to f16; real
    // parts at positions 0-3, imaginary parts at 4-7
    h8_t bh, bl;
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
        const h2_t hr = __builtin_bit_cast(h2_t, __builtin_amdgcn_cvt_pkrtz(y[i].x, y[i + 1].x));
        const h2_t hm = __builtin_bit_cast(h2_t, __builtin_amdgcn_cvt_pkrtz(y[i].y, y[i + 1].y));
        bh[i] = hr[0];
        bh[i + 1] = hr[1];
        bh[4 + i] = hm[0];
        bh[4 + i + 1] = hm[1];
        bl[i] = (_Float16)__builtin_fmaf((float)hr[0], k.m1, y[i].x);
        bl[i + 1] = (_Float16)__builtin_fmaf((float)hr[1], k.m1, y[i + 1].x);
        bl[4 + i] = (_Float16)__builtin_fmaf((float)hm[0], k.m1, y[i].y);
        bl[4 + i + 1] = (_Float16)__builtin_fmaf((float)hm[1], k.m1, y[i + 1].y);
    }
    zr = mfma_h(k.dl[0], bh, zero);
    zi = mfma_h(k.dl[1], bh, zero);
    zr = mfma_h(k.dh[0], bl, zr);
    zi = mfma_h(k.dh[1], bl, zi);
    zr = mfma_h(k.dh[0], bh, zr);
    zi = mfma_h(k.dh[1], bh, zi);
}

// The wavefront's T transforms of a round: bytes from the staging bb (dword
// d of a block at (d mod M/64) 16 + d div M/64, so that lane (j, g) finds the
// bytes it needs, z[16 s + j] (256) or z[32 s + 2j + p] (512) for s = 4g ..
// 4g + 3, at one byte of four consecutive dwords) to Z in slot z[t].  All
// reads come first and all writes last, so the transforms' products and
// vector work interleave.
template <int M, int T>
__device__ __forceinline__ void fft_mfma(const uint32_t *bb, float2 *const (&z)[T], const MfmaFft<M> &k) {
    constexpr int P = MfmaFft<M>::P;
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    uint4 w[T];
#pragma unroll
    for (int t = 0; t < T; ++t)
        w[t] = *reinterpret_cast<const uint4 *>(bb + t * (M / 4) + (j / (64 / (M / 16))) * 16 + 4 * g);
    f4_t zr[T][P], zi[T][P];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint32_t b = __builtin_amdgcn_perm(w[t].y, w[t].x, k.sel01[p]) |
                               __builtin_amdgcn_perm(w[t].w, w[t].z, k.sel23[p]);
            dft256_mfma<M>(b, k, zr[t][p], zi[t][p]);
        }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        if (z[t] == nullptr) continue;  // idle slot (wave-uniform)
        if constexpr (P == 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) z[t][pad(j + 16 * (4 * g + i))] = make_float2(zr[t][0][i], zi[t][0][i]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = j + 16 * (4 * g + i);
                const float2 e = make_float2(zr[t][0][i], zi[t][0][i]);
                const float2 o = cmul(make_float2(zr[t][1][i], zi[t][1][i]), k.w2[i]);
                z[t][pad(q)] = cadd(e, o);
                z[t][pad(q + 256)] = csub(e, o);
            }
        }
    }
}

// The per-lane constants of a transform of M points for records of PREC.
template <int M, int PREC>
using FftConsts = typename std::conditional<mfma_fft<M, PREC>(), MfmaFft<M>, PassTw<M>>::type;

// Signed nibble at bit offset `off` of w.
__device__ __forceinline__ float nib(uint32_t w, int off) {
    return (float)((int)(w << (28 - off)) >> 28);
}

// qm[t] = 1.5 * 2^23 + q[t] with q = clamp(rint(x[t] sc), -lim, lim).  One
// fused x sc + 1.5 * 2^23 rounds the exact product to the nearest integer
// (ties to even) and leaves it in the low bits of the sum (|x sc| < 2^22; a
// larger product lands beyond the clamp bounds, which the clamp then takes).
// The values share one scale sc > 0, so one can round past lim only if
// sc max|x| >= lim + 0.5, and the rounded product keeps that bound (never
// misses such a value).  The clamp, and the exact count of the values whose
// rounded magnitude exceeds lim (added to wsat, wave-uniform), run only in a
// wavefront where some lane reaches the bound, which saturation makes rare.
template <int NV>
__device__ __forceinline__ void quantise(const float (&x)[NV], float sc, float lim, unsigned &wsat,
                                         float (&qm)[NV]) {
    constexpr float kMagic = 12582912.0f;
    // max|x| as a chain of three-operand maxima (the NaN-propagating form
    // needs no canonicalised operands; the values here are finite)
    float m = 0.0f;
#pragma unroll
    for (int t = 0; t < NV; t += 2)
        m = __builtin_elementwise_maximum(__builtin_elementwise_maximum(m, fabsf(x[t])), fabsf(x[t + 1]));
#pragma unroll
    for (int t = 0; t < NV; ++t) qm[t] = __builtin_fmaf(x[t], sc, kMagic);
    if (__ballot(m * sc >= lim + 0.5f)) {
#pragma unroll
        for (int t = 0; t < NV; ++t) {
            wsat += (unsigned)__popcll(__ballot(fabsf(qm[t] - kMagic) > lim));
            qm[t] = __builtin_amdgcn_fmed3f(qm[t], kMagic - lim, kMagic + lim);
        }
    }
}

// Pack TS spectra of one (channel, antenna) into a 16-byte record
// [re x TS][im x TS] of the precision's type.  int8: the record holds
// q = clamp(rint(x sc), -127, 127), rounding to nearest even, with re[] and
// im[] here already multiplied by two and sc halved (both exact, so x sc is
// the same product); wsat (wave-uniform) counts the values whose rounded
// magnitude exceeds 127 (int16: 32512).
template <int PREC, int TS>
__device__ __forceinline__ uint4 make_record(const float *re, const float *im, float sc, unsigned &wsat) {
    uint4 out;
    if constexpr (PREC == kFP32) {
        static_assert(TS == 2, "fp32 record");
        out = make_uint4(__float_as_uint(re[0]), __float_as_uint(re[1]), __float_as_uint(im[0]),
                         __float_as_uint(im[1]));
    } else if constexpr (PREC == kFP16) {
        static_assert(TS == 4, "fp16 record");
        _Float16 h[8];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h[t] = (_Float16)re[t];
            h[4 + t] = (_Float16)im[t];
        }
        __builtin_memcpy(&out, h, 16);
    } else if constexpr (PREC == kINT16) {
        static_assert(TS == 4, "int16 record");
        // q = clamp(rint(x sc), -32512, 32512) as for int8, then the base-255
        // digits h = floor((q + 127.5) / 255), l = q - 255 h, both in
        // [-127, 127].  For an integer q that h is also the integer nearest
        // q / 255: q / 255 is never within 1/510 of a half-integer, and the
        // product by the rounded reciprocal is within 2^-17 of the quotient,
        // so adding 1.5 * 2^23 in the same fused operation rounds it to h
        // exactly and leaves h in the low bits.  The bits of 1.5 * 2^23 + x
        // are those of 1.5 * 2^23 plus x (an integer below 2^22), whose low
        // byte is zero; the low byte of the sum of the bits of q's and h's
        // biased floats is therefore (q + h) mod 256, which is
        // (q - 255 h) mod 256 = l mod 256, the byte the record holds.
        // Record: [h of re x4][h of im x4][l of re x4][l of im x4].
        constexpr float kMagic = 12582912.0f;
        uint32_t hb[8], lb[8];
        float x[8], qm[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = t < 4 ? re[t] : im[t - 4];
        quantise<8>(x, sc, (float)kI16Max, wsat, qm);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float hm = fmaf(qm[t] - kMagic, 1.0f / 255.0f, kMagic);
            hb[t] = __float_as_uint(hm);
            lb[t] = __float_as_uint(qm[t]) + __float_as_uint(hm);
        }
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const uint32_t *b = hb + 4 * k;
            w[k] = __builtin_amdgcn_perm(b[1], b[0], 0x0c0c0400u) | __builtin_amdgcn_perm(b[3], b[2], 0x04000c0cu);
            const uint32_t *c = lb + 4 * k;
            w[2 + k] = __builtin_amdgcn_perm(c[1], c[0], 0x0c0c0400u) | __builtin_amdgcn_perm(c[3], c[2], 0x04000c0cu);
        }
        out = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        static_assert(TS == 8, "int8 record");
        // the low byte of 1.5 * 2^23 + q is q as two's complement
        float x[16], qm[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = t < 8 ? re[t] : im[t - 8];
        quantise<16>(x, sc, 127.0f, wsat, qm);
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = __float_as_uint(qm[4 * k + t]);
            // low bytes of b[0..3] -> bytes 0..3 of the word
            w[k] = __builtin_amdgcn_perm(b[1], b[0], 0x0c0c0400u) | __builtin_amdgcn_perm(b[3], b[2], 0x04000c0cu);
        }
        out = make_uint4(w[0], w[1], w[2], w[3]);
    }
    return out;
}

// Real-input bins q and K-q (q = 0: bins 0 and K/2) from a transform slot;
// w = W_2K^q.  TWICE returns both bins multiplied by two (exact), which
// saves the halving where a scale follows.
template <int M, bool TWICE = false>
__device__ __forceinline__ void real_bins(const float2 *zs, int q, float2 w, float2 &xlo, float2 &xhi) {
    if (q == 0) {
        const float2 z0 = zs[0], zh = zs[pad(M / 2)];
        xlo = make_float2(z0.x + z0.y, 0.0f);
        xhi = make_float2(zh.x, -zh.y);
        if constexpr (TWICE) {
            xlo.x *= 2.0f;
            xhi = make_float2(2.0f * xhi.x, 2.0f * xhi.y);
        }
    } else {
        const float2 z0 = zs[pad(q)], z1 = zs[pad(M - q)];
        const float2 A = make_float2(z0.x + z1.x, z0.y - z1.y);
        const float2 B = make_float2(z0.x - z1.x, z0.y + z1.y);
        const float2 C = cmul(B, w);
        if constexpr (TWICE) {
            xlo = make_float2(A.x + C.y, A.y - C.x);
            xhi = make_float2(A.x - C.y, -A.y - C.x);
        } else {
            xlo = make_float2(0.5f * (A.x + C.y), 0.5f * (A.y - C.x));
            xhi = make_float2(0.5f * (A.x - C.y), 0.5f * (-A.y - C.x));
        }
    }
}

template <int M, int PREC, int GA, bool POWER>
struct FShape {
    static constexpr int L = M / 16;                  // lanes per transform
    static constexpr int FPR = kThreads / L;          // transforms per round
    static constexpr int SLOT = M + M / 16 + 1;       // padded float2 per transform
    static constexpr int TS = POWER ? kPowerTS : record_times(PREC);
    static constexpr int NF = TS * GA;                // transforms per tile
    static constexpr int ROUNDS = (NF + FPR - 1) / FPR;
    static constexpr int NTASK = (M / 2) * GA;        // (bin pair, antenna) tasks
    static constexpr int TPT = (NTASK + kThreads - 1) / kThreads;
    static constexpr int LDS = NF * SLOT * 8 + FPR * M;
};

// Frames of tile (tq, g): transform slot fi = r FPR + fs of round r takes the
// 16 bytes j of block (spectrum tq TS + fi / GA, antenna g GA + fi % GA);
// blocks past the chunk or past N are read from the zero bytes after the
// twiddle table.  Every lane issues its load and nothing selects on the data
// afterwards, so no branch or select ties a later wait to this load.
template <int M, int GA, int TS, int NF, int ROUNDS>
__device__ __forceinline__ void load_tile(const FArgs &args, int tq, int g, u32x4 (&raw)[ROUNDS]) {
    constexpr int L = M / 16, FPR = kThreads / L;
    const int fs = threadIdx.x / L, j = threadIdx.x % L;
    const uint8_t *zeros = reinterpret_cast<const uint8_t *>(args.tw + M + M / 2);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int fi = r * FPR + fs;
        const int s = tq * TS + fi / GA, a = g * GA + fi % GA;
        const bool ok = fi < NF && s < args.S && a < args.N;
        const uint8_t *src = ok ? args.in + ((int64_t)s * args.N + a) * M : zeros;
        // frames are read once: stream them past the caches
        raw[r] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src + 16 * j));
    }
}

// Transform the NF blocks of a tile, loaded by load_tile, into zbuf slots
// (ts * GA + ga).
template <int M, int PREC, int NF, int ROUNDS>
__device__ __forceinline__ void tile_ffts(const u32x4 (&raw)[ROUNDS], float2 *zbuf, uint32_t *bbuf,
                                          const FftConsts<M, PREC> &tw) {
    constexpr int L = M / 16, FPR = kThreads / L, SLOT = M + M / 16 + 1;
    const int fs = threadIdx.x / L, j = threadIdx.x % L;
    uint32_t *bb = bbuf + fs * (M / 4);
    // dword d of the block goes to (d mod L/4)*16 + d div L/4, so the 16
    // dwords pass 1 needs in a lane are contiguous
    auto stage = [&](const u32x4 &raw_r) {
        const uint32_t w[4] = {raw_r[0], raw_r[1], raw_r[2], raw_r[3]};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int d = 4 * j + c;
            bb[(d % (L / 4)) * 16 + d / (L / 4)] = w[c];
        }
    };
    if constexpr (mfma_fft<M, PREC>()) {
        // Every lane takes part (the matrix products need the whole
        // wavefront): the bytes of idle slots are the zero page's, and the
        // wavefront runs its own slots of the round one at a time.
        constexpr int W = 64 / L;
        const int f0 = (threadIdx.x >> 6) * W;
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            stage(raw[r]);
            wave_lds_sync();
            float2 *z[W];
#pragma unroll
            for (int t = 0; t < W; ++t) {
                const int ft = r * FPR + f0 + t;
                z[t] = (NF % FPR == 0 || ft < NF) ? zbuf + ft * SLOT : nullptr;
            }
            fft_mfma<M, W>(bbuf + f0 * (M / 4), z, tw);
            wave_lds_sync();
        }
    } else {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int fi = r * FPR + fs;
            if (NF < FPR && fi >= NF) break;  // idle transform slots (one round only)
            float2 *z = zbuf + fi * SLOT;
            stage(raw[r]);
            wave_lds_sync();
            // pass 1: radix 16 over z[j + r L], unpacked from the bytes
            {
                float2 v[16];
                const uint4 *src = reinterpret_cast<const uint4 *>(bb + (j / 4) * 16);
                const int off = 8 * (j & 3);
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const uint4 w4 = src[q4];
                    const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const uint32_t byte = w[c] >> off;
                        v[4 * q4 + c] = make_float2(nib(byte, 0), nib(byte, 4));
                    }
                }
                dft16(v);
#pragma unroll
                for (int q = 0; q < 16; ++q) z[pad(16 * j + q)] = v[q];
            }
            wave_lds_sync();
            fft_pass<M, PassTw<M>::R2>(z, j, 16, tw.w2);
            if constexpr (PassTw<M>::R3 > 1) {
                wave_lds_sync();
                fft_pass<M, PassTw<M>::R3>(z, j, 256, tw.w3);
            }
            wave_lds_sync();
        }
    }
}

// Per-workgroup constants of a records tile loop: every pass twiddle of the
// lane and W_2M^q of the thread's bin pairs (task t = bin pair q, antenna ga).
template <int M, int PREC, int GA>
struct TileConsts {
    using Sh = FShape<M, PREC, GA, false>;
    FftConsts<M, PREC> ptw;
    float2 bw[Sh::TPT];
    __device__ __forceinline__ void load(const FArgs &args) {
        const int tid = threadIdx.x;
        ptw.load(tid % (M / 16), args.tw);
#pragma unroll
        for (int it = 0; it < Sh::TPT; ++it) {
            const int t = tid + it * kThreads;
            bw[it] = (Sh::NTASK % kThreads == 0 || t < Sh::NTASK) ? args.tw[M + t / GA] : make_float2(1.0f, 0.0f);
        }
    }
};

// int8 scales of the thread's bin pairs in antenna group g, halved.  The loads are
// unconditional, as in load_tile; antennas past N have zero spectra and take
// antenna 0's scales.
template <int M, int PREC, int GA>
__device__ __forceinline__ void tile_scales(const FArgs &args, int g, float *slo, float *shi) {
    using Sh = FShape<M, PREC, GA, false>;
#pragma unroll
    for (int it = 0; it < Sh::TPT; ++it) {
        slo[it] = shi[it] = 1.0f;
        if constexpr (is_quant(PREC)) {
            const int t = threadIdx.x + it * kThreads;
            const bool ok = (Sh::NTASK % kThreads == 0 || t < Sh::NTASK) && g * GA + t % GA < args.N;
            const int a = ok ? g * GA + t % GA : 0, q = ok ? t / GA : 0;
            // halved: the bins come doubled (real_bins<M, true>)
            slo[it] = 0.5f * args.scales[(int64_t)a * M + q];
            shi[it] = 0.5f * args.scales[(int64_t)a * M + (q == 0 ? M / 2 : M - q)];
        }
    }
}

// Delay and phase tracking (Section 2.1: a phase applied to each subband
// before accumulation in time): channel ch of spectra s0 .. s0 + TS - 1 of
// one antenna, with model m = (delay, delay rate, phase, phase rate), is
// multiplied by exp(2 pi i rho), rho = ch (m.x + m.y s) / 2M + m.z + m.w s
// turns.  The phase of spectrum s0 and the step from one spectrum to the
// next are formed in double and reduced to [-1/2, 1/2] turns, so long
// integrations and large delays lose nothing to the argument's size; the
// hardware sine and cosine take turns; the record's later spectra follow by
// complex multiplication by the step (at most 7 steps).
template <int M, int TS>
__device__ __forceinline__ void track_rotate(const double4 &m, int ch, int s0, float *re, float *im) {
    const double kf = (double)ch * (1.0 / (2.0 * M));
    const double nu = fma(kf, m.y, m.w);
    const double rb = fma((double)s0, nu, fma(kf, m.x, m.z));
    const float fb = (float)(rb - rint(rb));
    float c = __builtin_amdgcn_cosf(fb), sn = __builtin_amdgcn_sinf(fb);
    float cs = 1.0f, ss = 0.0f;
    if constexpr (TS > 1) {
        const float fs = (float)(nu - rint(nu));
        cs = __builtin_amdgcn_cosf(fs);
        ss = __builtin_amdgcn_sinf(fs);
    }
#pragma unroll
    for (int ts = 0; ts < TS; ++ts) {
        const float x = re[ts], y = im[ts];
        re[ts] = x * c - y * sn;
        im[ts] = x * sn + y * c;
        if (ts + 1 < TS) {
            const float c2 = c * cs - sn * ss;
            sn = c * ss + sn * cs;
            c = c2;
        }
    }
}

// One tile (time record tq, antenna group g) of records from frames already
// loaded: TS spectra of GA antennas transformed, turned into bins, rotated by
// the tracking model trk of the thread's antenna (TRACK) and written as
// records.  The caller separates consecutive tiles with a barrier.
template <int M, int PREC, int GA, bool TRACK = false>
__device__ __forceinline__ void tile_records(const FArgs &args, int tq, int g,
                                             const u32x4 (&cur)[FShape<M, PREC, GA, false>::ROUNDS],
                                             const TileConsts<M, PREC, GA> &k, const float *slo, const float *shi,
                                             unsigned &wsat, float2 *zbuf, uint32_t *bbuf,
                                             const double4 &trk = double4{0, 0, 0, 0}) {
    using Sh = FShape<M, PREC, GA, false>;
    constexpr int TS = Sh::TS, SLOT = Sh::SLOT, NTASK = Sh::NTASK, TPT = Sh::TPT;
    const int tid = threadIdx.x;
    // The tile's records lie in one time block of `span` bytes, addressed
    // through a buffer resource.  Padding antennas that fill whole 128-byte
    // lines (8 records, from N rounded up to 8) are never stored: the buffer
    // is cleared when it is allocated, so their records stay zero.  Their
    // stores go to offset `span`, past the resource's range, where the
    // hardware drops them; no branch is needed (and the allocation has slack
    // beyond the last block, so that offset lies inside it in any case).
    // Padding that shares a line with real antennas is stored (as zeros): a
    // half-written line costs a read of the line to merge it.
    const int n_store = (args.N + 7) & ~7;
    const int tqb = __builtin_amdgcn_readfirstlane(tq / kTQB);
    const uint32_t span = (uint32_t)M * kTQB * (uint32_t)args.a_pad * kRecordBytes;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        args.spec + (int64_t)tqb * M * kTQB * args.a_pad, 0, (int)span, kBufferRsrcFlags);
    tile_ffts<M, PREC, Sh::NF, Sh::ROUNDS>(cur, zbuf, bbuf, k.ptw);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < TPT; ++it) {
        const int t = tid + it * kThreads;
        if (NTASK % kThreads != 0 && t >= NTASK) break;
        const int ga = t % GA, q = t / GA;
        const int a = g * GA + ga;
        float lr[TS], li[TS], hr[TS], hi[TS];
#pragma unroll
        for (int ts = 0; ts < TS; ++ts) {
            float2 xlo, xhi;
            real_bins<M, is_quant(PREC)>(zbuf + (ts * GA + ga) * SLOT, q, k.bw[it], xlo, xhi);
            lr[ts] = xlo.x; li[ts] = xlo.y; hr[ts] = xhi.x; hi[ts] = xhi.y;
        }
        const int clo = q, chi = q == 0 ? M / 2 : M - q;
        if constexpr (TRACK) {
            const int s0 = args.s_base + tq * TS;
            track_rotate<M, TS>(trk, clo, s0, lr, li);
            track_rotate<M, TS>(trk, chi, s0, hr, hi);
        }
        const uint4 rlo = make_record<PREC, TS>(lr, li, slo[it], wsat);
        const uint4 rhi = make_record<PREC, TS>(hr, hi, shi[it], wsat);
        const uint32_t row = (uint32_t)(tq % kTQB) * args.a_pad + a;
        const bool stored = a < n_store;
        const uint32_t olo = stored ? ((uint32_t)clo * kTQB * args.a_pad + row) * kRecordBytes : span;
        const uint32_t ohi = stored ? ((uint32_t)chi * kTQB * args.a_pad + row) * kRecordBytes : span;
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{rlo.x, rlo.y, rlo.z, rlo.w}, rs, olo, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{rhi.x, rhi.y, rhi.z, rhi.w}, rs, ohi, 0, 0);
    }
}

// Tiles t0, t0 + stride, ... below t1 of spectra records; tile = time record
// tq * ngroups + antenna group g.  The next tile's frames are read while the
// current one is transformed, and the twiddles are loaded once, so neither
// latency sits between a tile's stages.
template <int M, int PREC, int GA>
__device__ __forceinline__ void f_tiles(const FArgs &args, int t0, int stride, int t1, float2 *zbuf,
                                        uint32_t *bbuf) {
    using Sh = FShape<M, PREC, GA, false>;
    constexpr int TS = Sh::TS, NF = Sh::NF, ROUNDS = Sh::ROUNDS, TPT = Sh::TPT;
    if (t0 >= t1) return;
    TileConsts<M, PREC, GA> k;
    k.load(args);
    u32x4 raw[ROUNDS];
    load_tile<M, GA, TS, NF, ROUNDS>(args, t0 / args.ngroups, t0 % args.ngroups, raw);
    // Wait for the first frames here, before the loop: otherwise the wait at
    // the loop head, which must also cover this path, is a wait for every
    // memory operation, and each tile would wait for the previous tile's
    // record stores to land.  (vmcnt(0), expcnt and lgkmcnt left alone.)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    unsigned wsat = 0;  // saturated int8 values of this wave
    for (int tile = t0; tile < t1; tile += stride) {
        const int tq = tile / args.ngroups, g = tile % args.ngroups;
        float slo[TPT], shi[TPT];
        tile_scales<M, PREC, GA>(args, g, slo, shi);
        u32x4 cur[ROUNDS];
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) cur[r] = raw[r];
        // the last tile re-reads its own frames rather than branch around the load
        const int nxt = tile + stride < t1 ? tile + stride : tile;
        load_tile<M, GA, TS, NF, ROUNDS>(args, nxt / args.ngroups, nxt % args.ngroups, raw);
        tile_records<M, PREC, GA>(args, tq, g, cur, k, slo, shi, wsat, zbuf, bbuf);
        __syncthreads();  // zbuf and bbuf are rewritten by the next tile
    }
    if constexpr (is_quant(PREC)) {
        if ((threadIdx.x & 63) == 0 && wsat) atomicAdd(args.sat, (unsigned long long)wsat);
    }
}

// Tiles [lo, hi) of spectra records dealt out one per ticket by the counter
// *ctr (zero at launch).  Tickets are taken in order, so the tiles in flight
// on an XCD stay neighbours whose partial record lines meet in its L2, and a
// workgroup that runs faster than its neighbours on the CU takes more tiles,
// so all finish together.  Thread 0 takes the ticket of the tile after next
// when a tile starts and publishes it in s_tk before the barrier that ends the
// tile, so the atomic's latency hides behind a tile.
template <int M, int PREC, int GA, bool TRACK = false>
__device__ __forceinline__ void f_tiles_dyn(const FArgs &args, int lo, int hi, unsigned *ctr, int *s_tk,
                                            float2 *zbuf, uint32_t *bbuf) {
    using Sh = FShape<M, PREC, GA, false>;
    constexpr int TS = Sh::TS, NF = Sh::NF, ROUNDS = Sh::ROUNDS, TPT = Sh::TPT;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_tk[0] = (int)atomicAdd(ctr, 1u);
        s_tk[1] = (int)atomicAdd(ctr, 1u);
    }
    __syncthreads();
    int tile = lo + s_tk[0], next = lo + s_tk[1];
    __syncthreads();  // s_tk[0] is rewritten below
    if (tile >= hi) return;
    TileConsts<M, PREC, GA> k;
    k.load(args);
    u32x4 raw[ROUNDS];
    load_tile<M, GA, TS, NF, ROUNDS>(args, tile / args.ngroups, tile % args.ngroups, raw);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // as in f_tiles
    unsigned wsat = 0, tk = 0;  // saturated int8 values of this wave; thread 0's ticket
    for (;;) {
        // an increment (not an add) so the compiler's wave-level atomic
        // rewriting, which reads the result back at once, leaves it alone
        if (tid == 0) tk = atomicInc(ctr, 0xffffffffu);
        const int tq = tile / args.ngroups, g = tile % args.ngroups;
        float slo[TPT], shi[TPT];
        tile_scales<M, PREC, GA>(args, g, slo, shi);
        // the thread's antenna is the same for all its tasks (kThreads is a
        // multiple of GA); loaded, like the scales, before the prefetch, so
        // waiting for it does not wait for the next tile's frames
        double4 trk{0, 0, 0, 0};
        if constexpr (TRACK) trk = args.track[g * GA + tid % GA];
        u32x4 cur[ROUNDS];
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) cur[r] = raw[r];
        // the last tile re-reads its own frames rather than branch around the load
        const int pf = next < hi ? next : tile;
        load_tile<M, GA, TS, NF, ROUNDS>(args, pf / args.ngroups, pf % args.ngroups, raw);
        tile_records<M, PREC, GA, TRACK>(args, tq, g, cur, k, slo, shi, wsat, zbuf, bbuf, trk);
        if (tid == 0) s_tk[0] = (int)tk;
        __syncthreads();  // zbuf and bbuf are rewritten by the next tile; s_tk published
        if (next >= hi) break;
        tile = next;
        next = lo + s_tk[0];
    }
    if constexpr (is_quant(PREC)) {
        if ((threadIdx.x & 63) == 0 && wsat) atomicAdd(args.sat, (unsigned long long)wsat);
    }
}

// Power sums over the calibration window for block blk = group * nblk_t +
// time block: a run of tiles_per_wg consecutive time tiles of one antenna
// group, sums kept in registers (fixed task -> thread mapping, fixed order).
template <int M>
__device__ __forceinline__ void f_power_block(const FArgs &args, int blk, float2 *zbuf, uint32_t *bbuf) {
    constexpr int GA = power_group(M);
    using Sh = FShape<M, kFP32, GA, true>;
    constexpr int TS = Sh::TS, SLOT = Sh::SLOT, NF = Sh::NF, ROUNDS = Sh::ROUNDS;
    constexpr int NTASK = Sh::NTASK, TPT = Sh::TPT;
    const int tid = threadIdx.x;
    const int nblk_t = (args.ntq + args.tiles_per_wg - 1) / args.tiles_per_wg;
    const int pg = blk / nblk_t, pw = blk % nblk_t;
    if (pg >= args.ngroups) return;
    const int tile0 = pw * args.tiles_per_wg;
    const int tile1 = min(tile0 + args.tiles_per_wg, args.ntq);
    FftConsts<M, kFP32> ptw;
    ptw.load(tid % (M / 16), args.tw);
    float2 bw[TPT];
    float plo[TPT], phi[TPT];
#pragma unroll
    for (int it = 0; it < TPT; ++it) {
        const int t = tid + it * kThreads;
        bw[it] = (NTASK % kThreads == 0 || t < NTASK) ? args.tw[M + t / GA] : make_float2(1.0f, 0.0f);
        plo[it] = phi[it] = 0.0f;
    }
    for (int tq = tile0; tq < tile1; ++tq) {
        u32x4 raw[ROUNDS];
        load_tile<M, GA, TS, NF, ROUNDS>(args, tq, pg, raw);
        tile_ffts<M, kFP32, NF, ROUNDS>(raw, zbuf, bbuf, ptw);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < TPT; ++it) {
            const int t = tid + it * kThreads;
            if (NTASK % kThreads != 0 && t >= NTASK) break;
            const int ga = t % GA, q = t / GA;
#pragma unroll
            for (int ts = 0; ts < TS; ++ts) {
                float2 xlo, xhi;
                real_bins<M>(zbuf + (ts * GA + ga) * SLOT, q, bw[it], xlo, xhi);
                plo[it] += fmaf(xlo.x, xlo.x, xlo.y * xlo.y);
                phi[it] += fmaf(xhi.x, xhi.x, xhi.y * xhi.y);
            }
        }
        __syncthreads();  // zbuf is rewritten by the next tile
    }
#pragma unroll
    for (int it = 0; it < TPT; ++it) {
        const int t = tid + it * kThreads;
        if (NTASK % kThreads != 0 && t >= NTASK) break;
        const int ga = t % GA, q = t / GA;
        const int a = pg * GA + ga;
        const int clo = q, chi = q == 0 ? M / 2 : M - q;
        float *pw_row = args.power + ((int64_t)pw * args.a_pad + a) * M;
        pw_row[clo] = plo[it];
        pw_row[chi] = phi[it];
    }
}

// LDS bytes a tile of (M, PREC, GA) needs: transform slots, then (16-byte
// aligned) the byte staging of one round.
template <int M, int PREC, int GA, bool POWER>
constexpr int f_lds_bytes() {
    using Sh = FShape<M, PREC, GA, POWER>;
    return (Sh::NF * Sh::SLOT * 8 + 15) / 16 * 16 + Sh::FPR * (M / 4) * 4;
}

}  // namespace
}  // namespace corr
