/*
 * CPU oracle for the FX spectral correlator (Prasad & Subrahmanya,
 * "Software Spectral Correlator for the 44-Element Ooty Radio Telescope").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * correlator library never links, calls or falls back to it.  It shares no
 * code, header, table or constant with the HIP path.
 *
 * Everything is the plain definition of what the correlator computes
 * (Section 1: split each stream into channels with an FFT, cross-multiply the
 * spectra of every antenna pair per channel, accumulate), written out in
 * double precision and in exact 64-bit integers:
 *
 *   unpack    x[n]     = signed 4-bit sample n of a block (two per byte)
 *   spectra   X[s,a,k] = sum_n x[n] exp(-2 pi i k n / 2K), k = 0..K-1
 *                        (forward, unnormalised transform -- Section 4)
 *   cmac      V[a,b,k] = sum_s X[s,a,k] conj(X[s,b,k]),  0 <= a <= b < N
 *   int8 form scales from the calibration window, q = clamp(rint(x*sc)),
 *             then the same cmac in int64 (exact)
 *   track     X[s,a,k] *= exp(2 pi i rho(s,a,k)), the per-antenna delay and
 *             phase model applied before accumulation (Section 2.1)
 *   int16     the same requantisation to codes within +-32512 (Section 4's
 *             16-bit short complex type), and the cmac on them in int64
 *   ingest    frames (header + block) put into their blocks in index order,
 *             lost blocks zero, and the scales over the received blocks
 *             (Section 2.2)
 *
 * Readings of points the paper leaves open (each one a stated choice):
 *   - samples are two's-complement nibbles, -8..7; the low nibble of a byte
 *     is the earlier (even) sample;
 *   - a frame is [spectrum][antenna][2K samples] (Section 2.2: one packet of
 *     contiguous samples from all elements is one FFT block); no window, no
 *     overlap;
 *   - bins 0..K-1 are kept (DC kept, Nyquist bin K dropped);
 *   - baselines include autos, upper triangle, row-major:
 *     bl(a,b) = a*N - a*(a-1)/2 + (b-a);
 *   - int8: rms over the first W spectra of the integration, per non-zero
 *     component of the channel: a real-input transform's channel 0 (DC) has
 *     no imaginary part, so rms = sqrt(sum(re^2) / W) there and
 *     rms = sqrt(sum(re^2+im^2) / (2W)) in every other channel;
 *     sc = 127 / (4 rms) in float; a channel with zero power gets sc = 1;
 *     q = clamp(rint(float(x) * sc), -127, 127) with float arithmetic and
 *     ties to even;
 *   - int16: the same with the largest code 32512 standing for 8 rms (its
 *     steps are 128 times finer than int8's and a Gaussian component clips
 *     with probability about 1e-15), q clamped to +-32512.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (brute-force DFT, numpy's FFT, Parseval, Hermitian symmetry, exact integer
 * bins, tone bin, expected correlation coefficient, delay phase slope,
 * identical-input baselines, int64 == float64 on integer input; tracking:
 * the DFT shift theorem, quarter and half turns, common-phase invariance and
 * the removal of a delayed source's phase slope; int16: ties and clamp,
 * int64 sums against numpy, scales 128 times the int8 rule's; ingest:
 * hand-built order,
 * loss, repeats and every header fault, and the scales over received blocks
 * against the plain rule on the window without the lost blocks).  The int8
 * calibration rule itself is a reading, not something the paper fixes, so
 * its constants are "parity unpinned" against the paper; the tests pin that
 * the code implements the rule as stated.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static const double ORC_PI = 3.14159265358979323846264338327950288;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* Baseline index of antenna pair (a, b), a <= b, upper triangle row-major
 * with autos.  */
int64_t orc_baseline_index(int N, int a, int b)
{
    return (int64_t)a * N - (int64_t)a * (a - 1) / 2 + (b - a);
}

/* Unpack n_samples signed 4-bit samples, two per byte, low nibble first. */
int orc_unpack(const uint8_t *packed, int64_t n_samples, int8_t *out)
{
    if (!packed || !out || n_samples < 0 || (n_samples & 1)) return ORC_EINVAL;
    for (int64_t n = 0; n < n_samples; ++n) {
        int byte = packed[n / 2];
        int nib = (n % 2 == 0) ? (byte & 0xF) : (byte >> 4);
        out[n] = (int8_t)(nib >= 8 ? nib - 16 : nib);
    }
    return ORC_OK;
}

/* In-place forward, unnormalised complex FFT of length n (power of two):
 * textbook iterative radix-2 decimation in time with a bit-reversal
 * permutation.  Y[k] = sum_j y[j] exp(-2 pi i j k / n).  */
int orc_fft(int n, double *re, double *im)
{
    if (!re || !im || !is_pow2(n)) return ORC_EINVAL;
    /* bit reversal */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2;
        for (int start = 0; start < n; start += len) {
            for (int j = 0; j < half; ++j) {
                double ang = -2.0 * ORC_PI * (double)j / (double)len;
                double wr = cos(ang), wi = sin(ang);
                int p = start + j, q = start + j + half;
                double tr = re[q] * wr - im[q] * wi;
                double ti = re[q] * wi + im[q] * wr;
                re[q] = re[p] - tr; im[q] = im[p] - ti;
                re[p] += tr;        im[p] += ti;
            }
        }
    }
    return ORC_OK;
}

/* Full 2K-point DFT of one block of real samples: out is [2K][2]
 * (re, im) for every bin 0..2K-1.  */
int orc_fft_real(const double *x, int two_k, double *out)
{
    if (!x || !out || !is_pow2(two_k)) return ORC_EINVAL;
    double *re = (double *)malloc(sizeof(double) * two_k);
    double *im = (double *)malloc(sizeof(double) * two_k);
    if (!re || !im) { free(re); free(im); return ORC_ENOMEM; }
    for (int n = 0; n < two_k; ++n) { re[n] = x[n]; im[n] = 0.0; }
    orc_fft(two_k, re, im);
    for (int k = 0; k < two_k; ++k) { out[2 * k] = re[k]; out[2 * k + 1] = im[k]; }
    free(re); free(im);
    return ORC_OK;
}

/* F-stage: spectra of every (spectrum, antenna) block.
 * packed: [S][N][K] bytes (2K samples per block); out: [S][N][K][2] doubles
 * holding bins 0..K-1.  */
int orc_spectra(const uint8_t *packed, int S, int N, int K, double *out)
{
    if (!packed || !out || S < 0 || N < 1 || !is_pow2(K)) return ORC_EINVAL;
    const int two_k = 2 * K;
    int err = ORC_OK;
#pragma omp parallel
    {
        double *re = (double *)malloc(sizeof(double) * two_k);
        double *im = (double *)malloc(sizeof(double) * two_k);
        int8_t *x = (int8_t *)malloc(two_k);
        if (!re || !im || !x) {
#pragma omp atomic write
            err = ORC_ENOMEM;
        } else {
#pragma omp for schedule(static)
            for (int64_t blk = 0; blk < (int64_t)S * N; ++blk) {
                orc_unpack(packed + blk * K, two_k, x);
                for (int n = 0; n < two_k; ++n) { re[n] = x[n]; im[n] = 0.0; }
                orc_fft(two_k, re, im);
                double *o = out + blk * (int64_t)K * 2;
                for (int k = 0; k < K; ++k) { o[2 * k] = re[k]; o[2 * k + 1] = im[k]; }
            }
        }
        free(re); free(im); free(x);
    }
    return err;
}

/* Delay and phase tracking (Section 2.1: where the signal path disperses, a
 * phase is applied to each subband before accumulation in time).  In place on
 * spec [S][N][K][2], spectrum s being spectrum s0 + s of the integration:
 *   X[s,a,k] *= exp(2 pi i rho),
 *   rho = k (delay[a] + delay_rate[a] t) / 2K + phase[a] + phase_rate[a] t,
 *   t = s0 + s,
 * with delays in samples and phases in turns.  Each array holds N values, or
 * is NULL for zeros.  The whole turns of rho are dropped before the cosine
 * and sine (which changes nothing but the rounding of large arguments).  */
int orc_track(double *spec, int S, int N, int K, int s0, const double *delay, const double *delay_rate,
              const double *phase, const double *phase_rate)
{
    if (!spec || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    for (int64_t s = 0; s < S; ++s) {
        const double t = (double)(s0 + s);
        for (int a = 0; a < N; ++a) {
            const double d = (delay ? delay[a] : 0.0) + (delay_rate ? delay_rate[a] : 0.0) * t;
            const double p = (phase ? phase[a] : 0.0) + (phase_rate ? phase_rate[a] : 0.0) * t;
            for (int k = 0; k < K; ++k) {
                double rho = (double)k * d / (2.0 * K) + p;
                rho -= floor(rho);
                const double c = cos(2.0 * ORC_PI * rho), sn = sin(2.0 * ORC_PI * rho);
                double *x = spec + ((s * N + a) * (int64_t)K + k) * 2;
                const double re = x[0], im = x[1];
                x[0] = re * c - im * sn;
                x[1] = re * sn + im * c;
            }
        }
    }
    return ORC_OK;
}

/* Frame ingest (Section 2.2: packets are self-contained FFT blocks of every
 * element whose headers give sample timing, datatype and element count, and
 * they may be lost, repeated or reordered in transit).  A frame is a 32-byte
 * little-endian header -- magic 0x4D52464F, version (16 bits) 1, datatype
 * (16 bits) 1 = 4-bit, block number (64 bits), elements (32 bits), samples
 * per element (32 bits), 8 reserved bytes -- then N*K payload bytes.  Frames
 * are taken in index order; a frame is used when its header is valid for
 * this (N, 2K), its block lies in [first_seq, first_seq + S), and no earlier
 * frame filled that block.  Blocks no frame fills are zero.  stats: accepted,
 * rejected, duplicate frames, lost blocks; window_valid: blocks received
 * among the first W.  */
static uint64_t le_get(const uint8_t *p, int nbytes)
{
    uint64_t v = 0;
    for (int i = nbytes - 1; i >= 0; --i) v = (v << 8) | p[i];
    return v;
}

int orc_ingest(const uint8_t *frames, int64_t n_frames, int64_t stride, uint64_t first_seq, int S, int N, int K,
               int W, uint8_t *out, int64_t *stats, int64_t *window_valid)
{
    if ((!frames && n_frames > 0) || !out || !stats || !window_valid || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    const int64_t payload = (int64_t)N * K;
    if (stride < 32 + payload) return ORC_EINVAL;
    uint8_t *filled = (uint8_t *)calloc(S > 0 ? S : 1, 1);
    if (!filled) return ORC_ENOMEM;
    memset(out, 0, (size_t)S * payload);
    stats[0] = stats[1] = stats[2] = stats[3] = 0;
    for (int64_t i = 0; i < n_frames; ++i) {
        const uint8_t *f = frames + i * stride;
        const uint64_t seq = le_get(f + 8, 8);
        const int ok = le_get(f, 4) == 0x4D52464Fu && le_get(f + 4, 2) == 1 && le_get(f + 6, 2) == 1 &&
                       le_get(f + 16, 4) == (uint64_t)N && le_get(f + 20, 4) == (uint64_t)(2 * K) &&
                       seq >= first_seq && seq - first_seq < (uint64_t)S;
        if (!ok) { stats[1]++; continue; }
        stats[0]++;
        const int64_t slot = (int64_t)(seq - first_seq);
        if (filled[slot]) { stats[2]++; continue; }
        filled[slot] = 1;
        memcpy(out + slot * payload, f + 32, (size_t)payload);
    }
    *window_valid = 0;
    for (int s = 0; s < S; ++s) {
        if (!filled[s]) stats[3]++;
        else if (s < W) (*window_valid)++;
    }
    free(filled);
    return ORC_OK;
}

/* Components of channel k that can be non-zero: the DC channel of a
 * real-input transform is real, every other kept channel complex.  */
static double components(int k) { return k == 0 ? 1.0 : 2.0; }

/* Scales for a form whose largest code qmax stands for `clip` times the rms
 * of one component (int8: 127 at 4 rms; int16: 32512 at 8 rms), the mean
 * power dividing by n_div spectra (the ones received in the window; W when
 * none is lost); lost spectra are zero and add no power.  */
int orc_scales_n(const double *spec, int S, int N, int K, int W, int n_div, double qmax, double clip,
                 float *scales)
{
    if (!spec || !scales || N < 1 || K < 1 || W < 1 || W > S || n_div < 0 || !(qmax > 0) || !(clip > 0))
        return ORC_EINVAL;
    for (int a = 0; a < N; ++a) {
        for (int k = 0; k < K; ++k) {
            double p = 0.0;
            for (int s = 0; s < W; ++s) {
                const double *x = spec + (((int64_t)s * N + a) * K + k) * 2;
                p += x[0] * x[0] + x[1] * x[1];
            }
            double sc = 1.0;
            if (p > 0.0 && n_div > 0) sc = qmax / (clip * sqrt(p / (components(k) * n_div)));
            scales[(int64_t)a * K + k] = (float)sc;
        }
    }
    return ORC_OK;
}

/* X-stage in float64: V[a,b,k] = sum_s X[s,a,k] * conj(X[s,b,k]).
 * spec: [S][N][K][2].  full == 0: vis is [nb][K][2] over a <= b (baseline
 * order above); full != 0: vis is [N][N][K][2] over every ordered pair.
 * Each output sums s in increasing order.  */
int orc_cmac_f64(const double *spec, int S, int N, int K, int full, double *vis)
{
    if (!spec || !vis || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    const int64_t nout = full ? (int64_t)N * N : nb;
    memset(vis, 0, sizeof(double) * nout * K * 2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < N; ++a) {
        for (int s = 0; s < S; ++s) {
            const double *xa = spec + ((int64_t)s * N + a) * K * 2;
            for (int b = full ? 0 : a; b < N; ++b) {
                const double *xb = spec + ((int64_t)s * N + b) * K * 2;
                int64_t row = full ? (int64_t)a * N + b : orc_baseline_index(N, a, b);
                double *v = vis + row * K * 2;
                for (int k = 0; k < K; ++k) {
                    double ar = xa[2 * k], ai = xa[2 * k + 1];
                    double br = xb[2 * k], bi = xb[2 * k + 1];
                    /* (ar + i ai)(br - i bi) */
                    v[2 * k] += ar * br + ai * bi;
                    v[2 * k + 1] += ai * br - ar * bi;
                }
            }
        }
    }
    return ORC_OK;
}

/* int8 calibration: per-(antenna, channel) scale from the first W spectra,
 * full scale 127 at 4 times the rms of one non-zero component.
 * spec: [S][N][K][2] doubles; scales: [N][K] floats.  */
int orc_scales(const double *spec, int S, int N, int K, int W, float *scales)
{
    if (!spec || !scales || N < 1 || K < 1 || W < 1 || W > S) return ORC_EINVAL;
    for (int a = 0; a < N; ++a) {
        for (int k = 0; k < K; ++k) {
            double p = 0.0;
            for (int s = 0; s < W; ++s) {
                const double *x = spec + (((int64_t)s * N + a) * K + k) * 2;
                p += x[0] * x[0] + x[1] * x[1];
            }
            double sc = 1.0;
            if (p > 0.0) {
                double rms = sqrt(p / (components(k) * W));
                sc = 127.0 / (4.0 * rms);
            }
            scales[(int64_t)a * K + k] = (float)sc;
        }
    }
    return ORC_OK;
}

/* One component quantised to int8: the decision is taken in float with the
 * float value of the spectrum, rounding half to even, symmetric clamp.  */
static int8_t quantise_one(double x, float sc)
{
    float v = (float)x * sc;
    float r = rintf(v);
    if (r > 127.0f) r = 127.0f;
    if (r < -127.0f) r = -127.0f;
    return (int8_t)r;
}

/* spec: [S][N][K][2] doubles; scales: [N][K]; q: [S][N][K][2] int8.  */
int orc_quantise(const double *spec, int S, int N, int K, const float *scales, int8_t *q)
{
    if (!spec || !scales || !q || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    for (int64_t s = 0; s < S; ++s)
        for (int a = 0; a < N; ++a)
            for (int k = 0; k < K; ++k) {
                int64_t i = ((s * N + a) * K + k) * 2;
                float sc = scales[(int64_t)a * K + k];
                q[i] = quantise_one(spec[i], sc);
                q[i + 1] = quantise_one(spec[i + 1], sc);
            }
    return ORC_OK;
}

/* The 16-bit form (Section 4: the conversion of the float spectra to a short
 * complex integer type with prescaling): q = clamp(rint(float(x) * sc),
 * -32512, 32512), decided in float as for int8.  q: [S][N][K][2] int16.  */
int orc_quantise16(const double *spec, int S, int N, int K, const float *scales, int16_t *q)
{
    if (!spec || !scales || !q || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    for (int64_t s = 0; s < S; ++s)
        for (int a = 0; a < N; ++a)
            for (int k = 0; k < K; ++k) {
                const int64_t i = ((s * N + a) * K + k) * 2;
                const float sc = scales[(int64_t)a * K + k];
                for (int c = 0; c < 2; ++c) {
                    float r = rintf((float)spec[i + c] * sc);
                    if (r > 32512.0f) r = 32512.0f;
                    if (r < -32512.0f) r = -32512.0f;
                    q[i + c] = (int16_t)r;
                }
            }
    return ORC_OK;
}

/* Exact integer X-stage on 16-bit spectra, as orc_cmac_i64.  */
int orc_cmac_i64_16(const int16_t *q, int S, int N, int K, int full, int64_t *vis)
{
    if (!q || !vis || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    const int64_t nout = full ? (int64_t)N * N : nb;
    memset(vis, 0, sizeof(int64_t) * nout * K * 2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < N; ++a) {
        for (int s = 0; s < S; ++s) {
            const int16_t *xa = q + ((int64_t)s * N + a) * K * 2;
            for (int b = full ? 0 : a; b < N; ++b) {
                const int16_t *xb = q + ((int64_t)s * N + b) * K * 2;
                int64_t row = full ? (int64_t)a * N + b : orc_baseline_index(N, a, b);
                int64_t *v = vis + row * K * 2;
                for (int k = 0; k < K; ++k) {
                    int64_t ar = xa[2 * k], ai = xa[2 * k + 1];
                    int64_t br = xb[2 * k], bi = xb[2 * k + 1];
                    v[2 * k] += ar * br + ai * bi;
                    v[2 * k + 1] += ai * br - ar * bi;
                }
            }
        }
    }
    return ORC_OK;
}

/* Exact integer X-stage on quantised spectra: q [S][N][K][2] int8,
 * vis [nb][K][2] int64 (full == 0) or [N][N][K][2] (full != 0).  */
int orc_cmac_i64(const int8_t *q, int S, int N, int K, int full, int64_t *vis)
{
    if (!q || !vis || S < 0 || N < 1 || K < 1) return ORC_EINVAL;
    const int64_t nb = (int64_t)N * (N + 1) / 2;
    const int64_t nout = full ? (int64_t)N * N : nb;
    memset(vis, 0, sizeof(int64_t) * nout * K * 2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < N; ++a) {
        for (int s = 0; s < S; ++s) {
            const int8_t *xa = q + ((int64_t)s * N + a) * K * 2;
            for (int b = full ? 0 : a; b < N; ++b) {
                const int8_t *xb = q + ((int64_t)s * N + b) * K * 2;
                int64_t row = full ? (int64_t)a * N + b : orc_baseline_index(N, a, b);
                int64_t *v = vis + row * K * 2;
                for (int k = 0; k < K; ++k) {
                    int64_t ar = xa[2 * k], ai = xa[2 * k + 1];
                    int64_t br = xb[2 * k], bi = xb[2 * k + 1];
                    v[2 * k] += ar * br + ai * bi;
                    v[2 * k + 1] += ai * br - ar * bi;
                }
            }
        }
    }
    return ORC_OK;
}

/* One visibility computed on its own, straight from the packed samples:
 * each X[s,a,k] is the single-bin DFT sum_n x[n] exp(-2 pi i k n / 2K)
 * (no FFT), then V = sum_s X[s,a,k] conj(X[s,b,k]).  Used to check sampled
 * outputs of integrations too long for the full oracle.  out: [2].  */
int orc_vis_single(const uint8_t *packed, int S, int N, int K, int a, int b, int k, double *out)
{
    if (!packed || !out || S < 0 || N < 1 || K < 1 || a < 0 || b < 0 || a >= N ||
        b >= N || k < 0 || k >= K)
        return ORC_EINVAL;
    const int two_k = 2 * K;
    double *wr = (double *)malloc(sizeof(double) * two_k);
    double *wi = (double *)malloc(sizeof(double) * two_k);
    if (!wr || !wi) { free(wr); free(wi); return ORC_ENOMEM; }
    for (int n = 0; n < two_k; ++n) {
        /* exponent reduced mod 2K so the angle is exact before cos/sin */
        int64_t e = ((int64_t)k * n) % two_k;
        double ang = -2.0 * ORC_PI * (double)e / (double)two_k;
        wr[n] = cos(ang);
        wi[n] = sin(ang);
    }
    double vr = 0.0, vi = 0.0;
#pragma omp parallel for reduction(+ : vr, vi) schedule(static)
    for (int s = 0; s < S; ++s) {
        double xr[2] = {0.0, 0.0}, xi[2] = {0.0, 0.0};
        int ant[2] = {a, b};
        for (int t = 0; t < 2; ++t) {
            const uint8_t *blk = packed + ((int64_t)s * N + ant[t]) * K;
            for (int n = 0; n < two_k; ++n) {
                int byte = blk[n / 2];
                int nib = (n % 2 == 0) ? (byte & 0xF) : (byte >> 4);
                double x = (double)(nib >= 8 ? nib - 16 : nib);
                xr[t] += x * wr[n];
                xi[t] += x * wi[n];
            }
        }
        vr += xr[0] * xr[1] + xi[0] * xi[1];
        vi += xi[0] * xr[1] - xr[0] * xi[1];
    }
    out[0] = vr;
    out[1] = vi;
    free(wr); free(wi);
    return ORC_OK;
}

/* Threads the OpenMP loops above use (a timing control).  Every parallel
 * loop but one writes disjoint outputs in a fixed order of summation, so its
 * result does not depend on the count; orc_vis_single's reduction over
 * spectra regroups its float64 sum by thread, which moves it by rounding
 * only.  */
int orc_set_threads(int n)
{
    if (n < 1) return ORC_EINVAL;
    omp_set_num_threads(n);
    return ORC_OK;
}

int orc_get_threads(void)
{
    return omp_get_max_threads();
}
