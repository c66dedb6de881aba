// Float64 dump of tile partials and int8 scales, as device functions shared
// by the single-job kernels and the batch kernel.
#pragma once
#include "corr_internal.h"

namespace corr {
namespace {

// acc[e] += partial[0][e] + partial[1][e] + ... in this order, in float64
// (Section 1: the cross power spectra are accumulated to the cadence).
// Runs of 16 partials are loaded before any is added, so their loads are in
// flight together (as one loop each load waited for the previous add).
template <typename P>
__device__ __forceinline__ void dump_one(const P *partial, double2 *acc, int nsplit, int64_t n, int64_t e) {
    double2 v = acc[e];
    int s = 0;
    for (; s + 16 <= nsplit; s += 16) {
        P p[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) p[j] = partial[(int64_t)(s + j) * n + e];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            v.x += (double)p[j].x;
            v.y += (double)p[j].y;
        }
    }
    for (; s < nsplit; ++s) {
        const P p = partial[(int64_t)s * n + e];
        v.x += (double)p.x;
        v.y += (double)p.y;
    }
    acc[e] = v;
}

// Scale of (antenna, channel) e = ant * K + c: the power over the window is
// summed over its nparts partials in order; rms is that of one non-zero
// component, sqrt(P / W) in channel 0 (a real-input transform's DC has no
// imaginary part) and sqrt(P / (2W)) elsewhere; scale = codes_per_rms / rms,
// the form's largest code over the rms multiple it stands for (int8: 127 at
// 4 rms; int16: 32512 at 8 rms); a channel with no power keeps 1.
__device__ __forceinline__ float scale_one(const float *power, int nparts, int a_pad, int K, int W, int e,
                                           float codes_per_rms) {
    const int ant = e / K, c = e % K;
    const float *src = power + (int64_t)ant * K + c;
    const int64_t stride = (int64_t)a_pad * K;
    float p = 0.0f;
    // The adds stay in order.  Runs of 32 partials are loaded into registers
    // of their own before any is added, so their loads are in flight
    // together: written as one loop, the compiler gave every load the same
    // register and each load waited for the previous add (128 round trips
    // for a 1024-spectrum window, 35 us).
    int i = 0;
    for (; i + 32 <= nparts; i += 32) {
        float v[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) v[j] = src[(int64_t)(i + j) * stride];
#pragma unroll
        for (int j = 0; j < 32; ++j) p += v[j];
    }
    for (; i < nparts; ++i) p += src[(int64_t)i * stride];
    float sc = 1.0f;
    if (p > 0.0f && W > 0) {
        const float rms = sqrtf(p / ((c == 0 ? 1.0f : 2.0f) * (float)W));
        sc = codes_per_rms / rms;
    }
    return sc;
}

}  // namespace
}  // namespace corr
