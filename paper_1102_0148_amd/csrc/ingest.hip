// Frame ingest: assembles one integration's packed samples from
// self-contained frames that may arrive lost, repeated or out of order
// (Section 2.2), in two passes over device memory.
#include "corr_internal.h"

#include "../../include/corr.h"

namespace corr {
namespace {

// Pass 1, one thread per frame: check the header and claim the frame's
// spectrum.  The claim is the largest of ~i over the spectrum's accepted
// frames, i.e. the lowest frame index, whatever order the threads run in.
__global__ __launch_bounds__(256) void ingest_claim_kernel(const uint8_t *frames, int64_t n_frames,
                                                           int64_t stride, uint64_t first_seq, int S, int N,
                                                           int K, unsigned *owner, unsigned *counters) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool ok = false;
    if (i < n_frames) {
        const uint4 *h = reinterpret_cast<const uint4 *>(frames + i * stride);
        const uint4 h0 = h[0], h1 = h[1];
        const uint32_t magic = h0.x, version = h0.y & 0xffffu, dtype = h0.y >> 16;
        const uint64_t seq = (uint64_t)h0.z | ((uint64_t)h0.w << 32);
        const uint32_t n_el = h1.x, n_samp = h1.y;
        ok = magic == CORR_FRAME_MAGIC && version == CORR_FRAME_VERSION && dtype == CORR_DTYPE_INT4 &&
             n_el == (uint32_t)N && n_samp == (uint32_t)(2 * K) && seq >= first_seq && seq - first_seq < (uint64_t)S;
        if (ok) atomicMax(&owner[seq - first_seq], 0xffffffffu - (unsigned)i);
    }
    // one atomic per wave for each count
    const uint64_t acc = __ballot(ok), rej = __ballot(i < n_frames && !ok);
    if ((threadIdx.x & 63) == 0) {
        if (acc) atomicAdd(&counters[0], (unsigned)__popcll(acc));
        if (rej) atomicAdd(&counters[1], (unsigned)__popcll(rej));
    }
}

// Pass 2, one workgroup per spectrum: copy the owning frame's payload, or
// zeros when no frame was accepted, and count lost spectra (in the
// calibration window too).
__global__ __launch_bounds__(256) void ingest_copy_kernel(const uint8_t *frames, int64_t stride, int n16, int W,
                                                          const unsigned *owner, unsigned *counters,
                                                          uint4 *out) {
    const int s = blockIdx.x;
    const unsigned o = owner[s];
    uint4 *dst = out + (int64_t)s * n16;
    if (o == 0u) {
        for (int e = threadIdx.x; e < n16; e += 256) dst[e] = make_uint4(0u, 0u, 0u, 0u);
        if (threadIdx.x == 0) atomicAdd(&counters[2], 1u);
    } else {
        const int64_t i = (int64_t)(0xffffffffu - o);
        const uint4 *src = reinterpret_cast<const uint4 *>(frames + i * stride + CORR_FRAME_HEADER_BYTES);
        for (int e = threadIdx.x; e < n16; e += 256) dst[e] = src[e];
        if (threadIdx.x == 0 && s < W) atomicAdd(&counters[3], 1u);
    }
}

}  // namespace

hipError_t launch_ingest(const uint8_t *frames, int64_t n_frames, int64_t stride, uint64_t first_seq, int S,
                         int N, int K, int W, unsigned *owner, unsigned *counters, uint8_t *out, hipStream_t st) {
    // owner holds S entries rounded up to a multiple of 4 (whole 16-byte fills)
    hipError_t e = launch_fill_zero(owner, (size_t)(S + 3) / 4 * 16, st);
    if (e != hipSuccess) return e;
    if ((e = launch_fill_zero(counters, kIngestCounterBytes, st)) != hipSuccess) return e;
    if (n_frames > 0) {
        const int grid = (int)((n_frames + 255) / 256);
        hipLaunchKernelGGL(ingest_claim_kernel, dim3(grid), dim3(256), 0, st, frames, n_frames, stride, first_seq,
                           S, N, K, owner, counters);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ingest_copy_kernel, dim3(S), dim3(256), 0, st, frames, stride, N * K / 16, W, owner,
                       counters, reinterpret_cast<uint4 *>(out));
    return hipGetLastError();
}

}  // namespace corr
