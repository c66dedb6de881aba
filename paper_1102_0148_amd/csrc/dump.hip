// Integration-buffer kernels: the float64 dump of tile partials, the int8
// calibration scales, the read-out transpose and a plain fill.
#include "dump_dev.h"

namespace corr {
namespace {

template <typename P>
__global__ __launch_bounds__(256) void dump_kernel(const P *partial, double2 *acc, int nsplit,
                                                   int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) dump_one<P>(partial, acc, nsplit, n, e);
}

__global__ __launch_bounds__(256) void scales_kernel(const float *power, int nparts, int N, int a_pad,
                                                     int K, int W, const unsigned *w_valid,
                                                     float codes_per_rms, float *scales) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int w = w_valid ? (int)*w_valid : W;
    if (e < N * K) scales[e] = scale_one(power, nparts, a_pad, K, w, e, codes_per_rms);
}

// dst[bl][f] = acc[f][bl]; acc = 0
__global__ __launch_bounds__(256) void finalize_kernel(double2 *acc, double2 *dst, int K, int nb) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)K * nb) return;
    const int f = (int)(e / nb), bl = (int)(e % nb);
    dst[(int64_t)bl * K + f] = acc[e];
    acc[e] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint4 *p, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

hipError_t launch_dump(int prec, const void *partial, double2 *acc, int nsplit, int K, int nb,
                       hipStream_t st) {
    const int64_t n = (int64_t)K * nb;
    const int grid = (int)((n + 255) / 256);
    if (prec == kINT8)
        hipLaunchKernelGGL(dump_kernel<int2>, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<const int2 *>(partial), acc, nsplit, n);
    else if (prec == kINT16)
        hipLaunchKernelGGL(dump_kernel<double2>, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<const double2 *>(partial), acc, nsplit, n);
    else
        hipLaunchKernelGGL(dump_kernel<float2>, dim3(grid), dim3(256), 0, st,
                           reinterpret_cast<const float2 *>(partial), acc, nsplit, n);
    return hipGetLastError();
}

hipError_t launch_scales(const float *power, int nparts, int N, int a_pad, int K, int W,
                         const unsigned *w_valid, float codes_per_rms, float *scales, hipStream_t st) {
    const int grid = (N * K + 255) / 256;
    hipLaunchKernelGGL(scales_kernel, dim3(grid), dim3(256), 0, st, power, nparts, N, a_pad, K, W, w_valid,
                       codes_per_rms, scales);
    return hipGetLastError();
}

hipError_t launch_finalize(double2 *acc, double2 *dst, int K, int nb, hipStream_t st) {
    const int64_t n = (int64_t)K * nb;
    const int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(256), 0, st, acc, dst, K, nb);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    int64_t grid = (n16 + 255) / 256;
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((int)grid), dim3(256), 0, st, reinterpret_cast<uint4 *>(p), n16);
    return hipGetLastError();
}

}  // namespace corr
