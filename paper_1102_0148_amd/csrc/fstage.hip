// Single-job F-stage kernels over the device functions of fstage_dev.h.
#include "fstage_dev.h"

namespace corr {
namespace {

// Persistent workgroups; workgroup b runs on XCD b % 8 (round-robin
// dispatch), and the tiles of XCD x are the range [x t8, (x+1) t8), dealt one
// by one by that XCD's ticket counter: tiles in flight on one XCD are
// neighbours (consecutive antenna groups of nearby time records) whose
// partial lines meet in one L2.
template <int M, int PREC, int GA, bool TRACK>
__device__ __forceinline__ void f_records(const FArgs &args, float2 *zbuf, uint32_t *bbuf) {
    __shared__ int s_tk[2];
    const int t8 = (args.ntiles + 7) / 8;
    const int x = blockIdx.x % 8;
    const int lo = x * t8, hi = min(lo + t8, args.ntiles);
    f_tiles_dyn<M, PREC, GA, TRACK>(args, lo, hi, args.ticket + kTicketStride * x, s_tk, zbuf, bbuf);
}

template <int M, int PREC, int GA, bool POWER>
__global__ __launch_bounds__(kThreads) void fstage_kernel(FArgs kargs) {
    using Sh = FShape<M, PREC, GA, POWER>;
    // a replayed graph passes the input through a device slot that the host
    // rewrites before each replay; a chunk starts s_base spectra into it.
    // The cast through the global address space keeps the input loads
    // global: from a generic pointer they would be flat loads, which also
    // count against lgkmcnt, so every wait for LDS would wait for the next
    // tile's prefetch too.
    typedef const __attribute__((address_space(1))) uint8_t *gptr;
    FArgs args = kargs;
    if (args.in_slot)
        args.in = (const uint8_t *)*reinterpret_cast<const gptr *>(args.in_slot) + (int64_t)args.s_base * args.N * M;
    static_assert(Sh::LDS <= 160 * 1024, "LDS budget");
    __shared__ float2 zbuf[Sh::NF * Sh::SLOT];
    __shared__ __attribute__((aligned(16))) uint32_t bbuf[Sh::FPR * (M / 4)];
    if constexpr (!POWER) {
        f_records<M, PREC, GA, false>(args, zbuf, bbuf);
    } else {
        f_power_block<M>(args, blockIdx.x, zbuf, bbuf);
    }
}

// Records with delay and phase tracking: a kernel of its own, so the kernels
// without tracking are exactly the ones above.
template <int M, int PREC, int GA>
__global__ __launch_bounds__(kThreads) void fstage_track_kernel(FArgs args) {
    using Sh = FShape<M, PREC, GA, false>;
    __shared__ float2 zbuf[Sh::NF * Sh::SLOT];
    __shared__ __attribute__((aligned(16))) uint32_t bbuf[Sh::FPR * (M / 4)];
    f_records<M, PREC, GA, true>(args, zbuf, bbuf);
}

template <int M, int PREC, int GA, bool POWER>
hipError_t launch_one(const FArgs &a, int grid, hipStream_t st) {
    if constexpr (FShape<M, PREC, GA, POWER>::LDS > 160 * 1024) {
        return hipErrorInvalidValue;
    } else {
        const bool track = !POWER && a.track;
        if (!POWER) {
            // as many workgroups (a multiple of 8) as stay resident, at most one
            // per tile
            int per_cu = 0, dev = 0, cus = 0;
            hipError_t e = track ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                       &per_cu, fstage_track_kernel<M, PREC, GA>, kThreads, 0)
                                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                       &per_cu, fstage_kernel<M, PREC, GA, POWER>, kThreads, 0);
            if (e == hipSuccess) e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            const int cap = per_cu * cus / 8 > 0 ? per_cu * cus / 8 : 1;
            const int need = (a.ntiles + 7) / 8;
            grid = 8 * (need < cap ? need : cap);
        }
        if (!POWER) {
            const hipError_t z = launch_fill_zero(a.ticket, kTicketBytes, st);
            if (z != hipSuccess) return z;
        }
        if (track)
            hipLaunchKernelGGL((fstage_track_kernel<M, PREC, GA>), dim3(grid), dim3(kThreads), 0, st, a);
        else
            hipLaunchKernelGGL((fstage_kernel<M, PREC, GA, POWER>), dim3(grid), dim3(kThreads), 0, st, a);
        return hipGetLastError();
    }
}

template <int M, int PREC>
hipError_t launch_mp(int ga, int power, const FArgs &a, int grid, hipStream_t st) {
    if (power) return launch_one<M, kFP32, power_group(M), true>(a, grid, st);
    switch (ga) {
        case 1: return launch_one<M, PREC, 1, false>(a, grid, st);
        case 2: return launch_one<M, PREC, 2, false>(a, grid, st);
        case 4: return launch_one<M, PREC, 4, false>(a, grid, st);
        case 8: return launch_one<M, PREC, 8, false>(a, grid, st);
        case 16: return launch_one<M, PREC, 16, false>(a, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int M>
hipError_t launch_m(int prec, int ga, int power, const FArgs &a, int grid, hipStream_t st) {
    switch (prec) {
        case kFP32: return launch_mp<M, kFP32>(ga, power, a, grid, st);
        case kFP16: return launch_mp<M, kFP16>(ga, power, a, grid, st);
        case kINT8: return launch_mp<M, kINT8>(ga, power, a, grid, st);
        case kINT16: return launch_mp<M, kINT16>(ga, power, a, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int fstage_lds_bytes(int M, int prec, int ga) {
    const int L = M / 16, FPR = kThreads / L, SLOT = M + M / 16 + 1;
    return record_times(prec) * ga * SLOT * 8 + FPR * M;
}

int fstage_default_group(int M, int prec) {
    const int fpr = kThreads / (M / 16);
    const int g = fpr / record_times(prec);
    return g < 1 ? 1 : g;
}

hipError_t launch_fstage(int M, int prec, int ga, int power_mode, const FArgs &a, int grid,
                         hipStream_t st) {
    if (!power_mode && fstage_lds_bytes(M, prec, ga) > 160 * 1024) return hipErrorInvalidValue;
    switch (M) {
        case 128: return launch_m<128>(prec, ga, power_mode, a, grid, st);
        case 256: return launch_m<256>(prec, ga, power_mode, a, grid, st);
        case 512: return launch_m<512>(prec, ga, power_mode, a, grid, st);
        case 1024: return launch_m<1024>(prec, ga, power_mode, a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace corr
