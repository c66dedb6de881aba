// Single-job X-stage kernels over the device function of xstage_dev.h.
#include "xstage_dev.h"

namespace corr {
namespace {

// Region kinds of a launch: off-diagonal, diagonal, or both (regions
// [0, n_diag) diagonal, the rest off-diagonal), which lets every region of a
// channel read its records through one L2 in one launch.
constexpr int kOffDiag = 0, kDiag = 1, kBoth = 2;

// Two workgroups per CU (two waves per SIMD) keep the accumulators in
// ordinary VGPRs (without the bound the compiler splits them across VGPRs and
// AGPRs, and the larger regions fall to one wave per SIMD); the fp32
// off-diagonal 4 x 4-block region and the fp32 6-block diagonal region need
// more than 256 registers and keep the default.
template <int PREC, int RB, int KIND>
constexpr int x_min_blocks() {
    return (PREC == kFP32 && ((RB >= 4 && KIND != kDiag) || RB >= 6)) ? 1 : 2;
}

template <int PREC, int RB, int KIND>
__global__ __launch_bounds__(256, (x_min_blocks<PREC, RB, KIND>())) void xstage_kernel(XArgs a) {
    __shared__ float tbuf[4][16 * 17];
    // wave-uniform values live in scalar registers, so the loops have scalar
    // control flow
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // workgroup b runs on XCD b % 8 (round-robin dispatch); it takes logical
    // workgroup (b % 8) * (grid / 8) + b / 8, so consecutive logical
    // workgroups, the regions of one channel and split that read the same
    // records, share an XCD and its L2
    const int lb = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    const int wave = lb * 4 + w;
    if constexpr (KIND == kBoth) {
        if (wave % a.nregions < a.n_diag)
            x_wave<PREC, RB, true>(a, wave, tbuf[w]);
        else
            x_wave<PREC, RB, false>(a, wave, tbuf[w]);
    } else {
        x_wave<PREC, RB, KIND == kDiag>(a, wave, tbuf[w]);
    }
}

template <int PREC, int RB, int KIND>
hipError_t launch_one(const XArgs &a, hipStream_t st) {
    const int64_t waves = (int64_t)a.nregions * a.K * a.nsplit;
    const int grid = (int)(8 * ((waves + 31) / 32));  // a multiple of 8; waves past the end exit
    hipLaunchKernelGGL((xstage_kernel<PREC, RB, KIND>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_p(int rb, int kind, const XArgs &a, hipStream_t st) {
    if (kind == kDiag) {
        switch (rb) {
            case 1: return launch_one<PREC, 1, kDiag>(a, st);
            case 2: return launch_one<PREC, 2, kDiag>(a, st);
            case 3: return launch_one<PREC, 3, kDiag>(a, st);
            case 4: return launch_one<PREC, 4, kDiag>(a, st);
            case 5: return launch_one<PREC, 5, kDiag>(a, st);
            case 6: return launch_one<PREC, 6, kDiag>(a, st);
        }
    } else if (kind == kOffDiag) {
        switch (rb) {
            case 2: return launch_one<PREC, 2, kOffDiag>(a, st);
            case 3: return launch_one<PREC, 3, kOffDiag>(a, st);
            case 4: return launch_one<PREC, 4, kOffDiag>(a, st);
        }
    } else if (kind == kBoth) {
        switch (rb) {
            case 2: return launch_one<PREC, 2, kBoth>(a, st);
            case 3: return launch_one<PREC, 3, kBoth>(a, st);
            case 4: return launch_one<PREC, 4, kBoth>(a, st);
        }
    }
    return hipErrorInvalidValue;
}

// Region groups through a 3-stage LDS ring (3 x 16 KB); two workgroups per
// CU keep the 4 x 4-block accumulators in VGPRs.  The three stages are
// separate arrays so the compiler can tell a stage being read from the stage
// that a direct load is filling, and adds no wait between them.
template <int PREC>
__global__ __launch_bounds__(256, 2) void xgroup_kernel(XArgs a) {
    // one array per stage: the compiler then tells the stages apart and waits
    // for a stage's own loads only, not for every load to LDS in flight
    __shared__ __attribute__((aligned(16))) uint4 st0[kXStage];
    __shared__ __attribute__((aligned(16))) uint4 st1[kXStage];
    __shared__ __attribute__((aligned(16))) uint4 st2[kXStage];
#if X_RING >= 4
    __shared__ __attribute__((aligned(16))) uint4 st3[kXStage];
#endif
#if X_RING >= 5
    __shared__ __attribute__((aligned(16))) uint4 st4[kXStage];
#endif
    uint4 *const st[kXRing] = {st0, st1, st2
#if X_RING >= 4
                               , st3
#endif
#if X_RING >= 5
                               , st4
#endif
    };
    // logical workgroup as in xstage_kernel: a channel's groups share an XCD
    const int lb = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    x_group<PREC>(a, lb, st);
}

template <int PREC>
hipError_t launch_group(const XArgs &a, hipStream_t st) {
    const int64_t units = (int64_t)a.ngroups * a.K * a.nsplit;
    const int grid = (int)(8 * ((units + 7) / 8));  // a multiple of 8; units past the end exit
    hipLaunchKernelGGL((xgroup_kernel<PREC>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Whole-channel groups (16 antenna blocks; fp32, fp16 and int8): eight waves
// per workgroup, one workgroup per (channel, split), the 16 blocks of a
// k-block staged once, in a ring of kXChanRing stages (one workgroup per CU
// would leave LDS for up to eight; depths 3, 4, 6 and 8 measured the same at
// N = 256).
#ifndef X_CHAN_RING
#define X_CHAN_RING 3
#endif
constexpr int kXChanRing = X_CHAN_RING;

template <int PREC>
__global__ __launch_bounds__(kXChanWaves * 64, 1) void xchan_kernel(XArgs a) {
    // one array per stage, as in xgroup_kernel
    __shared__ __attribute__((aligned(16))) uint4 st0[kXStage];
    __shared__ __attribute__((aligned(16))) uint4 st1[kXStage];
    __shared__ __attribute__((aligned(16))) uint4 st2[kXStage];
#if X_CHAN_RING >= 4
    __shared__ __attribute__((aligned(16))) uint4 st3[kXStage];
#endif
#if X_CHAN_RING >= 5
    __shared__ __attribute__((aligned(16))) uint4 st4[kXStage];
#endif
#if X_CHAN_RING >= 6
    __shared__ __attribute__((aligned(16))) uint4 st5[kXStage];
#endif
#if X_CHAN_RING >= 7
    __shared__ __attribute__((aligned(16))) uint4 st6[kXStage];
#endif
#if X_CHAN_RING >= 8
    __shared__ __attribute__((aligned(16))) uint4 st7[kXStage];
#endif
    uint4 *const st[kXChanRing] = {st0, st1, st2
#if X_CHAN_RING >= 4
                                   , st3
#endif
#if X_CHAN_RING >= 5
                                   , st4
#endif
#if X_CHAN_RING >= 6
                                   , st5
#endif
#if X_CHAN_RING >= 7
                                   , st6
#endif
#if X_CHAN_RING >= 8
                                   , st7
#endif
    };
    // logical workgroup as in xstage_kernel: neighbouring channels share an XCD
    const int lb = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if constexpr (PREC == kFP32) {
        __shared__ float tb[kXChanWaves * 16 * 17];
        x_chan_f32<kXChanRing>(a, lb, st, tb);
    } else {
        x_chan<PREC, kXChanRing>(a, lb, st);
    }
}

template <int PREC>
hipError_t launch_chan(const XArgs &a, hipStream_t st) {
    const int64_t units = (int64_t)a.K * a.nsplit;
    const int grid = (int)(8 * ((units + 7) / 8));  // a multiple of 8; units past the end exit
    hipLaunchKernelGGL((xchan_kernel<PREC>), dim3(grid), dim3(kXChanWaves * 64), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_xchan(int prec, const XArgs &a, hipStream_t st) {
    switch (prec) {
        case kFP32: return launch_chan<kFP32>(a, st);
        case kFP16: return launch_chan<kFP16>(a, st);
        case kINT8: return launch_chan<kINT8>(a, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_xgroups(int prec, const XArgs &a, hipStream_t st) {
    switch (prec) {
        case kFP16: return launch_group<kFP16>(a, st);
        case kINT8: return launch_group<kINT8>(a, st);
    }
    return hipErrorInvalidValue;
}

namespace {

// int16: regions of at most 3 blocks on the diagonal and 2 off it (six
// accumulators per block pair).
template <int RB, int KIND>
__global__ __launch_bounds__(256, 2) void xstage16_kernel(XArgs a) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lb = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    x_wave16<RB, KIND == kDiag>(a, lb * 4 + w);
}

template <int RB, int KIND>
hipError_t launch16(const XArgs &a, hipStream_t st) {
    const int64_t waves = (int64_t)a.nregions * a.K * a.nsplit;
    const int grid = (int)(8 * ((waves + 31) / 32));
    hipLaunchKernelGGL((xstage16_kernel<RB, KIND>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_xstage16(int rb, int kind, const XArgs &a, hipStream_t st) {
    if (kind == kDiag) {
        switch (rb) {
            case 1: return launch16<1, kDiag>(a, st);
            case 2: return launch16<2, kDiag>(a, st);
            case 3: return launch16<3, kDiag>(a, st);
        }
    } else if (kind == kOffDiag) {
        switch (rb) {
            case 1: return launch16<1, kOffDiag>(a, st);
            case 2: return launch16<2, kOffDiag>(a, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_xstage(int prec, int rb, int kind, const XArgs &a, hipStream_t st) {
    if (prec == kINT16) return launch_xstage16(rb, kind, a, st);
    switch (prec) {
        case kFP32: return launch_p<kFP32>(rb, kind, a, st);
        case kFP16: return launch_p<kFP16>(rb, kind, a, st);
        case kINT8: return launch_p<kINT8>(rb, kind, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace corr
