// Single-job X-stage kernels over the device function of xstage_dev.h.
#include "xstage_dev.h"

namespace corr {
namespace {

// Two workgroups per CU (two waves per SIMD) keep the accumulators in
// ordinary VGPRs (without the bound the compiler splits them across VGPRs and
// AGPRs, and the larger regions fall to one wave per SIMD); the fp32
// off-diagonal 4 x 4-block region and the fp32 6-block diagonal region need
// more than 256 registers and keep the default.
template <int PREC, int RB, bool DIAG>
constexpr int x_min_blocks() {
    return (PREC == kFP32 && ((RB >= 4 && !DIAG) || RB >= 6)) ? 1 : 2;
}

template <int PREC, int RB, bool DIAG>
__global__ __launch_bounds__(256, (x_min_blocks<PREC, RB, DIAG>())) void xstage_kernel(XArgs a) {
    __shared__ float tbuf[4][16 * 17];
    // wave-uniform values live in scalar registers, so the loops have scalar
    // control flow
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    x_wave<PREC, RB, DIAG>(a, blockIdx.x * 4 + w, tbuf[w]);
}

template <int PREC, int RB, bool DIAG>
hipError_t launch_one(const XArgs &a, hipStream_t st) {
    const int64_t waves = (int64_t)a.nregions * a.K * a.nsplit;
    const int grid = (int)((waves + 3) / 4);
    hipLaunchKernelGGL((xstage_kernel<PREC, RB, DIAG>), dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_p(int rb, int diag, const XArgs &a, hipStream_t st) {
    if (diag) {
        switch (rb) {
            case 1: return launch_one<PREC, 1, true>(a, st);
            case 2: return launch_one<PREC, 2, true>(a, st);
            case 3: return launch_one<PREC, 3, true>(a, st);
            case 4: return launch_one<PREC, 4, true>(a, st);
            case 5: return launch_one<PREC, 5, true>(a, st);
            case 6: return launch_one<PREC, 6, true>(a, st);
        }
    } else {
        switch (rb) {
            case 2: return launch_one<PREC, 2, false>(a, st);
            case 3: return launch_one<PREC, 3, false>(a, st);
            case 4: return launch_one<PREC, 4, false>(a, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_xstage(int prec, int rb, int diag, const XArgs &a, hipStream_t st) {
    switch (prec) {
        case kFP32: return launch_p<kFP32>(rb, diag, a, st);
        case kFP16: return launch_p<kFP16>(rb, diag, a, st);
        case kINT8: return launch_p<kINT8>(rb, diag, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace corr
