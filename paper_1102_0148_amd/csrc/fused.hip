// Fused F -> X: the F-stage and the X-stage of one integration in one
// persistent kernel, handing chunks of records over through a small ring that
// stays in the caches (the GPU form of moving the FFT and the grouping of
// timeslices ahead of the cross-multiplier, which Section 4 leaves as future
// work).
//
// The kernel is launched cooperatively with as many workgroups as stay
// resident, so every workgroup runs from the start and a wait on another
// workgroup's progress always ends.  A cooperative launch places workgroup b
// on XCD b % 8 and fills the CUs breadth first (b and b + #CUs share a CU),
// so workgroups [0, n_fwg) with n_fwg a multiple of the CU count give every
// CU the same mix of F and X workgroups (mixed layout).  In the split layout
// the roles go by CU instead: CU slot p = b mod #CUs is CU p / 8 of XCD p % 8,
// and the first f_cus CUs of every XCD run only F workgroups, the others only
// X workgroups, which then keep several X waves per SIMD.
//
//   F workgroups: for chunk c = 0, 1, ... take the chunk's tiles one ticket at
//     a time (per-XCD counters, as the standalone F-stage), writing records
//     into ring slot c mod R; before chunk c (c >= R) wait until every X
//     workgroup has finished reading chunk c - R from that slot; after the
//     chunk, count itself on its XCD; the XCD's last F workgroup makes the
//     records visible to every XCD and counts the XCD done.
//   X workgroups: four waves, each one (channel, split) unit whose
//     accumulators stay in registers; for every chunk wait until all eight
//     XCDs have finished it, add the unit's share of its k-blocks, and
//     count the chunk consumed.  A unit writes a partial only every
//     flush_chunks chunks (the float forms' partial-length limits) and at the
//     end; the dump kernel adds the partials afterwards.
//
// Deadlock-free: F waits only for X on a chunk R earlier, X only for F on the
// same chunk, and every workgroup is resident; the smallest chunk any F
// workgroup is on has all of its dependencies finished or finishable.  Waits
// are bounded (about a second) and set the error flag when they give up, so
// every wave always exits.
#include "fstage_dev.h"
#include "xstage_dev.h"

namespace corr {
namespace {

constexpr int fx_group(int M, int prec) {
    return (kThreads / (M / 16)) / record_times(prec) < 1 ? 1 : (kThreads / (M / 16)) / record_times(prec);
}

__device__ __forceinline__ unsigned fx_load(unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *p >= v (bounded), then acquires at agent scope so
// that the data published before the count is visible to this workgroup.
// Once any wait has given up (the error flag is set) every later wait gives
// up at once, so a failed launch still ends within about one wait's limit.
__device__ __forceinline__ void fx_wait(unsigned *p, unsigned v, unsigned *err) {
    unsigned spins = 0;
    while (fx_load(p) < v) {
        if (++spins > kBatchSpinLimit) {
            atomicOr(err, 1u);
            break;
        }
        if ((spins & 255) == 0 && fx_load(err)) break;
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// An F workgroup has finished its tiles of a chunk: every wave's stores
// complete in its XCD's L2, and the workgroup counts itself on its XCD.  The
// last of the XCD's F workgroups writes that L2 back (agent-scope release;
// the other workgroups' records are in the same L2), waits for the
// write-back and counts the XCD done.  One write-back per XCD and chunk, not
// one per workgroup.
__device__ __forceinline__ void fx_publish(unsigned *xcd_count, unsigned per_xcd, unsigned *done) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned before = __hip_atomic_fetch_add(xcd_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1 == per_xcd) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int M, int PREC, int GA>
__device__ __forceinline__ void fx_f_role(const FxArgs &a, float2 *zbuf, uint32_t *bbuf, int *s_tk) {
    const int tg = record_times(PREC);
    const int x = blockIdx.x % 8;
    const int n_xwg = (int)gridDim.x - a.n_fwg;
    const int64_t frame = (int64_t)a.f.N * M;
    for (int c = 0; c < a.nchunks; ++c) {
        unsigned *cc = a.ctr + kFxHdr + (int64_t)c * kFxPerChunk;
        if (c >= a.ring) {
            // the slot is free once every X workgroup has read chunk c - R
            if (threadIdx.x == 0)
                fx_wait(a.ctr + kFxHdr + (int64_t)(c - a.ring) * kFxPerChunk + kFxConsumed, (unsigned)n_xwg, a.err);
            __syncthreads();
        }
        const int Sc = min(a.chunk, a.S - c * a.chunk);
        FArgs fa = a.f;
        fa.spec = a.f.spec + (int64_t)(c % a.ring) * a.slot_recs;
        fa.in = a.f.in + (int64_t)c * a.chunk * frame;
        fa.s_base = c * a.chunk;
        fa.S = Sc;
        const int ntq_used = ((Sc + tg - 1) / tg + 3) / 4 * 4;
        fa.ntiles = ntq_used * fa.ngroups;
        const int t8 = (fa.ntiles + 7) / 8;
        const int lo = x * t8, hi = min(lo + t8, fa.ntiles);
        f_tiles_dyn<M, PREC, GA>(fa, lo, hi, cc + kTicketStride * x, s_tk, zbuf, bbuf);
        fx_publish(cc + kFxXcdDone + kTicketStride * x, (unsigned)(a.n_fwg / 8), cc + kFxDone);
    }
}

template <int PREC, int RB>
__device__ __forceinline__ void fx_x_role(const FxArgs &a, int xrank, float *tb) {
    const int tg = record_times(PREC);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int unit = xrank * 4 + w;
    const bool active = unit < a.x.K * a.x.nsplit;
    const int f = unit % a.x.K, sp = unit / a.x.K;
    XRegion<PREC, RB, true> acc;
    acc.zero();
    int epoch = 0;
    for (int c = 0; c < a.nchunks; ++c) {
        unsigned *cc = a.ctr + kFxHdr + (int64_t)c * kFxPerChunk;
        if (threadIdx.x == 0) fx_wait(cc + kFxDone, 8u, a.err);
        __syncthreads();
        const int Sc = min(a.chunk, a.S - c * a.chunk);
        const int nkb = ((Sc + tg - 1) / tg + 3) / 4;
        if (active) {
            const int kb0 = (int)((int64_t)sp * nkb / a.x.nsplit);
            const int kb1 = (int)((int64_t)(sp + 1) * nkb / a.x.nsplit);
            acc.template run<kFxXBuf>(a.f.spec + (int64_t)(c % a.ring) * a.slot_recs, a.x.K, a.x.a_pad, f, 0, 0,
                                      kb0, kb1);
        }
        // every load of the chunk has returned before the slot can be reused
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(cc + kFxConsumed, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((c + 1) % a.flush_chunks == 0 || c + 1 == a.nchunks) {
            if (active) {
                acc.store(a.x.partial, ((int64_t)(epoch * a.x.nsplit + sp) * a.x.K + f) * a.x.nb, a.x.N, 0, 0, tb);
                acc.zero();
            }
            ++epoch;
        }
    }
}

// Workgroups per CU the kernel's registers are bounded to: up to 512-point
// transforms three, so that two of them run the F-stage beside one X
// workgroup (four made the fp16 and int8 kernels spill); larger transforms
// two.
constexpr int fx_min_blocks(int M, int prec) { return M <= 256 ? 3 : 2; }

template <int M, int PREC, int GA, int RB>
__global__ __launch_bounds__(kThreads, fx_min_blocks(M, PREC)) void fx_kernel(FxArgs kargs) {
    using Sh = FShape<M, PREC, GA, false>;
    static_assert(Sh::LDS <= 160 * 1024, "LDS budget");
    static_assert(Sh::NF * Sh::SLOT * 8 >= 4 * 16 * 17 * 4, "X transposes use the transform slots");
    __shared__ float2 zbuf[Sh::NF * Sh::SLOT];
    __shared__ __attribute__((aligned(16))) uint32_t bbuf[Sh::FPR * (M / 4)];
    __shared__ int s_tk[2];
    const FxArgs &a = kargs;
    const int b = blockIdx.x;
    bool f_role;
    int xrank;  // this workgroup's index among the X workgroups
    if (a.f_cus) {
        const int p = b % a.cus, nf = 8 * a.f_cus;
        f_role = p < nf;
        xrank = (b / a.cus) * (a.cus - nf) + (p - nf);
    } else {
        f_role = b < a.n_fwg;
        xrank = b - a.n_fwg;
    }
    if (f_role) {
        fx_f_role<M, PREC, GA>(a, zbuf, bbuf, s_tk);
    } else {
        float *tb = reinterpret_cast<float *>(zbuf) + (threadIdx.x >> 6) * 16 * 17;
        fx_x_role<PREC, RB>(a, xrank, tb);
    }
}

template <int M, int PREC, int RB>
hipError_t launch_fx(const FxArgs &a, int grid, hipStream_t st) {
    constexpr int GA = fx_group(M, PREC);
    void *args[] = {const_cast<FxArgs *>(&a)};
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(fx_kernel<M, PREC, GA, RB>),
                                              dim3(grid), dim3(kThreads), args, 0, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <int M, int PREC, int RB>
int fx_per_cu() {
    constexpr int GA = fx_group(M, PREC);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fx_kernel<M, PREC, GA, RB>, kThreads, 0) !=
        hipSuccess)
        return 0;
    return per_cu;
}

template <int M, int PREC>
hipError_t launch_fx_mp(int rb, const FxArgs &a, int grid, hipStream_t st) {
    switch (rb) {
        case 1: return launch_fx<M, PREC, 1>(a, grid, st);
        case 2: return launch_fx<M, PREC, 2>(a, grid, st);
        case 3: return launch_fx<M, PREC, 3>(a, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int M, int PREC>
int per_cu_mp(int rb) {
    switch (rb) {
        case 1: return fx_per_cu<M, PREC, 1>();
        case 2: return fx_per_cu<M, PREC, 2>();
        case 3: return fx_per_cu<M, PREC, 3>();
    }
    return 0;
}

template <int M>
hipError_t launch_fx_m(int prec, int rb, const FxArgs &a, int grid, hipStream_t st) {
    switch (prec) {
        case kFP32: return launch_fx_mp<M, kFP32>(rb, a, grid, st);
        case kFP16: return launch_fx_mp<M, kFP16>(rb, a, grid, st);
        case kINT8: return launch_fx_mp<M, kINT8>(rb, a, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int M>
int per_cu_m(int prec, int rb) {
    switch (prec) {
        case kFP32: return per_cu_mp<M, kFP32>(rb);
        case kFP16: return per_cu_mp<M, kFP16>(rb);
        case kINT8: return per_cu_mp<M, kINT8>(rb);
    }
    return 0;
}

}  // namespace

int fused_group(int M, int prec) { return fx_group(M, prec); }

int fused_blocks_per_cu(int M, int prec, int rb) {
    if (rb < 1 || rb > kFxMaxRB) return 0;
    switch (M) {
        case 128: return per_cu_m<128>(prec, rb);
        case 256: return per_cu_m<256>(prec, rb);
        case 512: return per_cu_m<512>(prec, rb);
        case 1024: return per_cu_m<1024>(prec, rb);
    }
    return 0;
}

hipError_t launch_fused(int M, int prec, int rb, const FxArgs &a, int grid, hipStream_t st) {
    switch (M) {
        case 128: return launch_fx_m<128>(prec, rb, a, grid, st);
        case 256: return launch_fx_m<256>(prec, rb, a, grid, st);
        case 512: return launch_fx_m<512>(prec, rb, a, grid, st);
        case 1024: return launch_fx_m<1024>(prec, rb, a, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace corr
