// Batched correlation: many jobs of different N and K in one persistent
// kernel launch (replayed from a captured HIP graph by the host).
//
// The host lays out an ordered work list: calibration power blocks and scale
// ranges (int8 jobs), F-stage tile ranges, X-stage workgroups and dump ranges
// of every job.  Each workgroup repeatedly takes the next ticket; an item
// whose inputs come from earlier items waits on a per-job counter, and a
// finished item increments its counter.  An item only ever waits for items
// with smaller tickets, so the queue always drains (see the kernel).  Counters are bumped with an agent-scope release and read
// with an agent-scope acquire, which carries the data across the XCDs' L2
// caches.
#include "dump_dev.h"
#include "fstage_dev.h"
#include "xstage_dev.h"

namespace corr {
namespace {

constexpr int dga(int M, int prec) {
    return (kThreads / (M / 16)) / record_times(prec) < 1 ? 1 : (kThreads / (M / 16)) / record_times(prec);
}

// Each job type is its own function so that registers are allocated per
// variant rather than for all of them at once.
template <int M, int PREC>
__device__ __noinline__ void f_range(const FArgs &fa, int t0, int t1, char *lds) {
    constexpr int GA = dga(M, PREC);
    using Sh = FShape<M, PREC, GA, false>;
    float2 *zbuf = reinterpret_cast<float2 *>(lds);
    uint32_t *bbuf = reinterpret_cast<uint32_t *>(lds + (Sh::NF * Sh::SLOT * 8 + 15) / 16 * 16);
    f_tiles<M, PREC, GA>(fa, t0, 1, t1, zbuf, bbuf);
}

template <int M>
__device__ __forceinline__ void f_dispatch(const FArgs &fa, int prec, int t0, int t1, char *lds) {
    switch (prec) {
        case kFP32: f_range<M, kFP32>(fa, t0, t1, lds); break;
        case kFP16: f_range<M, kFP16>(fa, t0, t1, lds); break;
        default: f_range<M, kINT8>(fa, t0, t1, lds); break;
    }
}

template <int M>
__device__ __noinline__ void p_block(const FArgs &pa, int blk, char *lds) {
    using Sh = FShape<M, kFP32, power_group(M), true>;
    float2 *zbuf = reinterpret_cast<float2 *>(lds);
    uint32_t *bbuf = reinterpret_cast<uint32_t *>(lds + (Sh::NF * Sh::SLOT * 8 + 15) / 16 * 16);
    f_power_block<M>(pa, blk, zbuf, bbuf);
}

template <int PREC, int RB, bool DIAG>
__device__ __noinline__ void x_one(const XArgs &xa, int wave, float *tb) {
    x_wave<PREC, RB, DIAG>(xa, wave, tb);
}

template <int PREC>
__device__ __forceinline__ void x_dispatch(const XArgs &xa, int rb, bool diag, int wave, float *tb) {
    if (diag) {
        switch (rb) {
            case 1: x_one<PREC, 1, true>(xa, wave, tb); break;
            case 2: x_one<PREC, 2, true>(xa, wave, tb); break;
            default: x_one<PREC, 3, true>(xa, wave, tb); break;
        }
    } else {
        switch (rb) {
            case 1: x_one<PREC, 1, false>(xa, wave, tb); break;
            default: x_one<PREC, 2, false>(xa, wave, tb); break;
        }
    }
}

// Coherent read of a counter without an acquire: the caller spins on this and
// acquires once afterwards (an acquire per iteration would invalidate the L2
// that the rest of the XCD is working out of).
__device__ __forceinline__ unsigned load_relaxed(unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256, 2) void batch_kernel(const BJob *jobs, const uint8_t *const *in_ptrs,
                                                   const BItem *items, int n_items, unsigned *ticket,
                                                   unsigned *ctr, unsigned *err) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    __shared__ int s_item;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Thread 0 only: the ticket of the next item, taken while the current one
    // runs so the atomic's latency hides behind an item (an increment, which
    // the compiler's wave-level atomic rewriting leaves asynchronous), and the
    // last counter wait it satisfied.  Holding one ticket ahead keeps the
    // queue deadlock-free: the smallest unfinished ticket is always some
    // workgroup's current item, and everything it waits for has a smaller
    // ticket, so it is finished.
    unsigned next = 0, seen_val = 0;
    int seen_ctr = -1;
    if (threadIdx.x == 0) next = atomicInc(ticket, 0xffffffffu);
    for (;;) {
        if (threadIdx.x == 0) {
            s_item = (int)next;
            next = atomicInc(ticket, 0xffffffffu);
        }
        __syncthreads();
        const int t = s_item;
        __syncthreads();  // every thread has read s_item before it is reused
        if (t >= n_items) break;
        const BItem it = items[t];
        if (it.wait >= 0) {
            // counters only grow, so a wait this workgroup has already seen
            // satisfied (and acquired) needs neither the spin nor another
            // cache invalidate
            if (threadIdx.x == 0 && !(it.wait == seen_ctr && (unsigned)it.wait_val <= seen_val)) {
                unsigned spins = 0;
                bool ok = true;
                while (load_relaxed(&ctr[it.wait]) < (unsigned)it.wait_val) {
                    if (++spins > kBatchSpinLimit) {
                        atomicOr(err, 1u);
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                // the producers' writes become visible to this workgroup: the
                // acquire invalidates this CU's and this XCD's caches, and the
                // wait keeps every wave's loads after the barrier behind it
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __builtin_amdgcn_s_waitcnt(0x0F70);
                if (ok) {
                    seen_ctr = it.wait;
                    seen_val = (unsigned)it.wait_val;
                }
            }
            __syncthreads();
        }
        const BJob &j = jobs[it.job];
        switch (it.type) {
            case BI_POWER: {
                FArgs pa = j.p;
                pa.in = in_ptrs[it.job];
                switch (j.K) {
                    case 128: p_block<128>(pa, it.a0, lds); break;
                    case 256: p_block<256>(pa, it.a0, lds); break;
                    case 512: p_block<512>(pa, it.a0, lds); break;
                    default: p_block<1024>(pa, it.a0, lds); break;
                }
                break;
            }
            case BI_SCALES:
                for (int e = it.a0 + (int)threadIdx.x; e < it.a1; e += 256)
                    j.scales[e] = scale_one(j.p.power, j.nparts, j.p.a_pad, j.K, j.W, e, kI8CodesPerRms);
                break;
            case BI_F: {
                FArgs fa = j.f;
                fa.in = in_ptrs[it.job];
                switch (j.K) {
                    case 128: f_dispatch<128>(fa, j.prec, it.a0, it.a1, lds); break;
                    case 256: f_dispatch<256>(fa, j.prec, it.a0, it.a1, lds); break;
                    case 512: f_dispatch<512>(fa, j.prec, it.a0, it.a1, lds); break;
                    default: f_dispatch<1024>(fa, j.prec, it.a0, it.a1, lds); break;
                }
                break;
            }
            case BI_XD:
            case BI_XO: {
                const bool diag = it.type == BI_XD;
                const XArgs &xa = diag ? j.xd : j.xo;
                float *tb = reinterpret_cast<float *>(lds) + w * 16 * 17;
                const int wave = it.a0 * 4 + w;
                switch (j.prec) {
                    case kFP32: x_dispatch<kFP32>(xa, diag ? j.rb_d : j.rb_o, diag, wave, tb); break;
                    case kFP16: x_dispatch<kFP16>(xa, diag ? j.rb_d : j.rb_o, diag, wave, tb); break;
                    default: x_dispatch<kINT8>(xa, diag ? j.rb_d : j.rb_o, diag, wave, tb); break;
                }
                break;
            }
            default: {  // BI_DUMP
                const int nsplit = j.xd.nsplit;
                for (int e = it.a0 + (int)threadIdx.x; e < it.a1; e += 256) {
                    if (j.prec == kINT8)
                        dump_one<int2>(reinterpret_cast<const int2 *>(j.xd.partial), j.acc, nsplit, j.n_acc, e);
                    else
                        dump_one<float2>(reinterpret_cast<const float2 *>(j.xd.partial), j.acc, nsplit, j.n_acc, e);
                }
                break;
            }
        }
        // Publish this item's writes, then count it.  Every wave first waits
        // until its own stores have completed in its XCD's L2 (vmcnt(0); a
        // workgroup-scope release does not wait for them), so that thread 0's
        // agent-scope release after the barrier, which writes that L2 back,
        // covers the writes of every wave and not only of wave 0.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (threadIdx.x == 0 && it.sig >= 0) {
            // the agent-scope release writes the L2 back; the wait makes that
            // write-back complete before the count can be seen
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0x0F70);
            __hip_atomic_fetch_add(&ctr[it.sig], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int M, int PREC>
constexpr int f_lds() {
    return f_lds_bytes<M, PREC, dga(M, PREC), false>();
}

}  // namespace

int batch_default_group(int M, int prec) {
    const int g = (kThreads / (M / 16)) / record_times(prec);
    return g < 1 ? 1 : g;
}

int batch_lds_bytes(int M, int prec) {
    int f = 0, p = 0;
    switch (M) {
        case 128:
            f = prec == kFP32 ? f_lds<128, kFP32>() : prec == kFP16 ? f_lds<128, kFP16>() : f_lds<128, kINT8>();
            p = f_lds_bytes<128, kFP32, power_group(128), true>();
            break;
        case 256:
            f = prec == kFP32 ? f_lds<256, kFP32>() : prec == kFP16 ? f_lds<256, kFP16>() : f_lds<256, kINT8>();
            p = f_lds_bytes<256, kFP32, power_group(256), true>();
            break;
        case 512:
            f = prec == kFP32 ? f_lds<512, kFP32>() : prec == kFP16 ? f_lds<512, kFP16>() : f_lds<512, kINT8>();
            p = f_lds_bytes<512, kFP32, power_group(512), true>();
            break;
        default:
            f = prec == kFP32 ? f_lds<1024, kFP32>() : prec == kFP16 ? f_lds<1024, kFP16>() : f_lds<1024, kINT8>();
            p = f_lds_bytes<1024, kFP32, power_group(1024), true>();
            break;
    }
    int x = 4 * 16 * 17 * 4;
    int m = f > p ? f : p;
    return m > x ? m : x;
}

hipError_t batch_prepare(int lds_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(batch_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

int batch_max_blocks(int lds_bytes) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, 256, lds_bytes) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

hipError_t launch_batch(const BJob *jobs, const uint8_t *const *in_ptrs, const BItem *items, int n_items,
                        unsigned *ticket, unsigned *ctr, unsigned *err, int grid, int lds_bytes,
                        hipStream_t st) {
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(256), lds_bytes, st, jobs, in_ptrs, items, n_items, ticket,
                       ctr, err);
    return hipGetLastError();
}

}  // namespace corr
