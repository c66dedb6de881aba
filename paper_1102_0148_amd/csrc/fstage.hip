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
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int kThreads = 256;
constexpr int kPowerTS = 2;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
    return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
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
    v[5] = make_float2(kC1 * v[5].x + kS1 * v[5].y, kC1 * v[5].y - kS1 * v[5].x);      // W^1
    v[6] = make_float2(kR * (v[6].x + v[6].y), kR * (v[6].y - v[6].x));                // W^2
    v[7] = make_float2(kS1 * v[7].x + kC1 * v[7].y, kS1 * v[7].y - kC1 * v[7].x);      // W^3
    v[9] = make_float2(kR * (v[9].x + v[9].y), kR * (v[9].y - v[9].x));                // W^2
    v[10] = mul_mi(v[10]);                                                              // W^4
    v[11] = make_float2(kR * (v[11].y - v[11].x), -kR * (v[11].x + v[11].y));          // W^6
    v[13] = make_float2(kS1 * v[13].x + kC1 * v[13].y, kS1 * v[13].y - kC1 * v[13].x); // W^3
    v[14] = make_float2(kR * (v[14].y - v[14].x), -kR * (v[14].x + v[14].y));          // W^6
    v[15] = make_float2(-kC1 * v[15].x - kS1 * v[15].y, kS1 * v[15].x - kC1 * v[15].y); // W^9
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

// Orders this wavefront's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stockham pass of radix R (p = product of the radices before it), in place
// in one transform's LDS slot.  Butterfly i reads z[i + r M/R], multiplies by
// W_{pR}^{r k} (k = i mod p), and writes z[(i - k) R + k + r p].
template <int M, int R>
__device__ __forceinline__ void fft_pass(float2 *z, int j, int p, const float2 *twM) {
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
        const int step = k * (M / (p * R));
#pragma unroll
        for (int r = 1; r < R; ++r) v[m * R + r] = cmul(v[m * R + r], twM[(r * step) & (M - 1)]);
        dft_r<R>(&v[m * R]);
        const int base = (i - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) z[pad(base + r * p)] = v[m * R + r];
    }
}

// Signed nibble at bit offset `off` of w.
__device__ __forceinline__ float nib(uint32_t w, int off) {
    return (float)((int)(w << (28 - off)) >> 28);
}

template <int PREC>
__device__ __forceinline__ void stage_store(void *stage, int rec, int ts, float re, float im, float sc,
                                            unsigned &nsat) {
    if constexpr (PREC == kFP32) {
        float *s = reinterpret_cast<float *>(stage) + rec * 4;
        s[ts] = re;
        s[2 + ts] = im;
    } else if constexpr (PREC == kFP16) {
        _Float16 *s = reinterpret_cast<_Float16 *>(stage) + rec * 8;
        s[ts] = (_Float16)re;
        s[4 + ts] = (_Float16)im;
    } else {
        int8_t *s = reinterpret_cast<int8_t *>(stage) + rec * 16;
        float vr = rintf(re * sc), vi = rintf(im * sc);
        nsat += (fabsf(vr) > 127.0f) + (fabsf(vi) > 127.0f);
        vr = fminf(fmaxf(vr, -127.0f), 127.0f);
        vi = fminf(fmaxf(vi, -127.0f), 127.0f);
        s[ts] = (int8_t)(int)vr;
        s[8 + ts] = (int8_t)(int)vi;
    }
}

template <int M, int PREC, int GA, bool POWER>
__global__ __launch_bounds__(kThreads) void fstage_kernel(FArgs args) {
    constexpr int L = M / 16;                  // lanes per transform
    constexpr int FPR = kThreads / L;          // transforms per round
    constexpr int SLOT = M + M / 16 + 1;       // padded float2 per transform
    constexpr int TS = POWER ? kPowerTS : record_times(PREC);
    constexpr int NF = TS * GA;                // transforms per tile
    constexpr int ROUNDS = (NF + FPR - 1) / FPR;
    constexpr int NTASK = FPR * (M / 2);       // output pairs per round
    static_assert(NTASK % kThreads == 0, "task split");
    static_assert(16 % GA == 0, "group divides 16");

    __shared__ float2 zbuf[FPR * SLOT];
    __shared__ __attribute__((aligned(16))) uint32_t bbuf[FPR * (M / 4)];
    __shared__ float2 tw[M + M / 2];
    __shared__ uint4 stage[POWER ? 1 : M * GA];
    __shared__ float pstage[POWER ? M * GA * TS : 1];
    __shared__ float prun[POWER ? M * GA : 1];

    const int tid = threadIdx.x;
    for (int i = tid; i < M + M / 2; i += kThreads) tw[i] = args.tw[i];
    __syncthreads();
    const float2 *twM = tw;
    const float2 *tw2 = tw + M;

    const int fs = tid / L;  // this lane's transform slot
    const int j = tid % L;   // lane within the transform
    float2 *z = zbuf + fs * SLOT;
    uint32_t *bb = bbuf + fs * (M / 4);
    unsigned nsat = 0;

    int tile0 = blockIdx.x, tile1 = args.ntiles, tstep = gridDim.x;
    int pg = 0, pw = 0;
    if constexpr (POWER) {
        // a workgroup owns a run of consecutive time tiles of one antenna group
        const int nblk_t = (args.ntq + args.tiles_per_wg - 1) / args.tiles_per_wg;
        pg = blockIdx.x / nblk_t;
        pw = blockIdx.x % nblk_t;
        tile0 = pw * args.tiles_per_wg;
        tile1 = min(tile0 + args.tiles_per_wg, args.ntq);
        tstep = 1;
        for (int i = tid; i < M * GA; i += kThreads) prun[i] = 0.0f;
        if (pg >= args.ngroups) return;
    }

    for (int tile = tile0; tile < tile1; tile += tstep) {
        int tq, g;
        if constexpr (POWER) {
            tq = tile;
            g = pg;
        } else {
            tq = tile / args.ngroups;
            g = tile % args.ngroups;
        }
#pragma unroll 1
        for (int r = 0; r < ROUNDS; ++r) {
            const int fi = r * FPR + fs;
            const int ts = fi / GA, ga = fi % GA;
            const int s = tq * TS + ts, a = g * GA + ga;
            const bool valid = fi < NF && s < args.S && a < args.N;
            uint4 raw = make_uint4(0u, 0u, 0u, 0u);
            if (valid)
                raw = *reinterpret_cast<const uint4 *>(args.in + ((int64_t)s * args.N + a) * M + 16 * j);
            // dword d of the block goes to (d mod L/4)*16 + d div L/4, so the
            // 16 dwords pass 1 needs in a lane are contiguous
            {
                const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int d = 4 * j + c;
                    bb[(d % (L / 4)) * 16 + d / (L / 4)] = w[c];
                }
            }
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
            if constexpr (M == 128) {
                fft_pass<M, 8>(z, j, 16, twM);
            } else {
                fft_pass<M, 16>(z, j, 16, twM);
                if constexpr (M == 512) {
                    wave_lds_sync();
                    fft_pass<M, 2>(z, j, 256, twM);
                } else if constexpr (M == 1024) {
                    wave_lds_sync();
                    fft_pass<M, 4>(z, j, 256, twM);
                }
            }
            __syncthreads();  // every slot's Z is complete

            // real-input spectrum from Z[q], Z[M-q]; task (slot, q) gives two bins
#pragma unroll 2
            for (int it = 0; it < NTASK / kThreads; ++it) {
                const int t = tid + it * kThreads;
                const int sl = t % FPR;
                const int q = t / FPR;
                const int fi2 = r * FPR + sl;
                if (fi2 >= NF) continue;
                const int ts2 = fi2 / GA, ga2 = fi2 % GA;
                const float2 *zs = zbuf + sl * SLOT;
                float2 xlo, xhi;
                int clo, chi;
                if (q == 0) {
                    const float2 z0 = zs[0], zh = zs[pad(M / 2)];
                    xlo = make_float2(z0.x + z0.y, 0.0f);
                    xhi = make_float2(zh.x, -zh.y);
                    clo = 0;
                    chi = M / 2;
                } else {
                    const float2 z0 = zs[pad(q)], z1 = zs[pad(M - q)];
                    const float2 A = make_float2(z0.x + z1.x, z0.y - z1.y);
                    const float2 B = make_float2(z0.x - z1.x, z0.y + z1.y);
                    const float2 C = cmul(B, tw2[q]);
                    xlo = make_float2(0.5f * (A.x + C.y), 0.5f * (A.y - C.x));
                    xhi = make_float2(0.5f * (A.x - C.y), 0.5f * (-A.y - C.x));
                    clo = q;
                    chi = M - q;
                }
                if constexpr (POWER) {
                    pstage[(clo * GA + ga2) * TS + ts2] = xlo.x * xlo.x + xlo.y * xlo.y;
                    pstage[(chi * GA + ga2) * TS + ts2] = xhi.x * xhi.x + xhi.y * xhi.y;
                } else {
                    float slo = 1.0f, shi = 1.0f;
                    if constexpr (PREC == kINT8) {
                        const int a2 = g * GA + ga2;
                        if (a2 < args.N) {
                            slo = args.scales[(int64_t)a2 * M + clo];
                            shi = args.scales[(int64_t)a2 * M + chi];
                        }
                    }
                    stage_store<PREC>(stage, clo * GA + ga2, ts2, xlo.x, xlo.y, slo, nsat);
                    stage_store<PREC>(stage, chi * GA + ga2, ts2, xhi.x, xhi.y, shi, nsat);
                }
            }
            __syncthreads();  // stage complete; zbuf free for the next round
        }
        if constexpr (POWER) {
            for (int i = tid; i < M * GA; i += kThreads) {
                float acc = prun[i];
#pragma unroll
                for (int t2 = 0; t2 < TS; ++t2) acc += pstage[i * TS + t2];
                prun[i] = acc;
            }
            // the next tile's first barrier orders these reads before new writes
        } else {
            // write-out: GA records of one channel are contiguous in global memory
            for (int i = tid; i < M * GA; i += kThreads) {
                const int c = i / GA, ga2 = i % GA;
                args.spec[((int64_t)c * args.ntq + tq) * args.a_pad + g * GA + ga2] = stage[i];
            }
        }
    }
    if constexpr (POWER) {
        __syncthreads();
        for (int i = tid; i < M * GA; i += kThreads) {
            const int c = i / GA, ga2 = i % GA;
            args.power[((int64_t)pw * args.a_pad + pg * GA + ga2) * M + c] = prun[i];
        }
    }
    if constexpr (PREC == kINT8 && !POWER) {
        if (nsat) atomicAdd(args.sat, (unsigned long long)nsat);
    }
}

template <int M, int PREC, int GA, bool POWER>
hipError_t launch_one(const FArgs &a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((fstage_kernel<M, PREC, GA, POWER>), dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <int M>
hipError_t launch_m(int prec, int ga, int power, const FArgs &a, int grid, hipStream_t st) {
    if (power) return launch_one<M, kFP32, 4, true>(a, grid, st);
    switch (prec * 16 + ga) {
        case kFP32 * 16 + 2: return launch_one<M, kFP32, 2, false>(a, grid, st);
        case kFP32 * 16 + 4: return launch_one<M, kFP32, 4, false>(a, grid, st);
        case kFP16 * 16 + 2: return launch_one<M, kFP16, 2, false>(a, grid, st);
        case kFP16 * 16 + 4: return launch_one<M, kFP16, 4, false>(a, grid, st);
        case kINT8 * 16 + 2: return launch_one<M, kINT8, 2, false>(a, grid, st);
        case kINT8 * 16 + 4: return launch_one<M, kINT8, 4, false>(a, grid, st);
        default: break;
    }
    if constexpr (M <= 512) {
        switch (prec) {
            case kFP32: return launch_one<M, kFP32, 8, false>(a, grid, st);
            case kFP16: return launch_one<M, kFP16, 8, false>(a, grid, st);
            case kINT8: return launch_one<M, kINT8, 8, false>(a, grid, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

int fstage_lds_bytes(int M, int ga) {
    const int L = M / 16, FPR = kThreads / L, SLOT = M + M / 16 + 1;
    return FPR * SLOT * 8 + FPR * M + (M + M / 2) * 8 + M * ga * 16;
}

hipError_t launch_fstage(int M, int prec, int ga, int power_mode, const FArgs &a, int grid,
                         hipStream_t st) {
    if (ga != 2 && ga != 4 && ga != 8) return hipErrorInvalidValue;
    if (M == 1024 && ga == 8 && !power_mode) return hipErrorInvalidValue;
    switch (M) {
        case 128: return launch_m<128>(prec, ga, power_mode, a, grid, st);
        case 256: return launch_m<256>(prec, ga, power_mode, a, grid, st);
        case 512: return launch_m<512>(prec, ga, power_mode, a, grid, st);
        case 1024: return launch_m<1024>(prec, ga, power_mode, a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace corr
