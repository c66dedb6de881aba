// Internal declarations shared by the host runtime and the kernels of
// libcorr.so.  Nothing here is part of the public ABI (include/corr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace corr {

// Precision codes (mirror enum corr_precision).
constexpr int kFP32 = 0;
constexpr int kFP16 = 1;
constexpr int kINT8 = 2;

// A spectra record is 16 bytes: TG consecutive spectra of one (channel,
// antenna) as [re x TG][im x TG].  Four records (one per MFMA lane group)
// form a k-block of the X-stage.
constexpr int kRecordBytes = 16;
__host__ __device__ constexpr int record_times(int prec) {
    return prec == kFP32 ? 2 : (prec == kFP16 ? 4 : 8);
}
__host__ __device__ constexpr int kblock_times(int prec) { return 4 * record_times(prec); }

// Records are grouped in time blocks of kTQB consecutive records:
// [time block][channel][kTQB records][antenna_pad].  The F-stage's writes of
// one time block stay within K*kTQB*a_pad*16 bytes, and a channel's k-block
// (4 records) is contiguous for the X-stage.
constexpr int kTQB = 16;
__host__ __device__ inline int64_t rec_index(int c, int tq, int a, int K, int a_pad) {
    return (((int64_t)(tq / kTQB) * K + c) * kTQB + (tq % kTQB)) * a_pad + a;
}

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
inline int64_t round_up64(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- F-stage
struct FArgs {
    const uint8_t *in;        // chunk's frames [s][N][M bytes]
    uint4 *spec;              // records, index rec_index(c, tq, a, M, a_pad)
    float *power;             // power mode: partial sums [nwg_per_group][a_pad][M]
    const float *scales;      // int8: [N][M]
    const float2 *tw;         // W_M^j (j < M), then W_2M^q (q < M/2)
    unsigned long long *sat;  // int8 saturation counter
    int N, a_pad, S;          // S = spectra in this chunk
    int ntq;                  // power mode: time tiles in the window
    int ngroups;              // antenna groups of GA covering [0, N)
    int ntiles;               // ntq_used * ngroups (normal mode)
    int tiles_per_wg;         // power mode: time tiles per workgroup
};

// Launch the F-stage for complex length M = K (channels).  mode: 0 = spectra
// records in precision `prec`; 1 = power sums over the calibration window
// (records not written).  Returns hipSuccess or the launch error.
hipError_t launch_fstage(int M, int prec, int ga, int power_mode, const FArgs &a, int grid,
                         hipStream_t st);
int fstage_lds_bytes(int M, int prec, int ga);
// antennas per tile that fill exactly one round of transforms
int fstage_default_group(int M, int prec);

// ---------------------------------------------------------------- X-stage
struct XArgs {
    const uint4 *spec;   // records, index rec_index(c, tq, a, K, a_pad)
    void *partial;       // [nsplit][K][nb] float2 (fp32/fp16) or int2 (int8)
    const int2 *regions; // (I0, J0) block coordinates of each region
    int nregions;
    int N, a_pad, K, ntq, nb;
    int nsplit;
    int nkb;             // k-blocks in the chunk = ntq / 4
};
// rb: region side in 16-antenna blocks; diag: regions on the diagonal
// (upper-triangle pairs only) or off the diagonal (full rb x rb).
hipError_t launch_xstage(int prec, int rb, int diag, const XArgs &a, hipStream_t st);

// ---------------------------------------------------------------- dump etc.
// acc[f][bl] (double2) += sum over splits of partial[sp][f][bl], in split order.
hipError_t launch_dump(int prec, const void *partial, double2 *acc, int nsplit, int K, int nb,
                       hipStream_t st);
// scales[a][f] from power partials summed in order over nparts.
hipError_t launch_scales(const float *power, int nparts, int N, int a_pad, int K, int W,
                         float *scales, hipStream_t st);
// dst[bl][f] = acc[f][bl] (raw layout), then acc = 0.
hipError_t launch_finalize(double2 *acc, double2 *dst, int K, int nb, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);

}  // namespace corr
