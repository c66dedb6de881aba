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
constexpr int kINT16 = 3;
// the requantised forms, which take per-(antenna, channel) scales
__host__ __device__ constexpr bool is_quant(int prec) { return prec == kINT8 || prec == kINT16; }
// int16 values: |q| <= 32512 = 255 * 127 + 127, each stored as two int8
// digits in base 255, q = 255 h + l with h, l in [-127, 127]
constexpr int kI16Max = 32512;
// Calibration: the largest code stands for a multiple of the rms of one
// component over the window, 4 rms for int8 (127 / 4 codes per rms) and
// 8 rms for int16 (32512 / 8 = 4064), where a Gaussian component clips with
// probability about 1e-15 and the 16-bit word buys precision rather than range.
constexpr float kI8CodesPerRms = 127.0f / 4.0f;
constexpr float kI16CodesPerRms = (float)kI16Max / 8.0f;
// spectra one int16 partial may sum: every digit sum stays below 2^31 (the
// cross sum adds 4 digit products per spectrum: 4 * 16384 * 127^2 < 2^31)
constexpr int kI16SplitSpectra = 16384;
// spectra one float partial may sum: the fp32 form's three-product
// combination Im = P3 - P1 + P2 cancels, so its error grows with the length
// of the sum, faster with stronger correlations (in coefficient units, 2e-6
// at 4096 for a weak common signal at N = 44, but 6e-5 at 4096 for three
// delayed sources at N = 256); the fp16 form's error is its half-precision
// spectra's at any length up to 16384
constexpr int kF32SplitSpectra = 2048;
constexpr int kF16SplitSpectra = 16384;

// A spectra record is 16 bytes: TG consecutive spectra of one (channel,
// antenna) as [re x TG][im x TG].  Four records (one per MFMA lane group)
// form a k-block of the X-stage.
constexpr int kRecordBytes = 16;
__host__ __device__ constexpr int record_times(int prec) {
    return prec == kFP32 ? 2 : (prec == kINT8 ? 8 : 4);
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

// Word 3 of a raw buffer resource on this target (no format conversion, no
// swizzle): stores at offsets past the resource's byte range are dropped.
constexpr int kBufferRsrcFlags = 0x00020000;
// Bytes allocated past the last record time block (see the F-stage's stores).
constexpr size_t kSpecSlack = 256;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Orders this wavefront's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline int64_t round_up64(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- F-stage
struct FArgs {
    const uint8_t *in;        // chunk's frames [s][N][M bytes]
    const uint8_t *const *in_slot;  // if set, `in` is read from here at run time (graph replays)
    uint4 *spec;              // records, index rec_index(c, tq, a, M, a_pad)
    float *power;             // power mode: partial sums [nwg_per_group][a_pad][M]
    const float *scales;      // int8: [N][M]
    const float2 *tw;         // W_M^j (j < M), W_2M^q (q < M/2), then M zero bytes
    unsigned long long *sat;  // int8 saturation counter
    unsigned *ticket;         // records mode: 8 tile-chunk counters, zero at launch
    const double4 *track;     // tracking model per antenna (a_pad entries), or null
    int s_base;               // integration index of the chunk's first spectrum
    int N, a_pad, S;          // S = spectra in this chunk
    int ntq;                  // power mode: time tiles in the window
    int ngroups;              // antenna groups of GA covering [0, N)
    int ntiles;               // ntq_used * ngroups (normal mode)
    int tiles_per_wg;         // power mode: time tiles per workgroup
};

// Tile-chunk ticket counters of the records-mode F-stage: one per XCD, each on
// its own 128-byte line.
constexpr int kTicketStride = 32;
constexpr size_t kTicketBytes = 8 * kTicketStride * sizeof(unsigned);

// Launch the F-stage for complex length M = K (channels).  mode: 0 = spectra
// records in precision `prec`, over as many persistent workgroups as stay
// resident (`grid` ignored; a.ticket zeroed first, on the same stream; with
// a.track set, the records are rotated by the tracking model);
// 1 = power sums over the calibration window (records not written), `grid`
// blocks.  Returns hipSuccess or the error.
hipError_t launch_fstage(int M, int prec, int ga, int power_mode, const FArgs &a, int grid,
                         hipStream_t st);
int fstage_lds_bytes(int M, int prec, int ga);
// antennas per tile that fill exactly one round of transforms
int fstage_default_group(int M, int prec);

// ---------------------------------------------------------------- X-stage
// A group of X regions that share their antenna blocks (large N, regions of
// 4 x 4 blocks): the blocks of rows [r0, r0 + 8) and columns [c0, c0 + 8)
// (the same range when diag) are staged in LDS once per k-block for all of
// the group's regions, one region per wave.
struct XGroup {
    int r0, c0;          // first block of the row range and of the column range
    int diag;            // 1: column range = row range (8 blocks staged), 0: 16
    int nreg;            // regions in the group (3 or 4)
    int2 reg[4];         // (I0, J0) block coordinates of each region
    int kind[4];         // 1: diagonal region (upper triangle), 0: off-diagonal
};

// The regions of rb x rb antenna blocks that tile the triangle of nr region
// rows: the nr diagonal regions first, then the off-diagonal ones row by row.
__host__ __device__ inline int region_count(int nr) { return nr * (nr + 1) / 2; }
__host__ __device__ inline int2 region_at(int idx, int nr, int rb) {
    if (idx < nr) return make_int2(idx * rb, idx * rb);
    idx -= nr;
    for (int i = 0; i < nr; ++i) {
        const int in_row = nr - 1 - i;
        if (idx < in_row) return make_int2(i * rb, (i + 1 + idx) * rb);
        idx -= in_row;
    }
    return make_int2(0, 0);
}

// Region groups sharing their blocks, for 4 x 4-block regions in an even
// number nr of region rows: region rows 2i and 2i+1 give a diagonal group
// (two diagonal regions and the off-diagonal one between them, 8 blocks) and,
// with region columns 2j and 2j+1 (j > i), an off-diagonal group of four
// regions (16 blocks).  Together they tile the triangle.  Listed per pair of
// region rows: the diagonal group, then the off-diagonal ones.
__host__ __device__ inline int group_count(int nr) { return (nr / 2) * (nr / 2 + 1) / 2; }
__host__ __device__ inline XGroup group_at(int idx, int nr) {
    XGroup g{};
    const int h = nr / 2;
    for (int ii = 0; ii < h; ++ii) {
        const int in_row = h - ii;
        if (idx >= in_row) {
            idx -= in_row;
            continue;
        }
        const int i = 2 * ii;
        if (idx == 0) {
            g.r0 = g.c0 = 4 * i;
            g.diag = 1;
            g.nreg = 3;
            g.reg[0] = make_int2(4 * i, 4 * i);
            g.kind[0] = 1;
            g.reg[1] = make_int2(4 * i, 4 * i + 4);
            g.kind[1] = 0;
            g.reg[2] = make_int2(4 * i + 4, 4 * i + 4);
            g.kind[2] = 1;
        } else {
            const int j = i + 2 * idx;
            g.r0 = 4 * i;
            g.c0 = 4 * j;
            g.nreg = 4;
            for (int k = 0; k < 4; ++k) {
                g.reg[k] = make_int2(4 * i + 4 * (k / 2), 4 * j + 4 * (k % 2));
                g.kind[k] = 0;
            }
        }
        return g;
    }
    return g;
}
// Region groups are used for 4 x 4-block regions in an even number (>= 2) of
// region rows.
__host__ __device__ inline bool uses_groups(int rb, int nr) { return rb == 4 && nr >= 2 && nr % 2 == 0; }

struct XArgs {
    const uint4 *spec;   // records, index rec_index(c, tq, a, K, a_pad)
    void *partial;       // [nsplit][K][nb] float2 (fp32/fp16) or int2 (int8)
    const int2 *regions; // (I0, J0) block coordinates of each region
    int nregions;
    int n_diag;          // launches of both kinds: regions [0, n_diag) are diagonal
    int N, a_pad, K, ntq, nb;
    int nsplit;
    int nkb;             // k-blocks in the chunk = ntq / 4
    const XGroup *groups; // group launches: the region groups of a channel
    int ngroups;
};
// rb: region side in 16-antenna blocks; kind 1: regions on the diagonal
// (upper-triangle pairs only), 0: off the diagonal (full rb x rb), 2: both,
// the first a.n_diag regions diagonal (rb 2..4).
hipError_t launch_xstage(int prec, int rb, int kind, const XArgs &a, hipStream_t st);
// int8 / fp16 with 4 x 4-block regions: one workgroup per (group, channel,
// split), the group's blocks staged through an LDS ring (a.groups).
hipError_t launch_xgroups(int prec, const XArgs &a, hipStream_t st);
// int8 / fp16 with 4 x 4-block regions in exactly 4 region rows (16 blocks):
// one workgroup per (channel, split) stages all 16 blocks of a k-block.
hipError_t launch_xchan(int prec, const XArgs &a, hipStream_t st);
// int16 (also reached through launch_xstage): rb <= 3 diagonal, rb <= 2 off
// the diagonal; a.nkb even; partials are double2 (exact integers).
hipError_t launch_xstage16(int rb, int kind, const XArgs &a, hipStream_t st);

// ---------------------------------------------------------------- fused F -> X
// One persistent kernel, launched cooperatively (every workgroup resident):
// workgroups [0, n_fwg) run the F-stage chunk by chunk into a ring of record
// slots, the others are X workers whose four waves each own one (channel,
// split) unit and keep its accumulators in registers across the chunks.  A
// chunk's records are read while they are still in the caches, and the
// X-stage's prologue, epilogue and partial writes are paid once per
// integration (or once per flush, for the float forms' accuracy) instead of
// once per chunk.  Single-region shapes only (at most 6 antenna blocks).
struct FxArgs {
    FArgs f;             // in: the whole integration; spec: the ring's first slot
    XArgs x;             // partial, N, a_pad, K, nb; nsplit = splits per channel
    unsigned *ctr;       // counters (layout below), zero at launch
    unsigned *err;       // set when a wait gives up (sticky: not cleared per launch)
    int S;               // spectra in the integration
    int chunk;           // spectra per chunk (a multiple of 64)
    int nchunks;
    int ring;            // slots in the ring
    int64_t slot_recs;   // records (uint4) per slot
    int n_fwg;           // workgroups that run the F-stage
    int flush_chunks;    // X units start a new partial every this many chunks
    int cus;             // CUs of the device (workgroup b runs on CU slot b mod cus)
    int f_cus;           // 0: workgroups [0, n_fwg) run F on every CU; else the
                         // first f_cus CUs of each XCD run only F, the rest only X
};
// Counter words: per chunk c from kFxHdr + c kFxPerChunk: the eight per-XCD
// tile tickets, the eight per-XCD counts of F workgroups that finished the
// chunk (kTicketStride apart), then `done` (XCDs whose F workgroups all
// finished it and whose L2 has been written back) and `consumed` (X
// workgroups that finished it), each on a 128-byte line of its own.
constexpr int kFxHdr = 32;
constexpr int kFxXcdDone = 8 * kTicketStride;
constexpr int kFxDone = kFxXcdDone + 8 * kTicketStride;
constexpr int kFxConsumed = kFxDone + 32;
constexpr int kFxPerChunk = kFxConsumed + 32;
// Register sets of an X worker's prefetch ring (a fused X wave runs alone on
// its SIMD, so it keeps three k-blocks in flight).
constexpr int kFxXBuf = 4;
// Largest region side (in 16-antenna blocks) the fused kernel is built for.
constexpr int kFxMaxRB = 3;
// The chunk's spin limit is the batch kernel's (about a second).
hipError_t launch_fused(int M, int prec, int rb, const FxArgs &a, int grid, hipStream_t st);
// Workgroups of the fused kernel that stay resident per CU (0 if the
// combination is not built), and its F group.
int fused_blocks_per_cu(int M, int prec, int rb);
int fused_group(int M, int prec);

// ---------------------------------------------------------------- dump etc.
// acc[f][bl] (double2) += sum over splits of partial[sp][f][bl], in split order.
hipError_t launch_dump(int prec, const void *partial, double2 *acc, int nsplit, int K, int nb,
                       hipStream_t st);
// scales[a][f] from power partials summed in order over nparts; the mean
// power divides by W spectra, or by *w_valid when given (the spectra of the
// window that arrived, counted on the device by the frame ingest), and by the
// channel's non-zero components (1 for DC, else 2); scale = codes_per_rms / rms.
hipError_t launch_scales(const float *power, int nparts, int N, int a_pad, int K, int W,
                         const unsigned *w_valid, float codes_per_rms, float *scales, hipStream_t st);
// dst[bl][f] = acc[f][bl] (raw layout), then acc = 0.
hipError_t launch_finalize(double2 *acc, double2 *dst, int K, int nb, hipStream_t st);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st);

// ---------------------------------------------------------------- ingest
// Counters of one ingest: accepted frames, rejected frames, lost spectra,
// spectra received in the calibration window.
constexpr size_t kIngestCounterBytes = 4 * sizeof(unsigned);
// Assemble S spectra of N x K bytes into `out` from n_frames frames (header
// and payload as in corr.h) at `stride` bytes: `owner` (S entries rounded up
// to a multiple of 4) and `counters` are scratch, cleared here; W is the
// calibration window.
hipError_t launch_ingest(const uint8_t *frames, int64_t n_frames, int64_t stride, uint64_t first_seq, int S,
                         int N, int K, int W, unsigned *owner, unsigned *counters, uint8_t *out, hipStream_t st);

// ---------------------------------------------------------------- batch
// One correlation job of a batch, as the persistent kernel sees it.  F-stage
// tiles use the group that fills one round of transforms; X regions are at
// most 3 blocks on a side (diagonal) or 2 (off the diagonal).
struct BJob {
    FArgs f;             // records (f.in is taken from the call's pointer table)
    FArgs p;             // calibration power sums (int8)
    XArgs xd, xo;        // X-stage over the diagonal / off-diagonal regions
    double2 *acc;        // integration buffer [K][nb]
    float *scales;
    int K, prec, rb_d, rb_o;
    int n_acc;           // K * nb
    int W, nparts;       // calibration window and power partials
    int sc_n;            // N * K scale entries
};

// A work item; `wait` counter must reach wait_val before the item runs and
// `sig` counter is incremented when it is done (-1: none).
enum { BI_POWER = 0, BI_SCALES, BI_F, BI_XD, BI_XO, BI_DUMP };
struct BItem {
    int type, job;
    int a0, a1;          // power block | scale range | tile range | X workgroup | dump range
    int wait, wait_val, sig, pad;
};
constexpr int kBatchCounters = 5;  // per job: power, scales, F, X, dump

// Tiles per F item (at least 16, and at most 64 once a job has enough tiles
// to keep every workgroup busy), elements per scale and per dump item.
constexpr int kBatchTilesPerItem = 16;
constexpr int kBatchMaxTilesPerItem = 64;
constexpr int kBatchScaleElemsPerItem = 256;
constexpr int kBatchElemsPerItem = 2048;
// spin limit of a dependency wait (about a second); past it the kernel
// records an error and goes on, so every wave always exits
constexpr unsigned kBatchSpinLimit = 1u << 22;

int batch_default_group(int M, int prec);
int batch_lds_bytes(int M, int prec);
hipError_t batch_prepare(int lds_bytes);
int batch_max_blocks(int lds_bytes);
hipError_t launch_batch(const BJob *jobs, const uint8_t *const *in_ptrs, const BItem *items, int n_items,
                        unsigned *ticket, unsigned *ctr, unsigned *err, int grid, int lds_bytes,
                        hipStream_t st);

}  // namespace corr
