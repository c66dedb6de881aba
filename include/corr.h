/*
 * corr.h -- C ABI of the MI355X FX spectral correlator (libcorr.so).
 *
 * The library computes, for N antennas of 4-bit real samples, the cross power
 * spectra of every antenna pair in every channel (Prasad & Subrahmanya,
 * Section 1): each 2K-sample block of each antenna is Fourier transformed into
 * K channels (the F-stage), the spectra are turned channel-major, and every
 * pair is cross-multiplied and accumulated over the spectra of an integration
 * (the X-stage).  Each time tile's partial result is added into a float64
 * integration buffer.  Around that path: the X-stage arithmetic (float32,
 * half, or spectra requantised to 8 or 16 bits), per-antenna delay and phase
 * tracking applied before accumulation, assembly of an integration from
 * self-contained frames that may be lost, repeated or reordered, and batches
 * of uneven jobs replayed from one HIP graph.
 *
 * Conventions common to every entry point:
 *   - Input frames: byte layout [spectrum][antenna][K bytes]; one antenna
 *     block holds 2K samples, two per byte, two's-complement nibbles -8..7,
 *     the low nibble being the earlier sample (Section 2.2: one frame carries
 *     contiguous samples of all elements and is one FFT block; Section 1:
 *     4-bit quantisation).
 *   - Transform: forward, unnormalised, no window (Section 4); channels are
 *     bins 0..K-1 of the 2K-point real transform (the Nyquist bin is dropped).
 *   - Visibilities: V[a,b,k] = sum_s X[s,a,k] * conj(X[s,b,k]) for a <= b,
 *     autos included.  Baseline index bl(a,b) = a*N - a*(a-1)/2 + (b-a)
 *     (upper triangle, row-major).  Output arrays are [baseline][channel]
 *     complex values, real part first.  The imaginary part of an auto is
 *     exactly 0.
 *   - Ownership: the caller owns every buffer it passes in; device input must
 *     stay valid until the stream has passed the call that consumed it.  The
 *     library owns its scratch (spectra chunk, partials, integration buffer,
 *     scales, twiddles) and frees it in corr_destroy.
 *   - Errors: functions return CORR_OK (0) or a negative status; creators
 *     return NULL.  corr_last_error() gives a thread-local message.  An
 *     asynchronous GPU error surfaces as CORR_EHIP on a later call.
 *   - Threading: a handle is not thread-safe; use one handle per stream.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef CORR_H
#define CORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct corr_ctx *corr_handle;

enum corr_status {
    CORR_OK = 0,
    CORR_EINVAL = -1, /* bad argument: size, pointer, mode, job index */
    CORR_ENOMEM = -2, /* device or host allocation failed */
    CORR_EHIP = -3,   /* the HIP runtime reported an error */
    CORR_ESTATE = -4  /* call not allowed in the handle's current state */
};

/* Arithmetic of the X-stage.  FP32: float spectra, float products and sums.
 * FP16: spectra rounded to half (ties to even), float accumulation.  INT8:
 * spectra requantised per antenna and channel (Section 4's conversion to a
 * short integer type with prescaling, here to 8 bits), exact int32 sums.
 * INT16: the same requantisation to 16 bits (the paper's short complex type;
 * codes within +-32512), products summed exactly (int32 digit sums combined
 * into exact integers); needs x_splits >= chunk_spectra / 16384, which the
 * default satisfies; not available in batches.  */
enum corr_precision { CORR_FP32 = 0, CORR_FP16 = 1, CORR_INT8 = 2, CORR_INT16 = 3 };

/* Limits checked by corr_create.  */
#define CORR_MAX_ANTENNAS 512
#define CORR_MIN_CHANNELS 128
#define CORR_MAX_CHANNELS 1024
/* int8 calibration window: the first min(n_spectra, CORR_CALIB_SPECTRA)
 * spectra of each integration set the scales of that integration.  */
#define CORR_CALIB_SPECTRA 1024

/* Create a correlator for N antennas, K channels (a 2K-point transform;
 * Section 1 counts K complex multipliers per 2K-point transform), and
 * integrations of n_spectra spectra.  2 <= N <= CORR_MAX_ANTENNAS; K a power
 * of two in [CORR_MIN_CHANNELS, CORR_MAX_CHANNELS]; 1 <= n_spectra <= 2^24
 * (int8 also needs n_spectra <= 65536 so every int32 partial is exact).
 * Allocates all device scratch on the current HIP device.  Precision starts
 * as CORR_FP32.  NULL on error.  */
corr_handle corr_create(int N, int K, int n_spectra);

/* Select the X-stage arithmetic (enum corr_precision).  Allowed only before
 * the first corr_process / corr_process_spectra, else CORR_ESTATE.  */
int corr_set_precision(corr_handle h, int mode);

/* Tile and chunk choices (written by the autotuner; 0 keeps the default).
 *   chunk_spectra: spectra per F->X chunk (multiple of 64).
 *   x_splits:      time splits of one chunk in the X-stage (partials per
 *                  channel per chunk; 1..64).
 *   f_group:       antennas per F-stage tile (2, 4 or 8).
 * Allowed only before the first process call, else CORR_ESTATE.  */
typedef struct {
    int chunk_spectra;
    int x_splits;
    int f_group;
} corr_tiles;
int corr_set_tiles(corr_handle h, const corr_tiles *t);
int corr_get_tiles(corr_handle h, corr_tiles *t);

/* How corr_process runs an integration (Section 4 leaves moving the FFT and
 * the timeslice grouping ahead of the cross-multiplier as future work; the
 * fused pipeline is that, on one GPU):
 *   CORR_PIPELINE_STAGED (default): per chunk of chunk_spectra spectra an
 *     F-stage launch writes the chunk's records, an X-stage launch reads them
 *     into partials and a dump adds those into float64.
 *   CORR_PIPELINE_FUSED: one persistent kernel per integration (launched
 *     cooperatively: all its workgroups resident).  Some workgroups transform
 *     chunks of chunk_spectra spectra into a ring of ring_slots record
 *     buffers small enough to stay in the caches; the others are X workers
 *     whose accumulators stay in registers across all chunks and are written
 *     out once (float forms: every 2048 (FP32) / 16384 (FP16) spectra of a
 *     partial); one dump follows.  Two layouts of the roles:
 *       mixed (f_cus_per_xcd = 0): every CU runs f_workgroups_per_cu F
 *         workgroups and its other resident workgroups run X;
 *       split (f_cus_per_xcd > 0): the first f_cus_per_xcd CUs of each XCD
 *         run only F workgroups and the other CUs only X workgroups
 *         (f_workgroups_per_cu must then be 0; at most CUs per XCD - 1).
 *     FP32, FP16 and INT8 with N <= 48; no delay / phase tracking; not in
 *     batches.  Results: INT8 identical to the staged pipeline, FP32 / FP16
 *     within their tolerance.
 * 0 for chunk_spectra (a multiple of 64), ring_slots (1..8) or
 * f_workgroups_per_cu picks a default; 0 for f_cus_per_xcd is the mixed
 * layout.  Both layout arguments non-zero: CORR_EINVAL.  Before the first process call only
 * (CORR_ESTATE after); a shape or precision the fused kernel does not cover
 * fails the first process call (and corr_get_tiles) with CORR_EINVAL.  With
 * FUSED, corr_get_tiles reports chunk_spectra, the partials per channel in
 * x_splits and the F group.  */
#define CORR_PIPELINE_STAGED 0
#define CORR_PIPELINE_FUSED 1
int corr_set_pipeline(corr_handle h, int pipeline, int chunk_spectra, int ring_slots, int f_workgroups_per_cu,
                      int f_cus_per_xcd);

/* Correlate one integration.  packed_samples: DEVICE pointer to
 * n_spectra*N*K bytes in the frame layout above.  Enqueues the whole F + X +
 * dump sequence on `stream` and returns without waiting; the result is added
 * into the handle's float64 integration buffer.  For INT8 the scales are
 * recomputed from this call's calibration window first.  */
int corr_process(corr_handle h, const void *packed_samples, void *stream);

/* Frames (Section 2.2: each packet is one FFT block of every element and is
 * self-contained, its header carrying the sample timing, the datatype and
 * the number of elements; packets are striped over several links, so they can
 * be lost, repeated or out of order).  A frame is a 32-byte header followed
 * by the block's N*K payload bytes in the corr_process layout ([antenna][K
 * bytes]).  All fields little-endian.  */
#define CORR_FRAME_MAGIC 0x4D52464Fu /* bytes "OFRM" */
#define CORR_FRAME_VERSION 1
#define CORR_DTYPE_INT4 1 /* two's-complement nibbles, low nibble first */
#define CORR_FRAME_HEADER_BYTES 32
typedef struct {
    uint32_t magic;      /* CORR_FRAME_MAGIC */
    uint16_t version;    /* CORR_FRAME_VERSION */
    uint16_t datatype;   /* CORR_DTYPE_INT4 */
    uint64_t seq;        /* block number: time of the first sample / 2K samples */
    uint32_t n_elements; /* N */
    uint32_t n_samples;  /* 2K samples per element */
    uint64_t reserved;   /* 0 */
} corr_frame_header;

typedef struct {
    int64_t frames_accepted;  /* valid headers inside the integration's range */
    int64_t frames_rejected;  /* bad magic, version, datatype, N or 2K, or seq out of range */
    int64_t frames_duplicate; /* accepted but not used: a lower-index frame had the same seq */
    int64_t spectra_lost;     /* spectra no frame arrived for (zero-filled) */
} corr_ingest_stats;

/* Assemble one integration of n_spectra spectra from frames.  frames: DEVICE
 * buffer, 16-byte aligned, frame i at frames + i * frame_stride (stride a
 * multiple of 16, at least 32 + N*K).  out: DEVICE buffer of n_spectra*N*K
 * bytes, 16-byte aligned, written in the corr_process layout.  Frame i is
 * accepted when its header has the magic, version and datatype above,
 * n_elements == N, n_samples == 2K and first_seq <= seq < first_seq +
 * n_spectra; it fills spectrum seq - first_seq.  Of several accepted frames
 * for one spectrum the lowest i is used, so the result does not depend on
 * scheduling.  A spectrum with no accepted frame is zero-filled, and adds
 * nothing to the correlation.  Enqueued on `stream`; the counts are read
 * with corr_get_ingest_stats.  The handle's next corr_process treats this
 * integration's lost spectra as lost: its INT8 calibration divides by the
 * spectra received in the window, not by the window's length (enqueue it on
 * the same stream, or order the two streams).  n_frames may be 0
 * (everything lost).  CORR_EINVAL for bad pointers, alignment, stride or
 * count.  */
int corr_ingest(corr_handle h, const void *frames, int64_t n_frames, int64_t frame_stride, uint64_t first_seq,
                void *out, void *stream);
/* Counts of the last corr_ingest; waits for its stream.  CORR_ESTATE if
 * there was none.  */
int corr_get_ingest_stats(corr_handle h, corr_ingest_stats *out);

/* Delay and phase tracking (Section 2.1: where the signal path disperses, a
 * phase has to be applied to each subband before accumulation in time).
 * Before the spectra are accumulated, channel k of antenna a's spectrum s
 * (s counted from 0 in every integration) is multiplied by exp(2 pi i rho),
 *     rho = k (delay[a] + delay_rate[a] s) / (2K) + phase[a] + phase_rate[a] s
 * with delays in samples, delay rates in samples per spectrum, phases in
 * turns and phase rates in turns per spectrum.  A delay of d samples undoes a
 * delay of the antenna's signal by d samples (a circular shift of each
 * 2K-sample block by d is undone exactly), so baseline (a, b) is turned by
 * rho_a - rho_b.  Arguments: HOST arrays of N doubles each, copied before
 * return; NULL stands for zeros, and four NULLs switch tracking off.  Applies
 * to the corr_process calls after it (the copy to the device is ordered on
 * their stream), not to corr_process_spectra.  INT8 scales are unaffected
 * (a rotation keeps |X|).  CORR_EINVAL for a non-finite value.  */
int corr_set_tracking(corr_handle h, const double *delay, const double *delay_rate, const double *phase,
                      const double *phase_rate);

/* Read the integration buffer and clear it.  Waits for `the last stream`
 * used with this handle.  out: HOST pointer to nb*K*2 floats, nb =
 * N(N+1)/2, layout [baseline][channel][re, im], in the units of the
 * unnormalised transform (INT8 and INT16 values are divided by s_a*s_b,
 * the two antennas' scales).  CORR_ESTATE if nothing was processed since the last
 * read, and for INT8 / INT16 sums that no calibration has scaled (spectra
 * given to corr_process_spectra only: read those with corr_read_cps_raw).  */
int corr_read_cps(corr_handle h, float *out);

/* As corr_read_cps but the float64 buffer as it is: for INT8 and INT16 the
 * exact integer sums in quantised units.  out: HOST pointer to nb*K*2 doubles.  */
int corr_read_cps_raw(corr_handle h, double *out);

/* Asynchronous read: enqueue on `stream` a copy of the raw float64 buffer
 * (layout as corr_read_cps_raw) into dst -- a DEVICE pointer, or pinned host
 * memory -- then clear the buffer.  Does not wait.  */
int corr_read_cps_async(corr_handle h, double *dst, void *stream);

/* INT8 and INT16 only: the scales [N][K] (float) used by the last
 * integration.  out: HOST pointer.  Waits for the handle's stream.
 * CORR_ESTATE for the float forms, and before the first calibrated
 * integration (corr_process or a batch replay; corr_get_tiles and
 * corr_process_spectra calibrate nothing).  */
int corr_read_scales(corr_handle h, float *out);

/* Bytes of spectra in the library layout for n_spectra spectra (the size of
 * the buffer corr_process_spectra reads and corr_debug_read_spectra writes),
 * or 0 on error.  Layout: records of 16 bytes indexed
 * [tq / 16][channel][tq mod 16][antenna_pad], tq = t / TG, antenna_pad = N
 * rounded up to 16 (to 64 above 96 antennas), tq padded to a multiple of 16;
 * a record holds TG consecutive spectra of one antenna and channel as
 * [re x TG][im x TG] in the precision's type (float, TG=2; half, TG=4; int8,
 * TG=8).  INT16 (TG=4) stores each code q as base-255 digits q = 255 h + l,
 * h and l int8 in [-127, 127]: [h of re x4][h of im x4][l of re x4][l of im
 * x4].  Records of padding antennas, and of spectra from n_spectra up to the
 * next multiple of 4*TG (8*TG for INT16), must be zero.  */
size_t corr_spectra_bytes(corr_handle h, int n_spectra);

/* X-stage + dump only, on n_spectra spectra already in the library layout
 * (DEVICE pointer, corr_spectra_bytes(h, n_spectra) bytes).  Adds into the
 * integration buffer like corr_process; INT8 and INT16 spectra are taken as
 * given (no calibration).  The x_splits of the handle's tiles were sized for
 * chunk_spectra; a longer n_spectra runs as consecutive ranges of whole time
 * blocks, each short enough that no partial sums more spectra than its form
 * allows (2048 for FP32, 16384 for FP16 and INT16; the INT16 bound keeps the
 * int32 digit sums exact).  */
int corr_process_spectra(corr_handle h, const void *spectra, int n_spectra, void *stream);

/* Copy the spectra of the last chunk the F-stage produced (library layout)
 * to HOST memory `out` (corr_spectra_bytes(h, *n_spectra) bytes; pass
 * out = NULL to query *n_spectra only).  Waits for the stream.  For tests.  */
int corr_debug_read_spectra(corr_handle h, void *out, int *n_spectra);

/* Counters and, when timing is on, per-stage GPU time summed over the calls
 * since timing was enabled (HIP events recorded on the caller's stream around
 * each stage; they are read, which waits for them, only here).  */
typedef struct {
    int64_t spectra_accumulated; /* spectra in the integration buffer */
    int64_t int8_saturated;      /* components clamped to the largest code (INT8: +-127, INT16: +-32512) */
    int precision;
    int chunk_spectra, x_splits, f_group;
    double ms_calib, ms_f, ms_x, ms_dump; /* 0 unless timing is on */
    int64_t launches_f, launches_x;
    double ms_fused;                      /* fused pipeline: the F + X kernel */
    int64_t launches_fused;
} corr_stats;
int corr_get_stats(corr_handle h, corr_stats *out);
/* on != 0: record HIP events around each stage (adds a little launch work). */
int corr_enable_timing(corr_handle h, int on);

/* Wait for the stream, free everything.  NULL-safe.  */
void corr_destroy(corr_handle h);

/* Thread-local message of the last failure ("" if none).  */
const char *corr_last_error(void);

/* ----------------------------------------------------------------- batch
 * Many independent correlations of different N and K run from one captured
 * HIP graph, replayed by each corr_batch_process (no counterpart in the
 * paper; the closest is Section 3.1's replication of core pairs to absorb
 * more elements or bandwidth).  Each job follows the single-job semantics
 * above.  Two ways to run the jobs (corr_batch_set_mode):
 *   CORR_BATCH_BRANCHES   (default) each job's own F-stage, X-stage and dump
 *                         kernels, the jobs spread over four parallel branches
 *                         of the graph;
 *   CORR_BATCH_PERSISTENT one persistent kernel over an ordered work list of
 *                         every job's F, X and dump items (one launch). */
#define CORR_BATCH_BRANCHES 0
#define CORR_BATCH_PERSISTENT 1
typedef struct {
    int N;
    int K;
    int n_spectra;
    int precision;
} corr_job;

/* Create a batch of n_jobs (1..64) jobs with the same limits as corr_create.
 * Tile choices come from the autotuner's table (corr_batch_set_tiles), else
 * defaults.  NULL on error.  */
corr_handle corr_batch_create(const corr_job *jobs, int n_jobs);
/* Tiles of one job, checked as by corr_set_tiles.  In CORR_BATCH_BRANCHES
 * mode a job runs its tiles as a single correlator would.  The persistent
 * kernel runs every job as one chunk with the F group it is compiled for, so
 * in CORR_BATCH_PERSISTENT mode chunk_spectra must be 0 or the whole job
 * rounded up to 64 and f_group 0 or the default for the job's K and
 * precision; otherwise the first corr_batch_process fails with CORR_EINVAL.
 * Before the first corr_batch_process only. */
int corr_batch_set_tiles(corr_handle b, int job, const corr_tiles *t);
/* mode: CORR_BATCH_BRANCHES or CORR_BATCH_PERSISTENT.  Before the first
 * corr_batch_process only (CORR_ESTATE after), CORR_EINVAL for another
 * value.  Both modes give the same results as the single-job path. */
int corr_batch_set_mode(corr_handle b, int mode);
/* packed_per_job: HOST array of n_jobs DEVICE pointers, job j's frames as in
 * corr_process.  Enqueues one graph launch on `stream`.  */
int corr_batch_process(corr_handle b, const void *const *packed_per_job, void *stream);
int corr_batch_read_cps(corr_handle b, int job, float *out);
int corr_batch_read_cps_raw(corr_handle b, int job, double *out);
int corr_batch_read_scales(corr_handle b, int job, float *out);

/* --------------------------------------------------- no-allocation entry
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One
 * integration of n_spectra spectra, computed by the same kernels in the same
 * order as corr_create + corr_set_precision + corr_process +
 * corr_read_cps_raw, with no handle and no allocation: every buffer beyond
 * the caller's input and outputs (records, partials, the float64 integration
 * buffer, calibration sums, tickets, twiddle and region tables) lives in one
 * static device array of 256 MiB per GPU, held until the process ends.  The
 * integration runs in chunks of spectra cut to fit that array (for N = 44,
 * K = 256: 2304 spectra in FP32, 9088 in INT8), so FP32 / FP16 results
 * agree with corr_process within their tolerance and INT8 / INT16 sums are
 * identical.
 *   N, K, n_spectra, precision: as corr_create and corr_set_precision (INT8
 *       also needs n_spectra <= 65536);
 *   packed: DEVICE pointer, 16-byte aligned, frames as in corr_process;
 *   cps: DEVICE pointer, 16-byte aligned, nb*K*2 doubles, overwritten with
 *       the integration in corr_read_cps_raw's layout and units;
 *   scales: INT8 / INT16: DEVICE pointer to N*K floats, written with the
 *       integration's scales (as corr_read_scales) and read by the F-stage;
 *       ignored (may be NULL) for FP32 / FP16;
 *   stream: hipStream_t; everything is enqueued on it, nothing waits.
 * The caller owns packed, cps and scales; they must stay valid until the
 * stream passes this call.  CORR_EINVAL for a bad argument, or for a shape
 * whose buffers do not fit the array even in chunks of 64 spectra (the
 * message gives the bytes it would need; e.g. N = 256 at K = 512 needs a
 * 269 MB integration buffer).  The first call on each device looks up the
 * array and writes its twiddle tables with a synchronous copy, so it must
 * not be captured; later calls only enqueue kernels.  Every call on one GPU
 * uses that GPU's one array: calls that overlap on it (other streams,
 * other threads) race and give wrong results.  */
int corr_process_noalloc(int N, int K, int n_spectra, int precision, const void *packed, double *cps,
                         float *scales, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CORR_H */
