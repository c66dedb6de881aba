// Host runtime of libcorr.so: the C ABI declared in include/corr.h.
//
// One handle owns the float64 integration buffer of one correlation and the
// scratch of its F -> X -> dump sequence.  corr_process splits an
// integration into chunks of spectra; for each chunk the F-stage writes
// channel-major records, the X-stage writes per-split partial visibilities
// and the dump kernel adds them into float64.  Everything is enqueued on the
// caller's stream; nothing blocks until a read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/corr.h"
#include "corr_internal.h"

using namespace corr;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(CORR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// (cos, sin) of 2 pi q / n with exact values at multiples of pi/4 and the
// same octant reduction for both, so cos and sin agree bit for bit where they
// should.
void cos_sin_2pi(int64_t q, int64_t n, double *c, double *s) {
    q %= n;
    if (q < 0) q += n;
    const double r = std::sqrt(0.5);
    if ((q * 8) % n == 0) {
        static const double cs[8][2] = {{1, 0}, {0, 0}, {0, 1}, {0, 0}, {-1, 0}, {0, 0}, {0, -1}, {0, 0}};
        const int oct = (int)(q * 8 / n);
        if (oct % 2 == 0) {
            *c = cs[oct][0];
            *s = cs[oct][1];
        } else {
            *c = (oct == 1 || oct == 7) ? r : -r;
            *s = (oct == 1 || oct == 3) ? r : -r;
        }
        return;
    }
    const int quad = (int)(4 * q / n);
    const int64_t rem4 = 4 * q - (int64_t)quad * n;  // 4 * (q - quad n/4), in (0, n)
    const long double pi = 3.141592653589793238462643383279502884L;
    long double c0, s0;
    if (2 * rem4 < n) {  // angle below pi/4
        const long double ang = 2.0L * pi * (long double)rem4 / (4.0L * n);
        c0 = cosl(ang);
        s0 = sinl(ang);
    } else {
        const long double ang = 2.0L * pi * (long double)(n - rem4) / (4.0L * n);
        c0 = sinl(ang);
        s0 = cosl(ang);
    }
    switch (quad) {
        case 0: *c = (double)c0; *s = (double)s0; break;
        case 1: *c = (double)-s0; *s = (double)c0; break;
        case 2: *c = (double)-c0; *s = (double)-s0; break;
        default: *c = (double)s0; *s = (double)-c0; break;
    }
}

// W_n^j = exp(-2 pi i j / n) as float2
float2 twiddle(int64_t j, int64_t n) {
    double c, s;
    cos_sin_2pi(j, n, &c, &s);
    return make_float2((float)c, (float)-s);
}

// The F-stage's twiddle table for K channels: W_K^j, j < K, then W_2K^q,
// q < K/2, then K bytes of zeros (the F-stage reads its absent blocks from
// there).
size_t tw_table_len(int K) { return (size_t)K + K / 2 + K / 8; }
void fill_twiddles(float2 *tw, int K) {
    for (size_t i = 0; i < tw_table_len(K); ++i) tw[i] = make_float2(0.0f, 0.0f);
    for (int j = 0; j < K; ++j) tw[j] = twiddle(j, K);
    for (int q = 0; q < K / 2; ++q) tw[K + q] = twiddle(q, 2 * K);
}

struct Timer {
    int stage;
    hipEvent_t a, b;
};

}  // namespace

struct corr_ctx {
    // shape
    int N = 0, K = 0, S = 0, prec = kFP32;
    int a_pad = 0, nb = 0;
    int device = 0;
    bool batch = false;
    // plan
    corr_tiles tiles{0, 0, 0};
    bool planned = false, started = false;
    int TG = 2, ntq_buf = 0;
    int nblk = 0, rb = 0, n_diag = 0, n_off = 0;
    XGroup *xgroups = nullptr;  // region groups for LDS-staged int8 / fp16 (large N)
    int n_xgroups = 0;
    // device buffers
    uint4 *spec = nullptr;
    size_t spec_bytes = 0;
    void *partial = nullptr;
    double2 *acc = nullptr;
    double2 *stage = nullptr;
    float2 *tw = nullptr;
    float *scales = nullptr;
    float *power = nullptr;
    bool scales_valid = false;  // a calibration has been enqueued into `scales`
    int2 *regions = nullptr;
    unsigned long long *sat = nullptr;
    unsigned *fticket = nullptr;  // F-stage tile-chunk counters
    // a job of a branches-mode batch: its input pointer, which the kernels
    // read from this device slot when the graph replays
    const uint8_t *const *in_slot = nullptr;
    // delay and phase tracking: the model per antenna (a_pad entries of
    // delay, delay rate, phase, phase rate) on the host, copied to the device
    // table on the next processing stream when changed
    std::vector<double4> track_host;
    double4 *track = nullptr;
    bool track_on = false, track_dirty = false;
    // frame ingest: owner table and counters of the last corr_ingest, and
    // whether the next corr_process still has to take its lost spectra into
    // account
    unsigned *ingest_owner = nullptr;
    unsigned *ingest_ctr = nullptr;
    hipStream_t ingest_stream = nullptr;
    bool ingested = false, ingest_pending = false;
    // fused pipeline: requested chunk, ring and F workgroups per CU (0 =
    // default), then the plan: grid, F workgroups, splits per channel, flush
    // period, chunks, partial slots, records per ring slot; counters and the
    // sticky error flag
    int pipeline = CORR_PIPELINE_STAGED;
    int fx_chunk = 0, fx_ring = 0, fx_fpc = 0, fx_fcus = 0, fx_cus = 0;
    int fx_grid = 0, fx_nfwg = 0, fx_nsplit = 0, fx_flush = 0, fx_nchunks = 0, fx_nslots = 0;
    int64_t fx_slot_recs = 0;
    unsigned *fx_ctr = nullptr;
    size_t fx_ctr_bytes = 0;
    unsigned *fx_err = nullptr;
    const uint4 *dbg_spec = nullptr;  // records of the last chunk (fused: its ring slot)
    // state
    int64_t accumulated = 0;
    int last_chunk = 0;
    hipStream_t last_stream = nullptr;
    bool timing = false;
    double ms[5] = {0, 0, 0, 0, 0};  // calib, F, X, dump, fused F + X
    int64_t launches_f = 0, launches_x = 0, launches_fused = 0;
    std::vector<Timer> timers;
    // batch: the jobs, their device descriptors, the work list, counters
    // (ticket, error flag, then kBatchCounters per job) and the captured graph
    std::vector<corr_ctx *> jobs;
    BJob *bjobs = nullptr;
    const uint8_t **in_ptrs = nullptr;
    BItem *items = nullptr;
    unsigned *bctr = nullptr;
    int n_items = 0, n_ctr = 0, b_grid = 0, b_lds = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int bmode = CORR_BATCH_BRANCHES;
    bool bfailed = false;
    std::vector<hipStream_t> br_streams;  // branches mode: capture-time side streams
    std::vector<hipEvent_t> br_events;    // fork, then one join per branch
};

namespace {

// time tiles (2 spectra each) per workgroup of the calibration power sums
constexpr int kCalibTilesPerWG = 4;

int check_shape(int N, int K, int S) {
    if (N < 2 || N > CORR_MAX_ANTENNAS) return fail(CORR_EINVAL, "N=%d out of [2, %d]", N, CORR_MAX_ANTENNAS);
    if (!is_pow2(K) || K < CORR_MIN_CHANNELS || K > CORR_MAX_CHANNELS)
        return fail(CORR_EINVAL, "K=%d is not a power of two in [%d, %d]", K, CORR_MIN_CHANNELS,
                    CORR_MAX_CHANNELS);
    if (S < 1 || S > (1 << 24)) return fail(CORR_EINVAL, "n_spectra=%d out of [1, 2^24]", S);
    return CORR_OK;
}

void free_ctx(corr_ctx *h) {
    if (!h) return;
    if (h->last_stream) hipStreamSynchronize(h->last_stream);
    hipDeviceSynchronize();
    for (auto &t : h->timers) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    if (h->gexec) hipGraphExecDestroy(h->gexec);
    if (h->graph) hipGraphDestroy(h->graph);
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
    for (hipStream_t s : h->br_streams) hipStreamDestroy(s);
    for (hipEvent_t e : h->br_events) hipEventDestroy(e);
    void *bufs[] = {h->spec,    h->partial, h->acc,     h->stage,   h->tw,     h->scales,
                    h->power,   h->regions, h->sat,     h->fticket, h->xgroups, h->bjobs,
                    h->in_ptrs, h->items,   h->bctr,    h->track,   h->ingest_owner, h->ingest_ctr,
                    h->fx_ctr,  h->fx_err};
    for (void *p : bufs)
        if (p) hipFree(p);
    for (corr_ctx *j : h->jobs) free_ctx(j);
    delete h;
}

int default_chunk(const corr_ctx *h) {
    const int64_t per_spectrum = (int64_t)h->a_pad * h->K * (kRecordBytes / h->TG);
    // the whole integration when it fits in 8 GB of scratch: fewer, longer
    // X-stage launches beat the small cache-resident chunks measured on MI355X
    const int64_t cap_bytes = (int64_t)8 << 30;
    int64_t c = std::max<int64_t>(64, cap_bytes / per_spectrum / 64 * 64);
    c = std::min<int64_t>(c, round_up64(h->S, 64));
    return (int)c;
}


int n_regions(const corr_ctx *h) { return h->n_diag + h->n_off; }

// X-stage splits for chunks of `chunk` spectra: enough waves to fill the chip
// (about 4096), and no partial summing more spectra than its form allows
// (fp32 2048 and fp16 16384 for accuracy, int16 16384 for exact int32 digit
// sums).
int splits_for(int nregions, int K, int prec, int chunk) {
    const int64_t waves_per_split = (int64_t)nregions * K;
    int s = (int)((4096 + waves_per_split - 1) / waves_per_split);
    s = std::max(1, std::min(64, s));
    const int cap = prec == kFP32 ? kF32SplitSpectra
                  : prec == kFP16 ? kF16SplitSpectra
                  : prec == kINT16 ? kI16SplitSpectra : 0;
    if (cap) s = std::max(s, std::min(64, (chunk + cap - 1) / cap));
    return s;
}

int default_splits(const corr_ctx *h) { return splits_for(n_regions(h), h->K, h->prec, h->tiles.chunk_spectra); }

hipError_t set_regions(corr_ctx *h, int rb);

// Resolve tiles and allocate the precision-dependent scratch.
// The fused pipeline's plan: roles, splits, chunks, ring and partials.
int plan_fused(corr_ctx *h) {
    if (h->prec != kFP32 && h->prec != kFP16 && h->prec != kINT8)
        return fail(CORR_EINVAL, "the fused pipeline runs FP32, FP16 and INT8 only");
    if (h->n_diag != 1 || h->n_off != 0 || h->rb > kFxMaxRB)
        return fail(CORR_EINVAL, "the fused pipeline covers N <= %d (one region of at most %d antenna blocks), got N=%d",
                    16 * kFxMaxRB, kFxMaxRB, h->N);
    const int per_cu = fused_blocks_per_cu(h->K, h->prec, h->rb);
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device), "hipDeviceGetAttribute");
    if (per_cu < 2 || cus < 1) return fail(CORR_EINVAL, "the fused kernel keeps %d workgroups per CU resident; it needs 2", per_cu);
    // workgroup b runs on XCD b mod 8 (gfx950: 8 XCDs of 32 CUs), and each
    // XCD's F workgroups publish through that XCD's L2
    if (cus % 8) return fail(CORR_EINVAL, "the fused pipeline expects the CUs in 8 XCDs (%d CUs)", cus);
    h->fx_grid = per_cu * cus;
    h->fx_cus = cus;
    int x_waves = 0;
    if (h->fx_fcus) {
        // split layout: whole CUs per role, f_cus of each XCD's CUs run F
        if (h->fx_fcus >= cus / 8)
            return fail(CORR_EINVAL, "f_cus_per_xcd=%d out of [1, %d] (%d CUs per XCD)", h->fx_fcus, cus / 8 - 1, cus / 8);
        h->fx_nfwg = 8 * h->fx_fcus * per_cu;
        x_waves = 4 * (cus - 8 * h->fx_fcus) * per_cu;
    } else {
        const int fpc = h->fx_fpc ? h->fx_fpc : per_cu - 1;
        if (fpc < 1 || fpc >= per_cu)
            return fail(CORR_EINVAL, "f_workgroups_per_cu=%d out of [1, %d] (%d workgroups per CU)", fpc, per_cu - 1,
                        per_cu);
        h->fx_nfwg = fpc * cus;
        x_waves = 4 * (per_cu - fpc) * cus;
    }
    h->fx_nsplit = std::max(1, std::min(64, x_waves / h->K));
    if (h->K > x_waves) return fail(CORR_EINVAL, "the fused pipeline needs %d X waves for K=%d, has %d", h->K, h->K, x_waves);
    // chunks: records of a slot about 72 MB, so a ring of three stays in the
    // 256 MB Infinity Cache (N = 44 fp32: 768 spectra, measured the fastest of
    // 512, 768 and 1024)
    const int64_t per_spectrum = (int64_t)h->a_pad * h->K * (kRecordBytes / h->TG);
    int chunk = h->fx_chunk;
    if (!chunk) chunk = (int)std::max<int64_t>(64, ((int64_t)72 << 20) / per_spectrum / 64 * 64);
    chunk = (int)std::min<int64_t>(chunk, round_up64(h->S, 64));
    h->fx_nchunks = (h->S + chunk - 1) / chunk;
    h->fx_ring = std::max(1, std::min(h->fx_ring ? h->fx_ring : 3, h->fx_nchunks));
    const int ntq_slot = round_up((chunk + h->TG - 1) / h->TG, kTQB);
    h->fx_slot_recs = (int64_t)h->K * ntq_slot * h->a_pad;
    // a partial sums at most 2048 (fp32) / 16384 (fp16) spectra; int8 sums
    // are exact over the whole integration
    const int kb_chunk = (chunk + 4 * h->TG - 1) / (4 * h->TG);
    const int per_unit = (kb_chunk + h->fx_nsplit - 1) / h->fx_nsplit * 4 * h->TG;
    const int cap = h->prec == kFP32 ? kF32SplitSpectra : h->prec == kFP16 ? kF16SplitSpectra : 0;
    h->fx_flush = cap ? std::max(1, cap / per_unit) : h->fx_nchunks;
    if (cap && per_unit > cap)
        return fail(CORR_EINVAL, "chunk_spectra=%d gives %d spectra per partial in one chunk, above %d", chunk, per_unit, cap);
    const int epochs = (h->fx_nchunks + h->fx_flush - 1) / h->fx_flush;
    h->fx_nslots = epochs * h->fx_nsplit;
    h->tiles.chunk_spectra = chunk;
    h->tiles.x_splits = h->fx_nslots;
    h->tiles.f_group = fused_group(h->K, h->prec);
    h->ntq_buf = ntq_slot;
    h->spec_bytes = (size_t)h->fx_ring * h->fx_slot_recs * kRecordBytes;
    HIP_TRY(hipMalloc(&h->spec, h->spec_bytes + kSpecSlack), "hipMalloc(record ring)");
    HIP_TRY(hipMemset(h->spec, 0, h->spec_bytes + kSpecSlack), "hipMemset(record ring)");
    HIP_TRY(hipMalloc(&h->partial, (size_t)h->fx_nslots * h->K * h->nb * 8), "hipMalloc(partials)");
    h->fx_ctr_bytes = (size_t)round_up((kFxHdr + h->fx_nchunks * kFxPerChunk) * (int)sizeof(unsigned), 16);
    HIP_TRY(hipMalloc(&h->fx_ctr, h->fx_ctr_bytes), "hipMalloc(fused counters)");
    HIP_TRY(hipMalloc(&h->fx_err, 16), "hipMalloc(fused error flag)");
    HIP_TRY(hipMemset(h->fx_err, 0, 16), "hipMemset(fused error flag)");
    return CORR_OK;
}

int alloc_calibration(corr_ctx *h) {
    if (!is_quant(h->prec)) return CORR_OK;
    const int W = std::min(h->S, CORR_CALIB_SPECTRA);
    const int ntq_w = (W + 1) / 2;
    const int nparts = (ntq_w + kCalibTilesPerWG - 1) / kCalibTilesPerWG;
    HIP_TRY(hipMalloc(&h->scales, (size_t)h->N * h->K * sizeof(float)), "hipMalloc(scales)");
    HIP_TRY(hipMalloc(&h->power, (size_t)nparts * h->a_pad * h->K * sizeof(float)), "hipMalloc(power)");
    return CORR_OK;
}

int plan(corr_ctx *h) {
    if (h->planned) return CORR_OK;
    HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    h->TG = record_times(h->prec);
    if (h->pipeline == CORR_PIPELINE_FUSED) {
        int rc = plan_fused(h);
        if (!rc) rc = alloc_calibration(h);
        if (rc) return rc;
        h->planned = true;
        return CORR_OK;
    }
    if (h->tiles.chunk_spectra == 0) h->tiles.chunk_spectra = default_chunk(h);
    if (h->tiles.f_group == 0) h->tiles.f_group = fstage_default_group(h->K, h->prec);
    if (h->tiles.x_splits == 0) h->tiles.x_splits = default_splits(h);
    if (fstage_lds_bytes(h->K, h->prec, h->tiles.f_group) > 160 * 1024)
        return fail(CORR_EINVAL, "f_group=%d needs more than 160 KB of LDS at K=%d in this precision",
                    h->tiles.f_group, h->K);
    const int chunk = h->tiles.chunk_spectra;
    if (h->prec == kINT16) {
        if ((int64_t)h->tiles.x_splits * kI16SplitSpectra < chunk)
            return fail(CORR_EINVAL, "INT16 needs x_splits >= %d for chunks of %d spectra (exact int32 digit sums)",
                        (chunk + kI16SplitSpectra - 1) / kI16SplitSpectra, chunk);
        // six accumulators per block pair: regions of at most 3 blocks on the
        // diagonal and 2 off it
        if (h->rb > 3) {
            hipError_t e = set_regions(h, h->nblk % 2 == 0 ? 2 : 1);
            if (e != hipSuccess) return hip_fail(e, "regions");
        }
    }
    h->ntq_buf = round_up((chunk + h->TG - 1) / h->TG, kTQB);
    h->spec_bytes = (size_t)h->K * h->ntq_buf * h->a_pad * kRecordBytes;
    // cleared once: records of padding antennas in lines of their own are
    // never written again
    HIP_TRY(hipMalloc(&h->spec, h->spec_bytes + kSpecSlack), "hipMalloc(spectra chunk)");
    HIP_TRY(hipMemset(h->spec, 0, h->spec_bytes + kSpecSlack), "hipMemset(spectra chunk)");
    HIP_TRY(hipMalloc(&h->partial, (size_t)h->tiles.x_splits * h->K * h->nb * (h->prec == kINT16 ? 16 : 8)),
            "hipMalloc(partials)");
    int rc = alloc_calibration(h);
    if (rc) return rc;
    h->planned = true;
    return CORR_OK;
}

int check_tiles(const corr_ctx *h, const corr_tiles *t) {
    if (t->chunk_spectra < 0 || (t->chunk_spectra % 64) != 0)
        return fail(CORR_EINVAL, "chunk_spectra=%d must be a non-negative multiple of 64", t->chunk_spectra);
    if (t->x_splits < 0 || t->x_splits > 64) return fail(CORR_EINVAL, "x_splits=%d out of [0, 64]", t->x_splits);
    if (t->f_group != 0 && t->f_group != 1 && t->f_group != 2 && t->f_group != 4 && t->f_group != 8 &&
        t->f_group != 16)
        return fail(CORR_EINVAL, "f_group=%d must be 0, 1, 2, 4, 8 or 16", t->f_group);
    if (t->f_group && fstage_lds_bytes(h->K, h->prec, t->f_group) > 160 * 1024)
        return fail(CORR_EINVAL, "f_group=%d needs more than 160 KB of LDS at K=%d", t->f_group, h->K);
    return CORR_OK;
}

void timer_begin(corr_ctx *h, int stage, hipStream_t st) {
    if (!h->timing) return;
    Timer t{stage, nullptr, nullptr};
    hipEventCreate(&t.a);
    hipEventCreate(&t.b);
    hipEventRecord(t.a, st);
    h->timers.push_back(t);
}

void timer_end(corr_ctx *h, hipStream_t st) {
    if (!h->timing || h->timers.empty()) return;
    hipEventRecord(h->timers.back().b, st);
}

int timers_collect(corr_ctx *h) {
    if (h->timers.empty()) return CORR_OK;
    HIP_TRY(hipEventSynchronize(h->timers.back().b), "hipEventSynchronize");
    for (auto &t : h->timers) {
        float ms = 0.0f;
        hipEventElapsedTime(&ms, t.a, t.b);
        h->ms[t.stage] += ms;
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    h->timers.clear();
    return CORR_OK;
}

int launch_x_and_dump(corr_ctx *h, const uint4 *spec, int ntq, int nkb, hipStream_t st) {
    XArgs xa{};
    xa.spec = spec;
    xa.partial = h->partial;
    xa.N = h->N;
    xa.a_pad = h->a_pad;
    xa.K = h->K;
    xa.ntq = ntq;
    xa.nb = h->nb;
    xa.nsplit = h->tiles.x_splits;
    xa.nkb = nkb;
    timer_begin(h, 2, st);
    xa.regions = h->regions;
    xa.n_diag = h->n_diag;
    const bool half_or_byte = h->prec == kFP16 || h->prec == kINT8;
    if (h->n_xgroups && (half_or_byte || h->prec == kFP32) && h->rb == 4 && h->n_diag == 4) {
        // 16 blocks: one workgroup per channel stages them all in LDS once per
        // k-block (the three region groups would fetch every block twice;
        // fp32's own 4x4 off-diagonal regions run one wave per SIMD)
        HIP_TRY(launch_xchan(h->prec, xa, st), "X-stage launch");
    } else if (h->n_xgroups && half_or_byte) {
        // groups of regions that share blocks stage them in LDS once per
        // k-block, with the loads two k-blocks ahead
        xa.groups = h->xgroups;
        xa.ngroups = h->n_xgroups;
        HIP_TRY(launch_xgroups(h->prec, xa, st), "X-stage launch");
    } else if (h->n_off && half_or_byte) {
        // one launch over every region of a channel (diagonal ones first), so
        // the regions that share records read them from HBM once, through one
        // L2: the int8 and fp16 forms are bound by that traffic
        xa.nregions = h->n_diag + h->n_off;
        HIP_TRY(launch_xstage(h->prec, h->rb, 2, xa, st), "X-stage launch");
    } else {
        // fp32 is bound by MFMA rate, and its diagonal regions keep more waves
        // per SIMD in a launch of their own
        xa.nregions = h->n_diag;
        HIP_TRY(launch_xstage(h->prec, h->rb, 1, xa, st), "X-stage launch");
        if (h->n_off) {
            xa.regions = h->regions + h->n_diag;
            xa.nregions = h->n_off;
            HIP_TRY(launch_xstage(h->prec, h->rb, 0, xa, st), "X-stage launch");
        }
    }
    timer_end(h, st);
    h->launches_x++;
    timer_begin(h, 3, st);
    HIP_TRY(launch_dump(h->prec, h->partial, h->acc, h->tiles.x_splits, h->K, h->nb, st), "dump launch");
    timer_end(h, st);
    return CORR_OK;
}

int calibrate(corr_ctx *h, const uint8_t *in, hipStream_t st) {
    const int W = std::min(h->S, CORR_CALIB_SPECTRA);
    FArgs fa{};
    fa.in = in;
    fa.in_slot = h->in_slot;
    fa.power = h->power;
    fa.tw = h->tw;
    fa.N = h->N;
    fa.a_pad = h->a_pad;
    fa.S = W;
    fa.ntq = (W + 1) / 2;  // power-mode tiles hold 2 spectra
    const int gp = (256 / (h->K / 16)) / 2;  // antennas per power-mode tile
    fa.ngroups = (h->N + gp - 1) / gp;
    fa.tiles_per_wg = kCalibTilesPerWG;
    const int nparts = (fa.ntq + kCalibTilesPerWG - 1) / kCalibTilesPerWG;
    fa.ntiles = fa.ntq;
    timer_begin(h, 0, st);
    HIP_TRY(launch_fstage(h->K, kFP32, gp, 1, fa, fa.ngroups * nparts, st), "calibration launch");
    // after a frame ingest, the spectra of the window that arrived
    const unsigned *w_valid = h->ingest_pending ? h->ingest_ctr + 3 : nullptr;
    const float fs = h->prec == kINT16 ? kI16CodesPerRms : kI8CodesPerRms;
    HIP_TRY(launch_scales(h->power, nparts, h->N, h->a_pad, h->K, W, w_valid, fs, h->scales, st),
            "scales launch");
    h->scales_valid = true;
    timer_end(h, st);
    return CORR_OK;
}

int process_one(corr_ctx *h, const uint8_t *in, hipStream_t st) {
    if (is_quant(h->prec)) {
        if (h->accumulated)
            return fail(CORR_ESTATE, "INT8/INT16: read the previous integration before processing the next");
        int rc = calibrate(h, in, st);
        if (rc) return rc;
    }
    const int chunk = h->tiles.chunk_spectra;
    const int ga = h->tiles.f_group;
    const int ngroups = (h->N + ga - 1) / ga;
    const int64_t frame = (int64_t)h->N * h->K;
    if (h->track_on && h->track_dirty) {
        // pageable source: the copy is staged before this call returns
        HIP_TRY(hipMemcpyAsync(h->track, h->track_host.data(), h->track_host.size() * sizeof(double4),
                               hipMemcpyHostToDevice, st),
                "hipMemcpyAsync(tracking)");
        h->track_dirty = false;
    }
    if (h->pipeline == CORR_PIPELINE_FUSED) {
        if (h->track_on) return fail(CORR_EINVAL, "the fused pipeline does not apply delay / phase tracking");
        if (h->in_slot) return fail(CORR_EINVAL, "the fused pipeline does not run in batches");
        FxArgs fx{};
        fx.f.in = in;
        fx.f.spec = h->spec;
        fx.f.scales = h->scales;
        fx.f.tw = h->tw;
        fx.f.sat = h->sat;
        fx.f.N = h->N;
        fx.f.a_pad = h->a_pad;
        fx.f.ntq = h->ntq_buf;
        fx.f.ngroups = (h->N + h->tiles.f_group - 1) / h->tiles.f_group;
        fx.x.partial = h->partial;
        fx.x.N = h->N;
        fx.x.a_pad = h->a_pad;
        fx.x.K = h->K;
        fx.x.nb = h->nb;
        fx.x.nsplit = h->fx_nsplit;
        fx.ctr = h->fx_ctr;
        fx.err = h->fx_err;
        fx.S = h->S;
        fx.chunk = chunk;
        fx.nchunks = h->fx_nchunks;
        fx.ring = h->fx_ring;
        fx.slot_recs = h->fx_slot_recs;
        fx.n_fwg = h->fx_nfwg;
        fx.cus = h->fx_cus;
        fx.f_cus = h->fx_fcus;
        fx.flush_chunks = h->fx_flush;
        HIP_TRY(launch_fill_zero(h->fx_ctr, h->fx_ctr_bytes, st), "fused counter clear");
        timer_begin(h, 4, st);
        HIP_TRY(launch_fused(h->K, h->prec, h->rb, fx, h->fx_grid, st), "fused F + X launch");
        timer_end(h, st);
        h->launches_fused++;
        timer_begin(h, 3, st);
        HIP_TRY(launch_dump(h->prec, h->partial, h->acc, h->fx_nslots, h->K, h->nb, st), "dump launch");
        timer_end(h, st);
        const int last = h->fx_nchunks - 1;
        h->last_chunk = h->S - last * chunk;
        h->dbg_spec = h->spec + (int64_t)(last % h->fx_ring) * h->fx_slot_recs;
        return CORR_OK;
    }
    for (int c0 = 0; c0 < h->S; c0 += chunk) {
        const int Sc = std::min(chunk, h->S - c0);
        // whole k-blocks; int16 steps take two k-blocks
        const int ntq_used = round_up((Sc + h->TG - 1) / h->TG, h->prec == kINT16 ? 8 : 4);
        FArgs fa{};
        // through a slot, the kernel adds the chunk's offset (s_base) itself
        fa.in = h->in_slot ? nullptr : in + (int64_t)c0 * frame;
        fa.in_slot = h->in_slot;
        fa.track = h->track_on ? h->track : nullptr;
        fa.s_base = c0;
        fa.spec = h->spec;
        fa.scales = h->scales;
        fa.tw = h->tw;
        fa.sat = h->sat;
        fa.ticket = h->fticket;
        fa.N = h->N;
        fa.a_pad = h->a_pad;
        fa.S = Sc;
        fa.ntq = h->ntq_buf;
        fa.ngroups = ngroups;
        fa.ntiles = ntq_used * ngroups;
        timer_begin(h, 1, st);
        HIP_TRY(launch_fstage(h->K, h->prec, ga, 0, fa, 0, st), "F-stage launch");
        timer_end(h, st);
        h->launches_f++;
        int rc = launch_x_and_dump(h, h->spec, h->ntq_buf, ntq_used / 4, st);
        if (rc) return rc;
        h->last_chunk = Sc;
        h->dbg_spec = h->spec;
    }
    return CORR_OK;
}

int sync_and_collect(corr_ctx *h) {
    HIP_TRY(hipStreamSynchronize(h->last_stream), "hipStreamSynchronize");
    return timers_collect(h);
}

int read_raw_into(corr_ctx *h, double *out) {
    if (!out) return fail(CORR_EINVAL, "out is NULL");
    if (h->accumulated == 0) return fail(CORR_ESTATE, "nothing processed since the last read");
    hipStream_t st = h->last_stream;
    HIP_TRY(launch_finalize(h->acc, h->stage, h->K, h->nb, st), "finalize launch");
    HIP_TRY(hipMemcpyAsync(out, h->stage, (size_t)h->nb * h->K * sizeof(double2), hipMemcpyDeviceToHost, st),
            "hipMemcpyAsync(read)");
    int rc = sync_and_collect(h);
    if (rc) return rc;
    HIP_TRY(hipGetLastError(), "asynchronous error");
    h->accumulated = 0;
    if (h->fx_err) {
        unsigned err = 0;
        HIP_TRY(hipMemcpy(&err, h->fx_err, sizeof err, hipMemcpyDeviceToHost), "hipMemcpy(fused error flag)");
        if (err) {
            HIP_TRY(hipMemset(h->fx_err, 0, sizeof err), "hipMemset(fused error flag)");
            return fail(CORR_EHIP, "fused pipeline: a wait between workgroups exceeded its limit; results are invalid");
        }
    }
    return CORR_OK;
}

int descale_to_float(corr_ctx *h, const double *raw, float *out) {
    const int64_t n = (int64_t)h->nb * h->K;
    if (!is_quant(h->prec)) {
        for (int64_t i = 0; i < 2 * n; ++i) out[i] = (float)raw[i];
        return CORR_OK;
    }
    if (!h->scales_valid)
        return fail(CORR_ESTATE, "no calibration yet: these sums are in code units (read them with corr_read_cps_raw)");
    std::vector<float> sc((size_t)h->N * h->K);
    HIP_TRY(hipMemcpy(sc.data(), h->scales, sc.size() * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy(scales)");
    int64_t bl = 0;
    for (int a = 0; a < h->N; ++a)
        for (int b = a; b < h->N; ++b, ++bl)
            for (int k = 0; k < h->K; ++k) {
                const double d = (double)sc[(size_t)a * h->K + k] * (double)sc[(size_t)b * h->K + k];
                const int64_t i = (bl * h->K + k) * 2;
                out[i] = (float)(raw[i] / d);
                out[i + 1] = (float)(raw[i + 1] / d);
            }
    return CORR_OK;
}

// Tile the triangle of 16-antenna block pairs with regions of rb x rb blocks
// (region_at: the diagonal regions first, then the off-diagonal ones), and
// for 4 x 4-block regions in an even number of region rows list the region
// groups that share their blocks (group_at).
hipError_t set_regions(corr_ctx *h, int rb) {
    const int nr = h->nblk / rb;
    std::vector<int2> regs(region_count(nr));
    for (int i = 0; i < (int)regs.size(); ++i) regs[i] = region_at(i, nr, rb);
    if (h->regions) hipFree(h->regions);
    h->regions = nullptr;
    hipError_t e = hipMalloc(&h->regions, regs.size() * sizeof(int2));
    if (e != hipSuccess) return e;
    e = hipMemcpy(h->regions, regs.data(), regs.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    h->rb = rb;
    h->n_diag = nr;
    h->n_off = (int)regs.size() - nr;
    if (h->xgroups) hipFree(h->xgroups);
    h->xgroups = nullptr;
    h->n_xgroups = 0;
    if (uses_groups(rb, nr)) {
        std::vector<XGroup> gs(group_count(nr));
        for (int i = 0; i < (int)gs.size(); ++i) gs[i] = group_at(i, nr);
        if ((e = hipMalloc(&h->xgroups, gs.size() * sizeof(XGroup))) != hipSuccess) return e;
        if ((e = hipMemcpy(h->xgroups, gs.data(), gs.size() * sizeof(XGroup), hipMemcpyHostToDevice)) != hipSuccess)
            return e;
        h->n_xgroups = (int)gs.size();
    }
    return hipSuccess;
}

corr_ctx *create_ctx(int N, int K, int S) {
    if (check_shape(N, K, S)) return nullptr;
    corr_ctx *h = new (std::nothrow) corr_ctx();
    if (!h) {
        fail(CORR_ENOMEM, "host allocation failed");
        return nullptr;
    }
    h->N = N;
    h->K = K;
    h->S = S;
    h->nb = N * (N + 1) / 2;
    h->nblk = (N + 15) / 16;
    if (h->nblk <= 6) {
        h->a_pad = 16 * h->nblk;
        h->rb = h->nblk;
    } else {
        h->a_pad = round_up(N, 64);
        h->nblk = h->a_pad / 16;
        h->rb = 4;
    }
    auto bail = [&](hipError_t e, const char *what) {
        hip_fail(e, what);
        free_ctx(h);
        return (corr_ctx *)nullptr;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(e, "hipGetDevice");
    if ((e = set_regions(h, h->rb)) != hipSuccess) return bail(e, "regions");
    std::vector<float2> tw(tw_table_len(K));
    fill_twiddles(tw.data(), K);
    if ((e = hipMalloc(&h->tw, tw.size() * sizeof(float2))) != hipSuccess) return bail(e, "hipMalloc(twiddles)");
    if ((e = hipMemcpy(h->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "hipMemcpy(twiddles)");
    const size_t accb = (size_t)h->nb * K * sizeof(double2);
    if ((e = hipMalloc(&h->acc, accb)) != hipSuccess) return bail(e, "hipMalloc(integration buffer)");
    if ((e = hipMemset(h->acc, 0, accb)) != hipSuccess) return bail(e, "hipMemset(integration buffer)");
    if ((e = hipMalloc(&h->stage, accb)) != hipSuccess) return bail(e, "hipMalloc(read stage)");
    if ((e = hipMalloc(&h->sat, sizeof(unsigned long long))) != hipSuccess) return bail(e, "hipMalloc(counter)");
    if ((e = hipMemset(h->sat, 0, sizeof(unsigned long long))) != hipSuccess) return bail(e, "hipMemset(counter)");
    if ((e = hipMalloc(&h->fticket, kTicketBytes)) != hipSuccess) return bail(e, "hipMalloc(tile tickets)");
    return h;
}

corr_ctx *single(corr_handle h) { return (h && !h->batch) ? h : nullptr; }

}  // namespace

extern "C" {

const char *corr_last_error(void) { return g_err; }

corr_handle corr_create(int N, int K, int n_spectra) {
    g_err[0] = 0;
    return create_ctx(N, K, n_spectra);
}

int corr_set_precision(corr_handle hh, int mode) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    if (mode != CORR_FP32 && mode != CORR_FP16 && mode != CORR_INT8 && mode != CORR_INT16)
        return fail(CORR_EINVAL, "unknown precision %d", mode);
    if (h->started || h->planned) return fail(CORR_ESTATE, "precision is fixed once processing has started");
    if (mode == CORR_INT8 && h->S > 65536)
        return fail(CORR_EINVAL, "INT8 needs n_spectra <= 65536 (exact int32 partials), got %d", h->S);
    h->prec = mode;
    return CORR_OK;
}

int corr_set_tiles(corr_handle hh, const corr_tiles *t) {
    corr_ctx *h = single(hh);
    if (!h || !t) return fail(CORR_EINVAL, "invalid handle or tiles");
    if (h->started || h->planned) return fail(CORR_ESTATE, "tiles are fixed once processing has started");
    int rc = check_tiles(h, t);
    if (rc) return rc;
    h->tiles = *t;
    return CORR_OK;
}

int corr_get_tiles(corr_handle hh, corr_tiles *t) {
    corr_ctx *h = single(hh);
    if (!h || !t) return fail(CORR_EINVAL, "invalid handle or tiles");
    int rc = plan(h);
    if (rc) return rc;
    *t = h->tiles;
    return CORR_OK;
}

int corr_set_pipeline(corr_handle hh, int pipeline, int chunk_spectra, int ring_slots, int f_workgroups_per_cu,
                      int f_cus_per_xcd) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    if (pipeline != CORR_PIPELINE_STAGED && pipeline != CORR_PIPELINE_FUSED)
        return fail(CORR_EINVAL, "pipeline %d is neither CORR_PIPELINE_STAGED nor CORR_PIPELINE_FUSED", pipeline);
    if (chunk_spectra < 0 || chunk_spectra % 64)
        return fail(CORR_EINVAL, "chunk_spectra=%d must be a non-negative multiple of 64", chunk_spectra);
    if (ring_slots < 0 || ring_slots > 8) return fail(CORR_EINVAL, "ring_slots=%d out of [0, 8]", ring_slots);
    if (f_workgroups_per_cu < 0 || f_workgroups_per_cu > 16)
        return fail(CORR_EINVAL, "f_workgroups_per_cu=%d out of [0, 16]", f_workgroups_per_cu);
    if (f_cus_per_xcd < 0 || f_cus_per_xcd > 64)
        return fail(CORR_EINVAL, "f_cus_per_xcd=%d out of [0, 64]", f_cus_per_xcd);
    if (f_workgroups_per_cu && f_cus_per_xcd)
        return fail(CORR_EINVAL, "f_workgroups_per_cu and f_cus_per_xcd select different layouts; set one");
    if (h->started || h->planned) return fail(CORR_ESTATE, "the pipeline is fixed once processing has started");
    h->pipeline = pipeline;
    h->fx_chunk = chunk_spectra;
    h->fx_ring = ring_slots;
    h->fx_fpc = f_workgroups_per_cu;
    h->fx_fcus = f_cus_per_xcd;
    return CORR_OK;
}

int corr_process(corr_handle hh, const void *packed, void *stream) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    if (!packed || (reinterpret_cast<uintptr_t>(packed) & 15))
        return fail(CORR_EINVAL, "packed_samples must be a 16-byte aligned device pointer");
    int rc = plan(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    h->started = true;
    h->last_stream = st;
    rc = process_one(h, (const uint8_t *)packed, st);
    if (rc) return rc;
    h->ingest_pending = false;
    h->accumulated += h->S;
    return CORR_OK;
}

int corr_ingest(corr_handle hh, const void *frames, int64_t n_frames, int64_t frame_stride, uint64_t first_seq,
                void *out, void *stream) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    if (n_frames < 0 || n_frames > 0x7fffffff) return fail(CORR_EINVAL, "n_frames=%lld out of [0, 2^31)", (long long)n_frames);
    if (n_frames > 0 && (!frames || (reinterpret_cast<uintptr_t>(frames) & 15)))
        return fail(CORR_EINVAL, "frames must be a 16-byte aligned device pointer");
    const int64_t payload = (int64_t)h->N * h->K;
    if (frame_stride % 16 || frame_stride < CORR_FRAME_HEADER_BYTES + payload)
        return fail(CORR_EINVAL, "frame_stride=%lld must be a multiple of 16 and at least %lld", (long long)frame_stride,
                    (long long)(CORR_FRAME_HEADER_BYTES + payload));
    if (!out || (reinterpret_cast<uintptr_t>(out) & 15)) return fail(CORR_EINVAL, "out must be a 16-byte aligned device pointer");
    HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    if (!h->ingest_owner) {
        HIP_TRY(hipMalloc(&h->ingest_owner, (size_t)(h->S + 3) / 4 * 16), "hipMalloc(ingest owners)");
        HIP_TRY(hipMalloc(&h->ingest_ctr, kIngestCounterBytes), "hipMalloc(ingest counters)");
    }
    hipStream_t st = (hipStream_t)stream;
    const int W = std::min(h->S, CORR_CALIB_SPECTRA);
    HIP_TRY(launch_ingest((const uint8_t *)frames, n_frames, frame_stride, first_seq, h->S, h->N, h->K, W,
                          h->ingest_owner, h->ingest_ctr, (uint8_t *)out, st),
            "ingest launch");
    h->ingest_stream = st;
    h->ingested = true;
    h->ingest_pending = true;
    return CORR_OK;
}

int corr_get_ingest_stats(corr_handle hh, corr_ingest_stats *out) {
    corr_ctx *h = single(hh);
    if (!h || !out) return fail(CORR_EINVAL, "invalid handle or out");
    if (!h->ingested) return fail(CORR_ESTATE, "no corr_ingest yet");
    HIP_TRY(hipStreamSynchronize(h->ingest_stream), "hipStreamSynchronize");
    unsigned c[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(c, h->ingest_ctr, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy(ingest counters)");
    out->frames_accepted = c[0];
    out->frames_rejected = c[1];
    out->spectra_lost = c[2];
    out->frames_duplicate = (int64_t)c[0] - ((int64_t)h->S - c[2]);
    return CORR_OK;
}

int corr_set_tracking(corr_handle hh, const double *delay, const double *delay_rate, const double *phase,
                      const double *phase_rate) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    const double *src[4] = {delay, delay_rate, phase, phase_rate};
    if (!delay && !delay_rate && !phase && !phase_rate) {
        h->track_on = false;
        return CORR_OK;
    }
    for (int m = 0; m < 4; ++m)
        for (int a = 0; src[m] && a < h->N; ++a)
            if (!std::isfinite(src[m][a])) return fail(CORR_EINVAL, "tracking value %d of antenna %d is not finite", m, a);
    if (!h->track) {
        HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
        HIP_TRY(hipMalloc(&h->track, (size_t)h->a_pad * sizeof(double4)), "hipMalloc(tracking)");
    }
    h->track_host.assign(h->a_pad, double4{0, 0, 0, 0});
    for (int a = 0; a < h->N; ++a) {
        double4 &t = h->track_host[a];
        t.x = delay ? delay[a] : 0.0;
        t.y = delay_rate ? delay_rate[a] : 0.0;
        t.z = phase ? phase[a] : 0.0;
        t.w = phase_rate ? phase_rate[a] : 0.0;
    }
    h->track_on = true;
    h->track_dirty = true;
    return CORR_OK;
}

int corr_read_cps_raw(corr_handle hh, double *out) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    return read_raw_into(h, out);
}

int corr_read_cps(corr_handle hh, float *out) {
    corr_ctx *h = single(hh);
    if (!h || !out) return fail(CORR_EINVAL, "invalid handle or out");
    std::vector<double> raw((size_t)h->nb * h->K * 2);
    int rc = read_raw_into(h, raw.data());
    if (rc) return rc;
    return descale_to_float(h, raw.data(), out);
}

int corr_read_cps_async(corr_handle hh, double *dst, void *stream) {
    corr_ctx *h = single(hh);
    if (!h || !dst) return fail(CORR_EINVAL, "invalid handle or dst");
    if (h->accumulated == 0) return fail(CORR_ESTATE, "nothing processed since the last read");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_finalize(h->acc, h->stage, h->K, h->nb, st), "finalize launch");
    HIP_TRY(hipMemcpyAsync(dst, h->stage, (size_t)h->nb * h->K * sizeof(double2), hipMemcpyDefault, st),
            "hipMemcpyAsync(read)");
    h->last_stream = st;
    h->accumulated = 0;
    return CORR_OK;
}

int corr_read_scales(corr_handle hh, float *out) {
    corr_ctx *h = single(hh);
    if (!h || !out) return fail(CORR_EINVAL, "invalid handle or out");
    if (!is_quant(h->prec) || !h->scales_valid)
        return fail(CORR_ESTATE, "scales exist only for INT8 / INT16 once an integration has been calibrated");
    HIP_TRY(hipStreamSynchronize(h->last_stream), "hipStreamSynchronize");
    HIP_TRY(hipMemcpy(out, h->scales, (size_t)h->N * h->K * sizeof(float), hipMemcpyDeviceToHost),
            "hipMemcpy(scales)");
    return CORR_OK;
}

size_t corr_spectra_bytes(corr_handle hh, int n_spectra) {
    corr_ctx *h = single(hh);
    if (!h || n_spectra < 1) return 0;
    const int tg = record_times(h->prec);
    const int ntq = round_up((n_spectra + tg - 1) / tg, kTQB);
    return (size_t)h->K * ntq * h->a_pad * kRecordBytes;
}

int corr_process_spectra(corr_handle hh, const void *spectra, int n_spectra, void *stream) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    if (!spectra || (reinterpret_cast<uintptr_t>(spectra) & 15))
        return fail(CORR_EINVAL, "spectra must be a 16-byte aligned device pointer");
    if (n_spectra < 1 || n_spectra > (1 << 24)) return fail(CORR_EINVAL, "n_spectra=%d out of range", n_spectra);
    if (h->prec == kINT8 && n_spectra > 65536) return fail(CORR_EINVAL, "INT8 needs n_spectra <= 65536");
    int rc = plan(h);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    h->started = true;
    h->last_stream = st;
    // Ranges of whole time blocks, each at most x_splits times the spectra one
    // partial may sum in this form (float accuracy, exact int16 digit sums):
    // the splits were sized for chunk_spectra, and n_spectra may be longer.
    const int cap = h->prec == kFP32 ? kF32SplitSpectra
                  : h->prec == kFP16 ? kF16SplitSpectra
                  : h->prec == kINT16 ? kI16SplitSpectra : 65536;
    const int64_t tb_spectra = (int64_t)kTQB * h->TG;
    const int64_t range = std::max<int64_t>(tb_spectra, (int64_t)h->tiles.x_splits * cap / tb_spectra * tb_spectra);
    for (int64_t s0 = 0; s0 < n_spectra; s0 += range) {
        const int n = (int)std::min<int64_t>(range, n_spectra - s0);
        const int ntq = round_up((n + h->TG - 1) / h->TG, h->prec == kINT16 ? 8 : 4);
        const uint4 *base = (const uint4 *)spectra + (s0 / tb_spectra) * h->K * kTQB * h->a_pad;
        rc = launch_x_and_dump(h, base, ntq, ntq / 4, st);
        if (rc) return rc;
    }
    h->accumulated += n_spectra;
    return CORR_OK;
}

int corr_debug_read_spectra(corr_handle hh, void *out, int *n_spectra) {
    corr_ctx *h = single(hh);
    if (!h || !n_spectra) return fail(CORR_EINVAL, "invalid handle or n_spectra");
    if (!h->last_chunk) return fail(CORR_ESTATE, "no chunk has been transformed yet");
    *n_spectra = h->last_chunk;
    if (!out) return CORR_OK;
    HIP_TRY(hipStreamSynchronize(h->last_stream), "hipStreamSynchronize");
    // time blocks are outermost, so the chunk's records are a prefix
    const size_t bytes = corr_spectra_bytes(hh, h->last_chunk);
    HIP_TRY(hipMemcpy(out, h->dbg_spec ? h->dbg_spec : h->spec, bytes, hipMemcpyDeviceToHost), "hipMemcpy(spectra)");
    return CORR_OK;
}

int corr_get_stats(corr_handle hh, corr_stats *out) {
    corr_ctx *h = single(hh);
    if (!h || !out) return fail(CORR_EINVAL, "invalid handle or out");
    int rc = timers_collect(h);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->spectra_accumulated = h->accumulated;
    if (h->sat) {
        unsigned long long s = 0;
        if (h->last_stream) HIP_TRY(hipStreamSynchronize(h->last_stream), "hipStreamSynchronize");
        HIP_TRY(hipMemcpy(&s, h->sat, sizeof(s), hipMemcpyDeviceToHost), "hipMemcpy(counter)");
        out->int8_saturated = (int64_t)s;
    }
    out->precision = h->prec;
    out->chunk_spectra = h->tiles.chunk_spectra;
    out->x_splits = h->tiles.x_splits;
    out->f_group = h->tiles.f_group;
    out->ms_calib = h->ms[0];
    out->ms_f = h->ms[1];
    out->ms_x = h->ms[2];
    out->ms_dump = h->ms[3];
    out->launches_f = h->launches_f;
    out->launches_x = h->launches_x;
    out->ms_fused = h->ms[4];
    out->launches_fused = h->launches_fused;
    return CORR_OK;
}

int corr_enable_timing(corr_handle hh, int on) {
    corr_ctx *h = single(hh);
    if (!h) return fail(CORR_EINVAL, "invalid handle");
    int rc = timers_collect(h);
    if (rc) return rc;
    h->timing = on != 0;
    for (double &m : h->ms) m = 0.0;
    h->launches_f = h->launches_x = h->launches_fused = 0;
    return CORR_OK;
}

void corr_destroy(corr_handle h) { free_ctx(h); }

// ------------------------------------------------------------------- batch

corr_handle corr_batch_create(const corr_job *jobs, int n_jobs) {
    g_err[0] = 0;
    if (!jobs || n_jobs < 1 || n_jobs > 64) {
        fail(CORR_EINVAL, "n_jobs=%d out of [1, 64]", n_jobs);
        return nullptr;
    }
    corr_ctx *b = new (std::nothrow) corr_ctx();
    if (!b) {
        fail(CORR_ENOMEM, "host allocation failed");
        return nullptr;
    }
    b->batch = true;
    if (hipGetDevice(&b->device) != hipSuccess) {
        fail(CORR_EHIP, "hipGetDevice failed");
        delete b;
        return nullptr;
    }
    for (int i = 0; i < n_jobs; ++i) {
        const corr_job &jd = jobs[i];
        corr_ctx *h = create_ctx(jd.N, jd.K, jd.n_spectra);
        if (h) b->jobs.push_back(h);
        if (h && jd.precision == CORR_INT16) {
            free_ctx(b);
            fail(CORR_EINVAL, "job %d: INT16 is not available in batches", i);
            return nullptr;
        }
        if (!h || corr_set_precision(h, jd.precision) != CORR_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "job %d: %s", i, g_err);
            free_ctx(b);
            fail(CORR_EINVAL, "%s", msg);
            return nullptr;
        }
    }
    return b;
}

int corr_batch_set_tiles(corr_handle b, int job, const corr_tiles *t) {
    if (!b || !b->batch || !t) return fail(CORR_EINVAL, "invalid batch handle or tiles");
    if (job < 0 || job >= (int)b->jobs.size()) return fail(CORR_EINVAL, "job %d out of range", job);
    if (b->gexec) return fail(CORR_ESTATE, "tiles are fixed once the batch has run");
    corr_ctx *h = b->jobs[job];
    // the same checks as for a single correlator; the persistent mode's own
    // constraints (one chunk, its F group) are checked when it is built
    const int rc = check_tiles(h, t);
    if (rc) return rc;
    h->tiles = *t;
    return CORR_OK;
}

int corr_batch_set_mode(corr_handle b, int mode) {
    if (!b || !b->batch) return fail(CORR_EINVAL, "invalid batch handle");
    if (mode != CORR_BATCH_BRANCHES && mode != CORR_BATCH_PERSISTENT)
        return fail(CORR_EINVAL, "batch mode %d is neither CORR_BATCH_BRANCHES nor CORR_BATCH_PERSISTENT", mode);
    if (b->gexec) return fail(CORR_ESTATE, "the mode is fixed once the batch has run");
    b->bmode = mode;
    return CORR_OK;
}

namespace {

constexpr int kBatchBranches = 4;

// Branches mode: plan every job with its own tiles and kernels, and capture
// them into one graph whose jobs run on up to kBatchBranches parallel
// branches, in order of decreasing work (fp32 jobs on one branch of their
// own, the others dealt round-robin).  (Dealing each job to the branch with
// the least work so far measured slower: it lined the small jobs up behind
// one another on one branch instead of beside the large ones' tails.)  The
// kernels read each job's input pointer from b->in_ptrs, which
// corr_batch_process rewrites before every replay.
int batch_build_branches(corr_ctx *b) {
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    const int nj = (int)b->jobs.size();
    HIP_TRY(hipMalloc(&b->in_ptrs, nj * sizeof(uint8_t *)), "hipMalloc(batch inputs)");
    HIP_TRY(hipMemset(b->in_ptrs, 0, nj * sizeof(uint8_t *)), "hipMemset(batch inputs)");
    std::vector<double> work(nj);
    for (int j = 0; j < nj; ++j) {
        corr_ctx *h = b->jobs[j];
        // the job's own tiles, as a single correlator would run them
        int rc = plan(h);
        if (rc) return rc;
        h->in_slot = b->in_ptrs + j;
        // F-stage samples plus X-stage complex products
        work[j] = (double)h->S * h->N * h->K * (2.0 + 0.25 * h->N);
    }
    std::vector<int> order(nj);
    for (int j = 0; j < nj; ++j) order[j] = j;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    // fp32 jobs (X-stage bound by the MFMA rate, F-stage by HBM writes) slow
    // one another down side by side: the 12-job fp32 batch took 4.45 ms on
    // four branches and 4.34 ms on one.  The int8 batch took 2.30 ms on four
    // and 2.97 ms on one.  So the fp32 jobs share one branch, and the other
    // jobs are dealt round-robin over the remaining branches.
    int n_f32 = 0;
    for (corr_ctx *h : b->jobs) n_f32 += h->prec == kFP32;
    const int f32_br = n_f32 ? 1 : 0;
    const int nbr = f32_br + std::min(kBatchBranches - f32_br, nj - n_f32);
    std::vector<int> branch_of(nj);
    for (int i = 0, next = 0; i < nj; ++i) {
        const int j = order[i];
        if (b->jobs[j]->prec == kFP32) {
            branch_of[j] = 0;
        } else {
            branch_of[j] = f32_br + next;
            next = (next + 1) % (nbr - f32_br);
        }
    }
    HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    for (int i = 0; i < nbr; ++i) {
        hipStream_t s = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
        b->br_streams.push_back(s);
    }
    for (int i = 0; i <= nbr; ++i) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
        b->br_events.push_back(e);
    }
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    // enqueue under capture; the capture ends whatever happens
    auto enqueue = [&]() -> int {
        HIP_TRY(hipEventRecord(b->br_events[0], b->cap_stream), "hipEventRecord(fork)");
        for (hipStream_t s : b->br_streams) HIP_TRY(hipStreamWaitEvent(s, b->br_events[0], 0), "hipStreamWaitEvent");
        for (int i = 0; i < nj; ++i) {
            int rc = process_one(b->jobs[order[i]], nullptr, b->br_streams[branch_of[order[i]]]);
            if (rc) return rc;
        }
        for (int i = 0; i < nbr; ++i) {
            HIP_TRY(hipEventRecord(b->br_events[i + 1], b->br_streams[i]), "hipEventRecord(join)");
            HIP_TRY(hipStreamWaitEvent(b->cap_stream, b->br_events[i + 1], 0), "hipStreamWaitEvent");
        }
        return CORR_OK;
    };
    const int rc = enqueue();
    const hipError_t ec = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (rc) return rc;
    HIP_TRY(ec, "hipStreamEndCapture");
    HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return CORR_OK;
}

// Persistent mode: plan every job as one chunk, lay out the work list and
// capture the graph.
int batch_build(corr_ctx *b) {
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    const int nj = (int)b->jobs.size();
    std::vector<BJob> bj(nj);
    std::vector<BItem> power, scales;
    std::vector<std::vector<BItem>> fitems(nj), xitems(nj), dumps(nj);
    int lds = 0;
    for (int j = 0; j < nj; ++j) {
        corr_ctx *h = b->jobs[j];
        // the persistent kernel runs each job as one chunk with the F group
        // it is compiled for
        const int whole = round_up(h->S, 64), g = batch_default_group(h->K, h->prec);
        if ((h->tiles.chunk_spectra != 0 && h->tiles.chunk_spectra != whole) ||
            (h->tiles.f_group != 0 && h->tiles.f_group != g))
            return fail(CORR_EINVAL,
                        "job %d: the persistent batch kernel needs chunk_spectra 0 or %d and f_group 0 or %d", j,
                        whole, g);
        h->tiles.chunk_spectra = whole;
        h->tiles.f_group = g;
        int rc = plan(h);
        if (rc) return rc;
        // regions small enough for the batch kernel's register budget
        const int rb = h->nblk <= 3 ? h->nblk : (h->nblk % 2 == 0 ? 2 : 1);
        HIP_TRY(set_regions(h, rb), "regions");
        lds = std::max(lds, batch_lds_bytes(h->K, h->prec));
        // this job's counters, indices into the counter array the kernel is
        // given (after the ticket and the error flag): power, scales, F, X, dump
        const int c0 = j * kBatchCounters;
        const int ga = h->tiles.f_group;
        const int ngroups = (h->N + ga - 1) / ga;
        const int ntq_used = round_up((h->S + h->TG - 1) / h->TG, 4);
        BJob &d = bj[j];
        std::memset(&d, 0, sizeof d);
        d.f.spec = h->spec;
        d.f.scales = h->scales;
        d.f.tw = h->tw;
        d.f.sat = h->sat;
        d.f.N = h->N;
        d.f.a_pad = h->a_pad;
        d.f.S = h->S;
        d.f.ntq = h->ntq_buf;
        d.f.ngroups = ngroups;
        d.f.ntiles = ntq_used * ngroups;
        XArgs xa{};
        xa.spec = h->spec;
        xa.partial = h->partial;
        xa.N = h->N;
        xa.a_pad = h->a_pad;
        xa.K = h->K;
        xa.ntq = h->ntq_buf;
        xa.nb = h->nb;
        xa.nsplit = h->tiles.x_splits;
        xa.nkb = ntq_used / 4;
        d.xd = xa;
        d.xd.regions = h->regions;
        d.xd.nregions = h->n_diag;
        d.xo = xa;
        d.xo.regions = h->regions + h->n_diag;
        d.xo.nregions = h->n_off;
        d.acc = h->acc;
        d.scales = h->scales;
        d.K = h->K;
        d.prec = h->prec;
        d.rb_d = rb;
        d.rb_o = rb;
        d.n_acc = h->K * h->nb;
        d.sc_n = h->N * h->K;
        int n_scales = 0;
        if (h->prec == kINT8) {
            const int W = std::min(h->S, CORR_CALIB_SPECTRA);
            const int gp = (256 / (h->K / 16)) / 2;
            d.p.power = h->power;
            d.p.tw = h->tw;
            d.p.N = h->N;
            d.p.a_pad = h->a_pad;
            d.p.S = W;
            d.p.ntq = (W + 1) / 2;
            d.p.ngroups = (h->N + gp - 1) / gp;
            d.p.tiles_per_wg = kCalibTilesPerWG;
            d.W = W;
            d.nparts = (d.p.ntq + kCalibTilesPerWG - 1) / kCalibTilesPerWG;
            const int n_power = d.p.ngroups * d.nparts;
            for (int i = 0; i < n_power; ++i) power.push_back(BItem{BI_POWER, j, i, 0, -1, 0, c0 + 0, 0});
            for (int e = 0; e < d.sc_n; e += kBatchScaleElemsPerItem, ++n_scales)
                scales.push_back(BItem{BI_SCALES, j, e, std::min(e + kBatchScaleElemsPerItem, d.sc_n), c0 + 0,
                                       n_power, c0 + 1, 0});
        }
        // longer F items amortise each item's fixed costs (twiddles, the first
        // frames' latency, the publish) once a job has tiles to spare
        const int tpi = std::max(kBatchTilesPerItem, std::min(kBatchMaxTilesPerItem, d.f.ntiles / 1024));
        int n_f = 0;
        for (int t = 0; t < d.f.ntiles; t += tpi, ++n_f)
            fitems[j].push_back(BItem{BI_F, j, t, std::min(t + tpi, d.f.ntiles), h->prec == kINT8 ? c0 + 1 : -1,
                                   n_scales, c0 + 2, 0});
        const int wd = (h->n_diag * h->K * xa.nsplit + 3) / 4, wo = (h->n_off * h->K * xa.nsplit + 3) / 4;
        for (int x = 0; x < wd; ++x) xitems[j].push_back(BItem{BI_XD, j, x, 0, c0 + 2, n_f, c0 + 3, 0});
        for (int x = 0; x < wo; ++x) xitems[j].push_back(BItem{BI_XO, j, x, 0, c0 + 2, n_f, c0 + 3, 0});
        for (int e = 0; e < d.n_acc; e += kBatchElemsPerItem)
            dumps[j].push_back(BItem{BI_DUMP, j, e, std::min(e + kBatchElemsPerItem, d.n_acc), c0 + 3,
                                     wd + wo, c0 + 4, 0});
    }
    // calibration first, then F of job j, X of job j-1 and dumps of job j-2:
    // the MFMA-heavy X-stage of one job overlaps the F-stage of the next, and
    // a job's X items are taken only once its F items have been handed out
    std::vector<BItem> items;
    items.insert(items.end(), power.begin(), power.end());
    items.insert(items.end(), scales.begin(), scales.end());
    for (int j = 0; j < nj + 2; ++j) {
        if (j < nj) items.insert(items.end(), fitems[j].begin(), fitems[j].end());
        if (j >= 1 && j - 1 < nj) items.insert(items.end(), xitems[j - 1].begin(), xitems[j - 1].end());
        if (j >= 2) items.insert(items.end(), dumps[j - 2].begin(), dumps[j - 2].end());
    }
    b->n_items = (int)items.size();
    b->n_ctr = 2 + nj * kBatchCounters;  // ticket, error flag, then the job counters
    for (const BItem &it : items)
        if (it.wait >= nj * kBatchCounters || it.sig >= nj * kBatchCounters)
            return fail(CORR_EHIP, "batch: work item counter index out of range");
    b->b_lds = lds;
    HIP_TRY(batch_prepare(lds), "hipFuncSetAttribute(batch)");
    const int maxb = batch_max_blocks(lds);
    if (maxb < 1) return fail(CORR_EHIP, "the batch kernel does not fit on this device (LDS %d bytes)", lds);
    b->b_grid = std::min(maxb, b->n_items);
    HIP_TRY(hipMalloc(&b->bjobs, nj * sizeof(BJob)), "hipMalloc(batch jobs)");
    HIP_TRY(hipMemcpy(b->bjobs, bj.data(), nj * sizeof(BJob), hipMemcpyHostToDevice), "hipMemcpy(batch jobs)");
    HIP_TRY(hipMalloc(&b->items, items.size() * sizeof(BItem)), "hipMalloc(batch items)");
    HIP_TRY(hipMemcpy(b->items, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice),
            "hipMemcpy(batch items)");
    HIP_TRY(hipMalloc(&b->in_ptrs, nj * sizeof(uint8_t *)), "hipMalloc(batch inputs)");
    const size_t ctr_bytes = (size_t)round_up(b->n_ctr * (int)sizeof(unsigned), 16);
    HIP_TRY(hipMalloc(&b->bctr, ctr_bytes), "hipMalloc(batch counters)");
    HIP_TRY(hipMemset(b->bctr, 0, ctr_bytes), "hipMemset(batch counters)");
    // the graph: clear ticket, error flag and counters, then the persistent kernel
    HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e1 = launch_fill_zero(b->bctr, ctr_bytes, b->cap_stream);
    hipError_t e2 = launch_batch(b->bjobs, b->in_ptrs, b->items, b->n_items, b->bctr, b->bctr + 2, b->bctr + 1,
                                 b->b_grid, lds, b->cap_stream);
    HIP_TRY(hipStreamEndCapture(b->cap_stream, &b->graph), "hipStreamEndCapture");
    HIP_TRY(e1, "batch counter clear");
    HIP_TRY(e2, "batch kernel launch");
    HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return CORR_OK;
}

corr_ctx *batch_job(corr_handle b, int job) {
    if (!b || !b->batch || job < 0 || job >= (int)b->jobs.size()) return nullptr;
    return b->jobs[job];
}

int batch_check_error(corr_ctx *b) {
    if (!b->bctr) return CORR_OK;  // branches mode: no dependency waits
    unsigned err = 0;
    HIP_TRY(hipMemcpy(&err, b->bctr + 1, sizeof err, hipMemcpyDeviceToHost), "hipMemcpy(batch error)");
    if (err) return fail(CORR_EHIP, "batch: a dependency wait exceeded its limit; results are invalid");
    return CORR_OK;
}

}  // namespace

int corr_batch_process(corr_handle b, const void *const *packed, void *stream) {
    if (!b || !b->batch || !packed) return fail(CORR_EINVAL, "invalid batch handle or pointer table");
    const int nj = (int)b->jobs.size();
    for (int j = 0; j < nj; ++j) {
        if (!packed[j] || (reinterpret_cast<uintptr_t>(packed[j]) & 15))
            return fail(CORR_EINVAL, "job %d: packed samples must be a 16-byte aligned device pointer", j);
        if (b->jobs[j]->prec == kINT8 && b->jobs[j]->accumulated)
            return fail(CORR_ESTATE, "job %d (INT8): read the previous integration first", j);
    }
    if (!b->gexec) {
        if (b->bfailed) return fail(CORR_ESTATE, "this batch failed to build; destroy it");
        int rc = b->bmode == CORR_BATCH_PERSISTENT ? batch_build(b) : batch_build_branches(b);
        if (rc) {
            b->bfailed = true;
            return rc;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    // pageable source: the copy is staged before this call returns
    HIP_TRY(hipMemcpyAsync(b->in_ptrs, packed, nj * sizeof(void *), hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(batch inputs)");
    HIP_TRY(hipGraphLaunch(b->gexec, st), "hipGraphLaunch");
    b->last_stream = st;
    for (corr_ctx *h : b->jobs) {
        // both modes calibrate every requantised job in each replay
        if (is_quant(h->prec)) h->scales_valid = true;
        h->started = true;
        h->last_stream = st;
        h->accumulated += h->S;
        h->last_chunk = h->S - (h->S - 1) / h->tiles.chunk_spectra * h->tiles.chunk_spectra;
    }
    return CORR_OK;
}

int corr_batch_read_cps_raw(corr_handle b, int job, double *out) {
    corr_ctx *h = batch_job(b, job);
    if (!h) return fail(CORR_EINVAL, "invalid batch handle or job");
    int rc = read_raw_into(h, out);
    if (rc) return rc;
    return batch_check_error(b);
}

int corr_batch_read_cps(corr_handle b, int job, float *out) {
    corr_ctx *h = batch_job(b, job);
    if (!h || !out) return fail(CORR_EINVAL, "invalid batch handle, job or out");
    std::vector<double> raw((size_t)h->nb * h->K * 2);
    int rc = read_raw_into(h, raw.data());
    if (rc) return rc;
    rc = batch_check_error(b);
    if (rc) return rc;
    return descale_to_float(h, raw.data(), out);
}

int corr_batch_read_scales(corr_handle b, int job, float *out) {
    corr_ctx *h = batch_job(b, job);
    if (!h) return fail(CORR_EINVAL, "invalid batch handle or job");
    return corr_read_scales(h, out);
}

}  // extern "C"

// ------------------------------------------------- no-allocation entry point
//
// corr_process_noalloc runs one integration exactly as corr_process does
// (same kernels, same calibration, the chunk cut to fit), with every buffer
// beyond the caller's input and outputs in `scratch`, one static device array
// per GPU that the library holds until the process ends.  Layout of the
// array:
//   [0, 32 KB)       twiddle tables of every channel count, each followed by
//                    its zero page (written once per device at set-up)
//   [32 KB, 33 KB)   F-stage tile tickets (cleared by every F-stage launch)
//   [33 KB, ...)     saturation counter (only ever added to)
//   [36 KB, 44 KB)   region table, [44 KB, 48 KB) region groups (per call)
//   [64 KB, end)     per call: integration buffer, power partials (int8 /
//                    int16), X-stage partials, spectra records + slack
// Calls that overlap on one GPU share the array and race.

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr size_t kScrTicket = (size_t)32 << 10;
constexpr size_t kScrSat = kScrTicket + kTicketBytes;
constexpr size_t kScrRegions = (size_t)36 << 10;
constexpr size_t kScrGroups = (size_t)44 << 10;
constexpr size_t kScrHeader = (size_t)64 << 10;
constexpr int kScrMaxDevices = 64;
static_assert(kScrSat + 8 <= kScrRegions, "scratch header overlap");
static_assert(kScrRegions + 528 * sizeof(int2) <= kScrGroups, "region table exceeds its slot");
static_assert(kScrGroups + 10 * sizeof(XGroup) <= kScrHeader, "group table exceeds its slot");

// Offset of the twiddle table of K channels: tables for K = 128, 256, ...
// each rounded up to 256 bytes.
size_t scr_tw_offset(int K) {
    size_t off = 0;
    for (int k = CORR_MIN_CHANNELS; k < K; k *= 2) off += round_up64(tw_table_len(k) * sizeof(float2), 256);
    return off;
}

}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

std::mutex g_scr_mu;
uint8_t *g_scr[kScrMaxDevices];  // the array's device address, per device

// Once per device, with that device current: find the array's address (the
// host-side name of a device variable is no device address) and write the
// twiddle tables.  The copy is synchronous, so the first call on a device
// must not be under stream capture.
int scratch_setup(uint8_t **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kScrMaxDevices)
        return fail(CORR_EINVAL, "device %d is beyond the %d the no-allocation entry point tracks", dev,
                    kScrMaxDevices);
    std::lock_guard<std::mutex> lock(g_scr_mu);
    if (!g_scr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        static float2 tw[kScrTicket / sizeof(float2)];
        for (int K = CORR_MIN_CHANNELS; K <= CORR_MAX_CHANNELS; K *= 2)
            fill_twiddles(tw + scr_tw_offset(K) / sizeof(float2), K);
        HIP_TRY(hipMemcpy(p, tw, sizeof tw, hipMemcpyHostToDevice), "hipMemcpy(scratch twiddles)");
        g_scr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scr[dev];
    return CORR_OK;
}

// The region table and region groups of one call, built on the device.
__global__ __launch_bounds__(256) void noalloc_tables_kernel(int2 *regs, int nreg, XGroup *groups, int ngroups,
                                                            int nr, int rb) {
    for (int i = threadIdx.x; i < nreg; i += 256) regs[i] = region_at(i, nr, rb);
    for (int i = threadIdx.x; i < ngroups; i += 256) groups[i] = group_at(i, nr);
}

// Scratch bytes for chunks of `chunk` spectra (the splits and record bytes
// returned through the pointers).
size_t noalloc_need(const corr_ctx &h, int chunk, size_t fixed, int *splits, size_t *spec_bytes) {
    *splits = splits_for(n_regions(&h), h.K, h.prec, chunk);
    const int ntq = round_up((chunk + h.TG - 1) / h.TG, kTQB);
    *spec_bytes = (size_t)h.K * ntq * h.a_pad * kRecordBytes;
    const size_t part = (size_t)*splits * h.K * h.nb * (h.prec == kINT16 ? 16 : 8);
    return fixed + round_up64(part, 256) + *spec_bytes + kSpecSlack;
}

}  // namespace

extern "C" int corr_process_noalloc(int N, int K, int n_spectra, int precision, const void *packed, double *cps,
                                    float *scales, void *stream) {
    g_err[0] = 0;
    if (check_shape(N, K, n_spectra)) return CORR_EINVAL;
    if (precision != CORR_FP32 && precision != CORR_FP16 && precision != CORR_INT8 && precision != CORR_INT16)
        return fail(CORR_EINVAL, "unknown precision %d", precision);
    if (precision == CORR_INT8 && n_spectra > 65536)
        return fail(CORR_EINVAL, "INT8 needs n_spectra <= 65536 (exact int32 partials), got %d", n_spectra);
    if (!packed || (reinterpret_cast<uintptr_t>(packed) & 15))
        return fail(CORR_EINVAL, "packed_samples must be a 16-byte aligned device pointer");
    if (!cps || (reinterpret_cast<uintptr_t>(cps) & 15))
        return fail(CORR_EINVAL, "cps must be a 16-byte aligned device pointer");
    if (is_quant(precision) && (!scales || (reinterpret_cast<uintptr_t>(scales) & 3)))
        return fail(CORR_EINVAL, "INT8 / INT16 need a 4-byte aligned device pointer for the scales");
    // the shape, regions and precision as corr_create / corr_set_precision /
    // plan set them for a handle
    corr_ctx h;
    h.N = N;
    h.K = K;
    h.S = n_spectra;
    h.prec = precision;
    h.TG = record_times(precision);
    h.nb = N * (N + 1) / 2;
    h.nblk = (N + 15) / 16;
    if (h.nblk <= 6) {
        h.a_pad = 16 * h.nblk;
        h.rb = h.nblk;
    } else {
        h.a_pad = round_up(N, 64);
        h.nblk = h.a_pad / 16;
        h.rb = 4;
    }
    if (precision == kINT16 && h.rb > 3) h.rb = h.nblk % 2 == 0 ? 2 : 1;
    const int nr = h.nblk / h.rb;
    h.n_diag = nr;
    h.n_off = region_count(nr) - nr;
    h.n_xgroups = uses_groups(h.rb, nr) ? group_count(nr) : 0;
    // per-call buffers after the header: integration buffer, power partials,
    // then X-stage partials and records for the largest chunk that fits
    const size_t acc_bytes = (size_t)h.nb * K * sizeof(double2);
    size_t power_bytes = 0;
    if (is_quant(precision)) {
        const int W = std::min(n_spectra, CORR_CALIB_SPECTRA);
        const int nparts = ((W + 1) / 2 + kCalibTilesPerWG - 1) / kCalibTilesPerWG;
        power_bytes = (size_t)nparts * h.a_pad * K * sizeof(float);
    }
    const size_t off_acc = kScrHeader;
    const size_t off_power = off_acc + round_up64(acc_bytes, 256);
    const size_t fixed = off_power + round_up64(power_bytes, 256);
    int splits = 0;
    size_t spec_bytes = 0;
    const int64_t whole = round_up64(n_spectra, 64);
    const size_t need64 = noalloc_need(h, 64, fixed, &splits, &spec_bytes);
    if (need64 > kScratchBytes)
        return fail(CORR_EINVAL,
                    "N=%d K=%d precision %d needs %zu bytes of scratch even in chunks of 64 spectra; "
                    "the no-allocation entry point has %zu", N, K, precision, need64, kScratchBytes);
    int64_t lo = 1, hi = whole / 64;  // chunks of 64 lo spectra fit
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (noalloc_need(h, (int)(mid * 64), fixed, &splits, &spec_bytes) <= kScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int chunk = (int)(lo * 64);
    noalloc_need(h, chunk, fixed, &splits, &spec_bytes);
    const size_t off_part = fixed;
    const size_t off_spec = off_part + round_up64((size_t)splits * K * h.nb * (precision == kINT16 ? 16 : 8), 256);

    uint8_t *base = nullptr;
    int rc = scratch_setup(&base);
    if (rc) return rc;
    h.device = 0;
    h.tw = reinterpret_cast<float2 *>(base + scr_tw_offset(K));
    h.fticket = reinterpret_cast<unsigned *>(base + kScrTicket);
    h.sat = reinterpret_cast<unsigned long long *>(base + kScrSat);
    h.regions = reinterpret_cast<int2 *>(base + kScrRegions);
    h.xgroups = h.n_xgroups ? reinterpret_cast<XGroup *>(base + kScrGroups) : nullptr;
    h.acc = reinterpret_cast<double2 *>(base + off_acc);
    h.power = power_bytes ? reinterpret_cast<float *>(base + off_power) : nullptr;
    h.scales = is_quant(precision) ? scales : nullptr;
    h.partial = base + off_part;
    h.spec = reinterpret_cast<uint4 *>(base + off_spec);
    h.tiles.chunk_spectra = chunk;
    h.tiles.x_splits = splits;
    h.tiles.f_group = fstage_default_group(K, precision);
    h.ntq_buf = round_up((chunk + h.TG - 1) / h.TG, kTQB);
    h.spec_bytes = spec_bytes;
    h.planned = h.started = true;
    hipStream_t st = (hipStream_t)stream;
    // Whatever the last call left: the tables of this shape, a cleared
    // integration buffer, and records cleared so that padding antennas and
    // padding spectra read as zeros.
    hipLaunchKernelGGL(noalloc_tables_kernel, dim3(1), dim3(256), 0, st, h.regions, region_count(nr), h.xgroups,
                       h.n_xgroups, nr, h.rb);
    HIP_TRY(hipGetLastError(), "region table launch");
    HIP_TRY(launch_fill_zero(h.acc, acc_bytes, st), "integration buffer clear");
    HIP_TRY(launch_fill_zero(h.spec, spec_bytes, st), "records clear");
    rc = process_one(&h, static_cast<const uint8_t *>(packed), st);
    if (rc) return rc;
    HIP_TRY(launch_finalize(h.acc, reinterpret_cast<double2 *>(cps), K, h.nb, st), "finalize launch");
    return CORR_OK;
}
