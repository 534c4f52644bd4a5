/*
 * daq.h -- C ABI of libdaqisland: T-method island chopping of waveform
 * digitizer fills on an AMD Instinct MI355X (gfx950).
 *
 * What is computed (Gohn, "Data Acquisition with GPUs: The DAQ for the Muon
 * g-2 Experiment at Fermilab", ICHEP 2016; Section 3, T-method paragraph,
 * and Table 2). For one calorimeter fill of C channels x N samples x[c][t]:
 *
 *   ped[c] = mean of the first min(Np, N) samples of channel c, rounded half
 *            up to an integer (Table 2, pedestal row); 0 when N = 0
 *   S[t]   = sum_c x[c][t] - sum_c ped[c]          (Table 2, waveform-sum row)
 *   F[t]   = S[t] < threshold (strict)             (Table 2, threshold row)
 *   every t with F[t] marks [t - pre, t + post] clipped to [0, N-1]
 *                                                  (Table 2, pre/post row)
 *   island = a maximal run of marked samples, so windows that overlap or
 *            touch are one island                  (Table 2, merge-check row)
 *   record = {start, stop, offset}, islands in increasing start, offset =
 *            sum of the lengths of the earlier islands
 *                                                  (Table 2, island-array row)
 *   out[c][offset + k] = x[c][start + k] for 0 <= k < stop - start: the raw
 *            (not pedestal-subtracted) samples of every channel
 *                                                  (Section 3, GPU thread:
 *                                                   chopped islands)
 *
 * All arithmetic is integer; results are exact and deterministic.
 *
 * Conventions shared by every call:
 *  - Pointers named d_* and every pointer inside daq_fill / daq_fill_out
 *    are DEVICE pointers on the context's GPU. The library never frees or
 *    keeps them past the call's completion on the stream.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call only enqueues work on it and returns; results are ready
 *    once the stream reaches that point. Counts and status are written to
 *    device memory.
 *  - A context is not thread-safe: one host thread at a time. Calls on the
 *    same context may use different streams; each stream gets its own
 *    scratch, so work on different streams may overlap.
 *  - Return value 0 = success, negative = error (daq_strerror names it).
 *    A call that returns an error enqueued nothing.
 */
#ifndef DAQ_H
#define DAQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DAQ_ABI_VERSION 1

/* ---- return codes ------------------------------------------------------- */
#define DAQ_OK 0
#define DAQ_EINVAL (-1)   /* bad argument (see each call)                     */
#define DAQ_EALIGN (-2)   /* raw base not 16-byte aligned or stride % 8 != 0  */
#define DAQ_EHIP (-3)     /* HIP runtime error; daq_last_hip_error() has it   */
#define DAQ_ENOMEM (-4)   /* device or pinned-host allocation failed          */
#define DAQ_EAGAIN (-5)   /* server: HBM budget or queue full, try later      */
#define DAQ_ERANGE (-6)   /* a size exceeds a documented limit                */
#define DAQ_EMISMATCH (-7) /* autotune: schedules disagreed (a library bug)   */

/* ---- device-written status bits (daq_counts.status) -------------------- */
#define DAQ_STATUS_CAPACITY 1   /* more islands than `capacity`: the first
                                   `capacity` records are valid, the counts
                                   hold the true totals                       */
#define DAQ_STATUS_OUT_STRIDE 2 /* total_len > out_stride: samples at packed
                                   positions >= out_stride were not written   */

/* ---- limits --------------------------------------------------------------- */
#define DAQ_MAX_SAMPLES ((int64_t)0x7FFFFFFF) /* N per fill                    */
#define DAQ_MAX_CHANNELS 65535               /* C per fill (int32 sums exact)  */
#define DAQ_MAX_WINDOW 32768                 /* pre and post, each             */

/* One calorimeter fill: C channel rows of int16 samples, channel-major. */
typedef struct daq_fill {
    const int16_t *raw;  /* device: raw[c * row_stride + t], 16-byte aligned;
                            must hold n_channels * row_stride elements       */
    int64_t n_samples;   /* N, 0 <= N <= DAQ_MAX_SAMPLES                      */
    int64_t row_stride;  /* elements between rows; multiple of 8, >= N      */
    int32_t n_channels;  /* C, 1..DAQ_MAX_CHANNELS                            */
    int32_t ped_samples; /* Np >= 1 (the paper uses 100)                      */
    int32_t threshold;   /* a sample crosses when S[t] < threshold            */
    int32_t pre;         /* samples kept before a crossing, 0..DAQ_MAX_WINDOW */
    int32_t post;        /* samples kept after a crossing, 0..DAQ_MAX_WINDOW  */
    int32_t reserved;    /* must be 0                                         */
} daq_fill;

/* One island: samples [start, stop) of the fill; their packed copies sit at
 * out[c * out_stride + offset + k], 0 <= k < stop - start. */
typedef struct daq_island {
    int64_t start;
    int64_t stop;   /* exclusive */
    int64_t offset;
} daq_island;

/* Per-fill totals, written by the device. */
typedef struct daq_counts {
    int64_t n_islands; /* true number of islands (may exceed capacity)       */
    int64_t total_len; /* sum of island lengths = packed samples per channel */
    int32_t status;    /* DAQ_STATUS_* bits                                  */
    int32_t reserved;
} daq_counts;

/* Where one fill's results go (all device pointers). */
typedef struct daq_fill_out {
    daq_island *islands; /* capacity records                                  */
    int64_t capacity;    /* >= 0; daq_max_islands() never overflows           */
    daq_counts *counts;  /* one record                                        */
    int32_t *ped;        /* n_channels pedestals, or NULL                      */
    int16_t *out;        /* n_channels rows of out_stride, or NULL: find only */
    int64_t out_stride;  /* elements per packed row; N never overflows        */
} daq_fill_out;

/* Launch schedule of the fused kernel (chosen by daq_autotune or set). */
#define DAQ_VARIANT_RELOAD 0   /* rows read into registers, read again for the
                                  write-out                                   */
#define DAQ_VARIANT_REGISTERS 1 /* 54-channel tiles kept in registers; a call
                                   with any other channel count runs
                                   DAQ_VARIANT_RELOAD instead                 */
#define DAQ_VARIANT_LDS 2      /* 54-channel tiles loaded straight into LDS,
                                  two work-groups per CU (threads = 256)      */
#define DAQ_VARIANT_RELOAD18 3 /* as RELOAD with 18 rows in flight (6 there) */
#define DAQ_VARIANT_RELOAD27 4 /* as RELOAD with 27 rows in flight          */
#define DAQ_VARIANT_SPLIT 5    /* three passes: a streaming scan that writes
                                  island-mask bits and tile totals, a prefix
                                  pass, and an emit pass that copies only the
                                  island samples (threads = 256 or 512)       */
typedef struct daq_schedule {
    int32_t threads;     /* work-group size: 128, 256 or 512                    */
    int32_t wgs_per_cu;  /* persistent grid = wgs_per_cu x CUs (1..16); 0 =
                            one work-group per tile                            */
    int32_t variant;     /* DAQ_VARIANT_*; under DAQ_VARIANT_LDS, fills it
                            cannot take (other channel counts, halos wider
                            than a quarter of its tile) use the re-read path
                            inside the same launch                             */
    int32_t reserved;
} daq_schedule;

typedef struct daq_ctx daq_ctx;

/* Library identification. */
const char *daq_version(void);
/* Message for a DAQ_* return code. Never NULL. */
const char *daq_strerror(int code);
/* Last HIP error code seen by this thread (0 if none). */
int daq_last_hip_error(void);

/* Upper bound on the island count of an N-sample fill: flagged samples of
 * different islands are at least pre + post + 2 apart, so
 * n <= floor((N - 1) / (pre + post + 2)) + 1 (0 for N <= 0; -1 for bad
 * arguments). Capacity of this size never overflows. */
int64_t daq_max_islands(int64_t n_samples, int32_t pre, int32_t post);

/* Create a context on HIP device `device` (allocates nothing large; scratch
 * grows on demand). *out receives the handle. */
int daq_ctx_create(daq_ctx **out, int device);
/* Waits for the context's streams, frees its scratch and graphs. NULL ok. */
void daq_ctx_destroy(daq_ctx *ctx);

/* Pedestals, sum, threshold, dilation, merge and island array for one fill
 * (Table 2 rows 1-6). Writes capacity records at most to d_islands (in
 * increasing start), the totals to *d_counts and, when d_ped is not NULL,
 * the C pedestals. Errors: EINVAL (NULL ctx/fill/d_counts, d_islands NULL
 * with capacity > 0, sizes out of range, reserved != 0), EALIGN, ERANGE. */
int daq_find_islands(daq_ctx *ctx, const daq_fill *fill, daq_island *d_islands,
                     int64_t capacity, daq_counts *d_counts, int32_t *d_ped,
                     void *stream);

/* Chopped islands (Section 3): copies every channel's raw samples of the
 * islands found by daq_find_islands for the same fill into
 * d_out[c * out_stride + offset + k]. Reads the island count from d_counts
 * on the device and copies at most `capacity` islands; positions at or past
 * out_stride are skipped (and DAQ_STATUS_OUT_STRIDE is or-ed into
 * d_counts->status). Errors: as daq_find_islands, plus EINVAL for
 * d_out == NULL or out_stride < 0. */
int daq_gather_islands(daq_ctx *ctx, const daq_fill *fill,
                       const daq_island *d_islands, int64_t capacity,
                       daq_counts *d_counts, int16_t *d_out, int64_t out_stride,
                       void *stream);

/* Both calls in one pass over the fill: the fused kernel finds the islands
 * and writes the packed samples in the same read of the raw data. Same
 * results as daq_find_islands followed by daq_gather_islands. */
int daq_chop_fill(daq_ctx *ctx, const daq_fill *fill, const daq_fill_out *out,
                  void *stream);

/* Many independent fills (uneven N, thresholds, windows) in one persistent
 * launch of the fused kernel, replayed from a captured HIP graph when the
 * context's graphs are on. Results per fill are identical to daq_chop_fill.
 * The two arrays are host arrays of n entries; they are copied before the
 * call returns. n = 0 is a no-op. */
int daq_process_batch(daq_ctx *ctx, const daq_fill *fills,
                      const daq_fill_out *outs, int32_t n, void *stream);

/* Schedule of the fused kernel used by daq_chop_fill / daq_process_batch.
 * EINVAL for values outside the documented sets. */
int daq_ctx_set_schedule(daq_ctx *ctx, const daq_schedule *s);
int daq_ctx_get_schedule(daq_ctx *ctx, daq_schedule *s);

/* Use captured HIP graphs for daq_process_batch (default on). */
int daq_ctx_set_graphs(daq_ctx *ctx, int enable);

/* Kernel timing: when on, each fused-kernel launch is bracketed by a pair of
 * HIP events on its stream (between the two graph launches when graphs are
 * used). Off by default. Turning it on or off discards unread timings. */
int daq_ctx_set_timing(daq_ctx *ctx, int enable);
/* Waits for the last timed launch and returns its duration in ms; marks
 * every timing read. EINVAL when no unread timed launch exists. */
int daq_ctx_kernel_time(daq_ctx *ctx, float *ms);
/* Waits for and returns (oldest first) up to max unread launch durations in
 * ms; returns how many were written (the newest 16384 are kept), or a
 * negative error code. */
int daq_ctx_kernel_times(daq_ctx *ctx, float *ms, int32_t max);

/* Times every candidate schedule on the given batch, checks that each one's
 * island tables, counts and packed samples equal the first candidate's byte
 * for byte (DAQ_EMISMATCH otherwise), keeps the fastest as the context's
 * schedule and writes it to *best. Synchronises `stream`; the outputs hold
 * the last candidate's (identical) results. When cache_path is not NULL the
 * choice is looked up there first and stored there after tuning, keyed by
 * device name and batch shape. */
int daq_autotune(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs,
                 int32_t n, void *stream, const char *cache_path,
                 daq_schedule *best);

#ifdef __cplusplus
}
#endif

#endif /* DAQ_H */
