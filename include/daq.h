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
#define DAQ_ETIMEDOUT (-8) /* server: a batch outlived the batch time-out     */

/* ---- device-written status bits (daq_counts.status) -------------------- */
#define DAQ_STATUS_CAPACITY 1   /* more islands than `capacity`: the first
                                   `capacity` records are valid, the counts
                                   hold the true totals                       */
#define DAQ_STATUS_OUT_STRIDE 2 /* total_len > out_stride: samples at packed
                                   positions >= out_stride were not written   */
#define DAQ_STATUS_INCOMPLETE 4 /* DAQ_VARIANT_PIPE: a work-group gave up
                                   waiting for other work-groups (a launch
                                   that never drained); the fill's packed rows
                                   are incomplete                             */

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

/* Launch schedule of the chop (chosen by daq_autotune or set). */
#define DAQ_VARIANT_RELOAD 0   /* rows read into registers, read again for the
                                  write-out                                   */
#define DAQ_VARIANT_REGISTERS 1 /* 54-channel tiles kept in registers; a call
                                   with any other channel count runs
                                   DAQ_VARIANT_RELOAD instead                 */
#define DAQ_VARIANT_LDS 2      /* 54-channel tiles loaded straight into LDS,
                                  two work-groups per CU (threads = 256)      */
#define DAQ_VARIANT_RELOAD18 3 /* as RELOAD with 18 rows in flight (6 there) */
#define DAQ_VARIANT_RELOAD27 4 /* as RELOAD with 27 rows in flight          */
#define DAQ_VARIANT_SPLIT 5    /* a streaming scan that writes island-mask
                                  bits and tile totals, an edge pass
                                  (prefixes, records, run table, counts) and
                                  a copy pass that copies only the island
                                  samples (threads = 256 or 512)             */
#define DAQ_VARIANT_PIPE 6     /* one persistent kernel: work-groups take scan
                                  tiles (each finds its islands and prefix at
                                  once) and copy chunks of fills whose tiles
                                  are all done, so a fill's copy overlaps the
                                  scan of later fills (threads = 256 or 512) */
typedef struct daq_schedule {
    int32_t threads;     /* work-group size: 128, 256 or 512                    */
    int32_t wgs_per_cu;  /* persistent grid = wgs_per_cu x CUs (1..16); 0 =
                            one work-group per tile                            */
    int32_t variant;     /* DAQ_VARIANT_*; under DAQ_VARIANT_LDS, fills it
                            cannot take (other channel counts, halos wider
                            than a quarter of its tile) use the re-read path
                            inside the same launch                             */
    int32_t parts;       /* DAQ_VARIANT_SPLIT only: a batch is cut into this
                            many groups of fills (0 or 1: one group, at most
                            4), each on its own HIP stream, group k's scan
                            starting after group k-1's so that it overlaps
                            group k-1's copy; 0 for the other variants       */
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
 * grows on demand). *out receives the handle.
 *
 * Two environment variables, read by the library itself:
 *   DAQ_SCHEDULE="threads,wgs_per_cu,variant,parts[,graphs]" gives every new
 *     context that schedule (and, with the fifth field 0 or 1, the graph mode
 *     of daq_ctx_set_graphs); daq_autotune then returns it without tuning.
 *     daq_ctx_set_schedule still changes it. A value that does not parse or
 *     that daq_ctx_set_schedule refuses makes daq_ctx_create fail with
 *     DAQ_EINVAL and print the reason on stderr.
 *   DAQ_LOG=0|1|2 (read once per process; unset is 0) prints diagnostic lines
 *     starting "[daq] " on stderr: 1, failures (failed HIP calls named,
 *     batches the server's watchdog gave up on or that failed); 2, also
 *     context creation, every schedule the tuner timed and the one it kept,
 *     graph captures, scratch growth, server creation and shutdown with its
 *     counters, and the start of each deadtime period. */
int daq_ctx_create(daq_ctx **out, int device);
/* Waits for the context's streams, frees its scratch and graphs. NULL ok. */
void daq_ctx_destroy(daq_ctx *ctx);
/* HIP device of the context. */
int daq_ctx_get_device(daq_ctx *ctx, int *device);

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

/* Both calls at once, with the context's schedule: by default the split
 * schedule's scan, edge and copy passes; the fused schedules find the
 * islands and write the packed samples in the same read of the raw data.
 * Same results as daq_find_islands followed by daq_gather_islands. */
int daq_chop_fill(daq_ctx *ctx, const daq_fill *fill, const daq_fill_out *out,
                  void *stream);

/* Many independent fills (uneven N, thresholds, windows) in one launch of
 * the context's schedule (by default the split schedule's three kernels over
 * every fill, with persistent grids), replayed from a captured HIP graph when
 * the context's graphs are on and launched plainly otherwise. Results per
 * fill are identical to daq_chop_fill whatever the schedule. The paper
 * chops each fill as it arrives (Section 3, fills in bursts at 12 Hz);
 * taking several in one launch is this library's addition, for throughput.
 * The two arrays are host arrays of n entries; they are copied before the
 * call returns. n = 0 is a no-op. Errors: EINVAL (NULL ctx, n < 0, NULL
 * arrays with n > 0, or any fill or output that daq_chop_fill would refuse),
 * EALIGN, ERANGE, all checked for every fill before anything is launched;
 * ENOMEM or EHIP when scratch cannot grow or a launch fails. */
int daq_process_batch(daq_ctx *ctx, const daq_fill *fills,
                      const daq_fill_out *outs, int32_t n, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as daq_process_batch, computed with the split schedule (the
 * context's thread count and persistent grid when it holds a split schedule,
 * else 512 threads and 8 work-groups per CU) by plain kernel launches only:
 * no allocation, no graph, no event, no memset and no host staging. Every
 * scratch buffer of the call (look-back words, tile totals,
 * effective thresholds, the descriptor table, each fill's mask bits, run
 * table and chunk map) lives in one static device array of
 * DAQ_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from the first
 * daq_ctx_create on that GPU until the process ends; the descriptors reach it
 * through kernel arguments. Calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other contexts or threads) race
 * and must be serialised by the caller; each call clears what it needs.
 * Needs daq_noalloc_scratch_bytes(fills, n) <= DAQ_NOALLOC_SCRATCH_BYTES
 * (DAQ_ERANGE otherwise, before anything is launched; 16 fills of
 * 54 x 560,000 need about 3.5 MB). Other errors as for daq_process_batch;
 * the context's timing, graph and fill-group settings do not apply. */
#define DAQ_NOALLOC_SCRATCH_BYTES ((int64_t)32 << 20)
int64_t daq_noalloc_scratch_bytes(const daq_fill *fills, int32_t n);
int daq_process_batch_noalloc(daq_ctx *ctx, const daq_fill *fills,
                              const daq_fill_out *outs, int32_t n,
                              void *stream);

/* ---- Q-method -------------------------------------------------------------
 * The second output stream of the GPU (Section 3, Q-method paragraph; Table 2,
 * the decimation and fill-by-fill rows): instead of chopping, the detector
 * current is integrated. With S[t] the pedestal-subtracted calorimeter sum of
 * the T-method (pedestals as there: the mean of the first min(Np, N) samples
 * of each channel, rounded half up):
 *   qsum[b]  = sum of S[t] over t in [32 b, 32 b + 32), t < N  (the decimated
 *              sum: 17.5k bins for 560k samples);
 *   acc[c][t] += x[c][t] - ped[c] for every channel and t < N (the
 *              fill-by-fill sum of waveforms), int32, modulo 2^32 (exact
 *              while fewer than 32768 fills of any int16 data, or 524288
 *              fills of 12-bit data, have been added).
 * threshold, pre and post of the fill are not used. */
#define DAQ_Q_DECIMATION 32  /* samples per decimated bin                     */

typedef struct daq_q_out {
    int64_t *qsum;       /* ceil(n_samples / 32) bins, or NULL; 8-byte aligned */
    int32_t *acc;        /* n_channels rows of acc_stride int32, or NULL;
                            16-byte aligned; elements >= n_samples of a row
                            are not touched                                  */
    int64_t acc_stride;  /* elements per accumulator row: >= n_samples and a
                            multiple of 4 when acc is set                     */
    int32_t *ped;        /* n_channels pedestals written, or NULL             */
} daq_q_out;             /* 32 bytes, device pointers                          */

/* The Q-method for n fills in one launch (a pedestal kernel, then one pass
 * that reads every raw sample once and updates qsum and acc). The arrays are
 * host arrays of n entries, copied before the call returns; n = 0 is a
 * no-op. Fills of one call must not share accumulator memory (DAQ_EINVAL):
 * calls on one stream accumulate in order. Errors as for daq_process_batch,
 * and DAQ_EALIGN for misaligned qsum or acc. */
int daq_qmethod_batch(daq_ctx *ctx, const daq_fill *fills,
                      const daq_q_out *outs, int32_t n, void *stream);

/* Both methods on one read (Section 3 and Table 2 run the T-method and the
 * Q-method on every fill): daq_process_batch's T-method results in outs and
 * the Q-method's in qouts (as daq_qmethod_batch computes them), the sums and
 * accumulator updates taken inside the chop's scan pass, so the raw samples
 * are read once for both. Runs the split schedule whatever the context's
 * (plain launches, no graph). The pedestals go to outs[i].ped or, when that
 * is NULL, to qouts[i].ped (DAQ_EINVAL if both are set). Errors as for both
 * calls. */
int daq_process_batch_q(daq_ctx *ctx, const daq_fill *fills,
                        const daq_fill_out *outs, const daq_q_out *qouts,
                        int32_t n, void *stream);

/* ---- 12-bit ingest ---------------------------------------------------------
 * The digitizers deliver 12-bit samples (Section 3); the frontend unpacks them
 * before a fill is copied to the GPU. Here the packed words can be copied
 * instead (a quarter fewer bytes over PCIe) and unpacked on the device. A
 * channel row of N samples is packed two samples to three bytes,
 * little-endian: for a = x[2k], b = x[2k + 1], byte 3k = a & 0xFF, byte
 * 3k + 1 = (a >> 8) | (b & 0xF) << 4, byte 3k + 2 = b >> 4; an odd last sample
 * has no third byte. Row c starts at d_packed + c * packed_stride (bytes,
 * packed_stride >= ceil(3 N / 2), a multiple of 4; d_packed 4-byte aligned).
 * Samples t < N of row c are written to d_raw[c * row_stride + t] as int16
 * 0 .. 4095 (d_raw 16-byte aligned, row_stride >= N and a multiple of 8);
 * elements >= N are not touched. Asynchronous on `stream`. */
int daq_unpack12(daq_ctx *ctx, const uint8_t *d_packed, int64_t packed_stride,
                 int32_t n_channels, int64_t n_samples, int16_t *d_raw,
                 int64_t row_stride, void *stream);

/* ---- Island compression --------------------------------------------------
 * Section 3: the frontend compresses the chopped data without loss before it
 * goes to the event builder (the paper does not name the code). This one is
 * a per-block delta code. Each of a fill's n_channels packed rows holds L
 * samples, L = min(max(total_len, 0), max_len) with total_len read from the
 * fill's daq_counts on the device, so a call can follow daq_chop_fill or
 * daq_process_batch on the same stream. A row is cut into blocks of 64
 * samples (the last one may be short); block b = c * nb + k, nb = ceil(L /
 * 64), covers samples 64 k .. of row c. For a block of n samples x[0..n):
 *   z[i] = zigzag(x[i] - x[i - 1]) = (r << 1) ^ (r >> 31) on the int32
 *          difference r, for 1 <= i < n (0 <= z < 2^17);
 *   w    = bit length of max z (0 when n = 1 or all z are 0), at most 17;
 *   hdr[b] = (uint16_t)x[0] | w << 16;
 *   payload: ceil((n - 1) w / 32) uint32 words; z[i] occupies bits
 *          (i - 1) w .. (i - 1) w + w - 1 of it, bit j of the payload being
 *          bit j % 32 of its word j / 32 (a little-endian bit stream).
 * The payloads follow each other in block order: block b's starts at word
 * offsets[b], and *n_words is the stream's length in words (the caller reads
 * nb back from total_len). Decoding needs only hdr and words. */
#define DAQ_Z_BLOCK 64       /* samples per compressed block                */
#define DAQ_Z_MAX_WIDTH 17   /* widest difference code, bits                 */

typedef struct daq_z_fill {
    const int16_t *packed;     /* n_channels rows of stride int16 (16-byte
                                  aligned; a daq_fill_out.out)                */
    int64_t stride;            /* elements per row: >= max_len, % 8 == 0     */
    const daq_counts *counts;  /* the fill's counts (8-byte aligned)          */
    int64_t max_len;           /* samples a row holds at most, >= 0           */
    uint32_t *hdr;             /* n_channels * ceil(max_len / 64) words       */
    int64_t *offsets;          /* as many int64, or NULL                     */
    uint32_t *words;           /* words_cap words                            */
    int64_t words_cap;         /* words past it are not written; the stream
                                  never needs more than 34 per block         */
    int64_t *n_words;          /* one int64: the stream's words (may exceed
                                  words_cap: then the stream is cut short)   */
    int32_t n_channels;
    int32_t reserved;          /* 0                                          */
} daq_z_fill;                  /* 80 bytes, device pointers                   */

/* Compress n fills (host array, copied before the call returns; n = 0 is a
 * no-op), asynchronously on `stream`: a size pass and a pack pass over up to
 * 16 fills at a time. The context keeps per-stream scratch of 8 bytes per
 * wave of a launch (at most 128 KB), allocated (synchronously) on first
 * need. DAQ_EINVAL for a null pointer, a negative size, stride < max_len or
 * reserved != 0;
 * DAQ_ERANGE past DAQ_MAX_CHANNELS / DAQ_MAX_SAMPLES; DAQ_EALIGN for packed
 * or stride as stated above, or another pointer not aligned to its type.
 * Fills of one call must not share outputs. */
int daq_compress_batch(daq_ctx *ctx, const daq_z_fill *fills, int32_t n,
                       void *stream);

/* One compressed stream to decode (the inverse of daq_compress_batch, for a
 * reader of the stream: the event builder's side). */
typedef struct daq_z_stream {
    const uint32_t *hdr;      /* n_channels * ceil(n_samples / 64) headers   */
    const int64_t *offsets;   /* as many payload word offsets (required)     */
    const uint32_t *words;    /* the payload                                 */
    int64_t n_words;          /* words readable at `words`                   */
    int16_t *out;             /* n_channels rows of out_stride int16 (16-byte
                                 aligned): samples t < n_samples are written */
    int64_t out_stride;       /* >= n_samples, % 8 == 0                       */
    int64_t n_samples;        /* L of the stream (its fill's total_len)       */
    int32_t n_channels;
    int32_t reserved;         /* 0                                           */
} daq_z_stream;               /* 64 bytes, device pointers                   */

/* Decode n streams (host array, copied; n = 0 is a no-op), asynchronously on
 * `stream`, up to 16 per launch. A stream written by daq_compress_batch
 * decodes to exactly the packed rows it was made from. For any other input
 * the samples are unspecified, but no word at or past n_words is read and
 * widths above 17 are taken as 17. Errors as for daq_compress_batch
 * (DAQ_EALIGN for out or out_stride, or an array not aligned to its type). */
int daq_decompress_batch(daq_ctx *ctx, const daq_z_stream *streams, int32_t n,
                         void *stream);

/* Schedule of the chop used by daq_chop_fill / daq_process_batch
 * (a new context holds the split variant, 512 threads, 8 work-groups per
 * CU). EINVAL for values outside the documented sets. */
int daq_ctx_set_schedule(daq_ctx *ctx, const daq_schedule *s);
int daq_ctx_get_schedule(daq_ctx *ctx, daq_schedule *s);

/* Use captured HIP graphs for daq_process_batch (default on; daq_autotune
 * may switch it). daq_ctx_get_graphs writes the current mode (0 or 1). */
int daq_ctx_set_graphs(daq_ctx *ctx, int enable);
int daq_ctx_get_graphs(daq_ctx *ctx, int *enable);

/* Kernel timing: when on, each chop launch of daq_process_batch (and of the
 * single-fill calls) is bracketed by a pair of HIP events on its stream;
 * where a schedule computes the pedestals in a kernel of its own
 * (k_prepare), that kernel runs before the first event. Each event pair adds
 * a few microseconds to the launch. Off by default. Turning it on or off
 * discards unread timings. */
int daq_ctx_set_timing(daq_ctx *ctx, int enable);
/* Waits for the last timed launch and returns its duration in ms; marks
 * every timing read. EINVAL when no unread timed launch exists. */
int daq_ctx_kernel_time(daq_ctx *ctx, float *ms);
/* Waits for and returns (oldest first) up to max unread launch durations in
 * ms; returns how many were written (the newest 16384 are kept), or a
 * negative error code. */
int daq_ctx_kernel_times(daq_ctx *ctx, float *ms, int32_t max);

/* Times every candidate schedule on the given batch, checks that each one's
 * results equal the first candidate's byte for byte (DAQ_EMISMATCH
 * otherwise), keeps the fastest as the context's schedule and writes it to
 * *best. Before its checked run every candidate's output buffers are filled
 * with a poison pattern (records and counts all ones, pedestals and packed
 * rows 0x5A bytes), so a candidate that leaves an output unwritten fails the
 * check; the check compares the counts, the records below min(n_islands,
 * capacity), the pedestals and every packed row below min(total_len,
 * out_stride) with a copy of the first candidate's outputs (the library's
 * default split schedule). The menu holds the split, re-read, register and
 * LDS variants; DAQ_VARIANT_PIPE is chosen only by daq_ctx_set_schedule.
 * The winning schedule is then timed replayed from its captured graph and as
 * plain kernel launches, and the context's graph mode (daq_ctx_set_graphs)
 * is set to the faster one. Allocates a device copy of the outputs for the
 * duration of the call. Synchronises `stream`; the outputs hold the last
 * candidate's (identical) results. When cache_path is not NULL the choice
 * (schedule and graph mode) is looked up there first and stored there after
 * tuning, keyed by device name and batch shape. A context whose schedule
 * came from DAQ_SCHEDULE (daq_ctx_create) is not tuned: *best receives that
 * schedule and DAQ_OK is returned. In both of these cases (a cached choice,
 * a schedule from the environment) nothing is launched and the outputs are
 * left as they were. */
int daq_autotune(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs,
                 int32_t n, void *stream, const char *cache_path,
                 daq_schedule *best);

/* ---- serving loop ----------------------------------------------------------
 * Fills arrive in bursts, eight fills 10 ms apart (Section 3), and records
 * must be deadtime-free (abstract): a fill has to be taken while earlier
 * ones are still being processed. A
 * server admits each submitted fill only if its results fit in the device
 * arena it was given (the HBM budget) and keeps them resident there until
 * the caller releases them. Worker threads, one per HIP stream, take every
 * admitted fill not yet running (up to max_batch, oldest first) and launch
 * them as one batch (daq_process_batch); fills that arrive while a batch
 * runs go out with the next free worker on its own stream, so batches
 * overlap on the device. Each fill's results are the same as those of
 * daq_chop_fill on that fill alone.
 *
 * Slot of one fill in the arena, in this order, each part aligned to 256
 * bytes: counts (one daq_counts), ped (C int32), islands (capacity =
 * daq_max_islands(N, pre, post) records), out (C rows of out_stride = N
 * rounded up to a multiple of 8), for DAQ_SUBMIT_HOST_RAW the raw rows
 * (C x row_stride int16), and for DAQ_SUBMIT_HOST_PACKED12 the raw rows and
 * the packed words (C x daq_packed12_stride(N) bytes).
 *
 * daq_submit_fill, daq_poll, daq_release and daq_server_get_stats may be
 * called from any host thread. */
typedef struct daq_server daq_server;

#define DAQ_SUBMIT_HOST_RAW 1 /* fill->raw is host memory (pinned for speed):
                                 the server copies it into the fill's slot on
                                 the worker's stream before the launch; the
                                 host buffer may be reused once the fill's
                                 completion is returned by daq_poll          */
#define DAQ_SUBMIT_HOST_PACKED12 2 /* fill->raw is host memory holding the
                                 fill's rows as 12-bit words (the packing of
                                 daq_unpack12), row c at byte
                                 c * daq_packed12_stride(n_samples); the
                                 server copies the words into the slot and
                                 unpacks them on the device before the launch
                                 (a quarter fewer bytes over PCIe); the host
                                 buffer may be reused once the completion is
                                 returned. Not combined with HOST_RAW         */

/* Bytes per channel row of a DAQ_SUBMIT_HOST_PACKED12 fill:
 * ceil(3 n_samples / 2) rounded up to a multiple of 4. */
int64_t daq_packed12_stride(int64_t n_samples);

/* One finished fill, as returned by daq_poll. */
typedef struct daq_completion {
    uint64_t tag;        /* as given to daq_submit_fill                       */
    uint64_t ticket;     /* as returned by daq_submit_fill                    */
    daq_counts counts;   /* host copy of the fill's device counts            */
    daq_fill_out out;    /* device pointers into the arena, valid until
                            daq_release(ticket)                               */
    const int16_t *raw;  /* device raw rows the fill was chopped from        */
    int32_t status;      /* DAQ_OK, the error of the batch launch, or
                            DAQ_ETIMEDOUT (counts are then zero and the slot
                            is held until the device has finished with it)   */
    int32_t batch_fills; /* fills in the launch that carried this one        */
    int64_t t_submit_ns; /* steady clock (ns): the fill's arrival (the time
                            given to daq_submit_fill_at, else its admission)  */
    int64_t t_launch_ns; /* its batch handed to the device                    */
    int64_t t_ready_ns;  /* results complete in device memory                 */
} daq_completion;

typedef struct daq_server_stats {
    uint64_t submitted;   /* fills admitted                                  */
    uint64_t rejected;    /* submits refused with DAQ_EAGAIN                 */
    uint64_t completed;   /* fills whose results are ready                   */
    uint64_t released;    /* slots returned by daq_release                   */
    uint64_t batches;     /* launches                                        */
    uint64_t arena_bytes; /* usable budget                                   */
    uint64_t arena_in_use;
    uint64_t arena_peak;
    int32_t pending;      /* admitted, not yet launched                      */
    int32_t running;      /* launched, not yet complete                      */
    /* deadtime accounting (the abstract asks for deadtime-free records):   */
    uint64_t late;        /* fills admitted later than the admission deadline
                             after their arrival                              */
    uint64_t timed_out;   /* fills whose batch outlived the batch time-out   */
    uint64_t deadtime_ns; /* total time during which the server refused
                             fills: from a refused submit to the next
                             admission                                        */
    uint64_t admit_wait_max_ns; /* longest arrival-to-admission wait         */
} daq_server_stats;

/* Bytes of arena one fill takes (its slot, above). EINVAL as
 * daq_find_islands for a bad fill, or a NULL `bytes`; host-only. */
int daq_server_slot_bytes(const daq_fill *fill, int32_t flags, uint64_t *bytes);

/* Starts a server on ctx's device with ctx's current schedule and graph mode
 * (each worker has a context of its own with both; ctx is not used
 * afterwards). d_arena: caller-owned device memory of arena_bytes,
 * 256-byte aligned, that the server sub-allocates (never frees).
 * n_streams: 1..8 workers; max_batch: 1..256 fills per launch. */
int daq_server_create(daq_server **out, daq_ctx *ctx, void *d_arena,
                      size_t arena_bytes, int32_t n_streams, int32_t max_batch);

/* Admits one fill: reserves its slot and queues it; *ticket (not NULL)
 * receives its number (increasing from 1). fill->raw must stay valid and
 * unchanged until the fill's completion is returned. DAQ_EAGAIN when the
 * slot does not fit in the free arena now (retry after releasing),
 * DAQ_ERANGE when it can never fit, EINVAL/EALIGN as daq_find_islands
 * (a host raw needs no alignment). */
int daq_submit_fill(daq_server *srv, const daq_fill *fill, int32_t flags,
                    uint64_t tag, uint64_t *ticket);

/* daq_submit_fill for a fill that arrived at t_arrive_ns on the steady clock
 * (CLOCK_MONOTONIC, ns; 0 = now): a caller that retries after DAQ_EAGAIN
 * passes the first attempt's time, so the admission wait, the deadline check
 * and the completion's t_submit_ns run from the arrival. A time in the
 * future is taken as now. */
int daq_submit_fill_at(daq_server *srv, const daq_fill *fill, int32_t flags,
                       uint64_t tag, int64_t t_arrive_ns, uint64_t *ticket);

/* Limits of the serving loop (both 0 = none; at creation: a 10 ms admission
 * deadline, the spacing of fills inside a burst (Section 3), and a 10 s
 * batch time-out).
 * admit_deadline_us: a fill admitted later than this after its arrival
 *   counts in stats.late.
 * batch_timeout_us: the longest a worker waits for its batch. Past it the
 *   batch's fills complete with status DAQ_ETIMEDOUT and the worker takes
 *   new work; their slots are freed (after daq_release) only once the device
 *   has finished with them. EINVAL for negative values. */
int daq_server_set_limits(daq_server *srv, int64_t admit_deadline_us,
                          int64_t batch_timeout_us);

/* Copies up to max finished fills (oldest completion first) to out and
 * returns how many; waits up to timeout_us for the first one (0 = do not
 * wait). Negative on error. */
int daq_poll(daq_server *srv, daq_completion *out, int32_t max,
             int32_t timeout_us);

/* Frees the slot of a finished fill (for a DAQ_ETIMEDOUT fill: once the
 * device has finished with it). DAQ_EAGAIN while the fill is queued or
 * running, EINVAL for an unknown or already released ticket. */
int daq_release(daq_server *srv, uint64_t ticket);

int daq_server_get_stats(daq_server *srv, daq_server_stats *st);

/* Stops the workers after their current launches (queued fills are dropped),
 * waits for the device to finish every launch (timed-out ones included) and
 * frees the server's host and scratch memory. NULL ok. */
void daq_server_destroy(daq_server *srv);

/* ---- measurement -----------------------------------------------------------
 * The device's plain streaming-read rate, the ceiling the chop's summing scan
 * (which reads every raw sample once) is measured against: reads
 * floor(bytes / 16) 16-byte words of d_buf (16-byte aligned) once with
 * non-temporal loads (eight in flight per thread) in a grid of `blocks`
 * work-groups of 256 threads, and writes one word per wave (an XOR of what it
 * read) to d_sink, which must hold blocks * 4 words. layout 0: grid-stride
 * (consecutive waves read consecutive 1 KB pieces); layout 1: each
 * work-group reads one contiguous chunk. Asynchronous on `stream`; time it
 * with events. EINVAL for null pointers, bytes < 16, blocks < 1, a
 * misaligned buffer or another layout. */
int daq_read_stream(const void *d_buf, int64_t bytes, unsigned int *d_sink,
                    int32_t blocks, int32_t layout, void *stream);

/* The rate of the chop scan's own read pattern, with nothing else done:
 * reads n_fills fills of `channels` rows of n_samples int16 each (row r of
 * fill f at d_raw + (f * channels + r) * n_samples, 16-byte aligned) in the
 * split scan's tiles at 512 threads (4,048 owned samples plus a 32-sample
 * left and 16-sample right halo, every channel row, 9 rows in flight, 16-byte
 * non-temporal loads; groups of 8 outside a row are skipped), in a persistent
 * grid of `blocks` work-groups of 512 threads striding over the tiles.
 * Writes the wrapping sum of the 32-bit words each wave read to d_sink (blocks
 * * 8 words). mode 0: that read alone. Modes 1 and 2 model a single pass
 * that writes the islands from the scan: after each tile, the threads whose
 * 8-sample group (sample / 8 of the row) is below 11 modulo 70 read their
 * group of every row again (9 rows in flight, added to the sums); mode 2
 * also stores each of those 16-byte words to d_out at word
 * (t * channels + r) * 512 + k, t the tile's index in the launch (fill by
 * fill) and k the thread's rank among the tile's pattern threads (d_out:
 * n_fills * ceil(n_samples / 4048) * channels * 512 words of 16 bytes,
 * 16-byte aligned; ignored by modes 0 and 1). Asynchronous on `stream`.
 * EINVAL for null pointers, n_fills or channels < 1, n_samples < 8 or not a
 * multiple of 8, blocks < 1, another mode or a misaligned buffer. */
int daq_read_tiles(const int16_t *d_raw, int32_t n_fills, int32_t channels,
                   int64_t n_samples, unsigned int *d_sink, int32_t blocks,
                   int32_t mode, void *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DAQ_H */
