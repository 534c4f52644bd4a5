// daq_runtime.cpp -- host runtime and C ABI of libdaqisland (include/daq.h).
//
// Owns per-stream scratch (look-back words, tile dispenser, effective
// thresholds, device descriptor tables and their pinned staging ring),
// validates arguments, lays out tiles, launches the kernels directly or by
// replaying captured HIP graphs, times the fused kernel on request and runs
// the schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "chop_internal.h"
#include "daq.h"
#include "daq_log.h"

using daqk::BatchHdr;
using daqk::FillDev;
using daqk::GatherArgs;
using daqk::KArgs;

namespace {

thread_local int g_last_hip = 0;

// Records a failed HIP call (daq_last_hip_error) and maps it to a status.
int hip_fail(hipError_t e, const char *what = "a HIP call") {
    g_last_hip = (int)e;
    daqlog::say(1, "%s failed: %s (%d)", what, hipGetErrorName(e), (int)e);
    return e == hipErrorOutOfMemory ? DAQ_ENOMEM : DAQ_EHIP;
}

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr int kRing = 4;          // pinned staging slots per stream
// Launches reading more raw bytes than this stream them with non-temporal
// loads; smaller ones keep their rows cached for the island write-out (the
// last-level cache holds 256 MB).
#ifndef DAQ_STREAM_LOAD_MB
#define DAQ_STREAM_LOAD_MB 128
#endif
constexpr int64_t kStreamLoadBytes = (int64_t)DAQ_STREAM_LOAD_MB << 20;
constexpr int kPrepareBlocks = 1024;

struct GraphKey {
    int threads = 0, wgs = 0, variant = 0, parts = 0;
    const void *table = nullptr;
    const void *state = nullptr;
    bool operator==(const GraphKey &o) const {
        return threads == o.threads && wgs == o.wgs && variant == o.variant && parts == o.parts &&
               table == o.table && state == o.state;
    }
};

struct Scratch {
    hipStream_t stream = nullptr;
    uint64_t *tile_state = nullptr;
    int64_t tile_cap = 0;
    uint32_t *ticket = nullptr;
    int64_t *thr_eff = nullptr;
    BatchHdr *hdr = nullptr;    // device: the header, then the table (one upload)
    FillDev *table = nullptr;   // device, inside the hdr allocation
    std::vector<uint8_t> last_desc;  // bytes of the last uploaded header and table
    int32_t fill_cap = 0;
    void *ring_host[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_pos = 0;
    hipGraphExec_t g_prep = nullptr, g_chop = nullptr;  // the two halves (timed launches)
    hipGraphExec_t g_all = nullptr;                     // both in one graph (untimed launches)
    GraphKey key;
    uint64_t *tile_pref = nullptr;  // split variant: tile prefixes (tile_cap)
    uint8_t *mask = nullptr;        // split variant: island-mask bits of all fills
    int64_t mask_cap = 0;
    int32_t *q_ped = nullptr;       // Q-method: pedestals of fills that have no ped output
    int64_t q_ped_cap = 0;
    int64_t *z_gofs = nullptr;      // compression: payload offsets of block groups
    int64_t z_gofs_cap = 0;
    // split variant with fill groups: streams of groups 1.., fork/join events
    hipStream_t part_stream[daqk::kMaxParts] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_scan[daqk::kMaxParts] = {};
    hipEvent_t ev_join[daqk::kMaxParts] = {};
};

}  // namespace

struct daq_ctx {
    int device = 0;
    int n_cu = 0;
    std::string name;
    std::vector<Scratch *> scratch;
    daq_schedule sched{512, 8, daqk::kVariantSplit, 0};
    bool graphs = true;
    bool timing = false;
    bool pinned = false;  // schedule (and graph mode) fixed by DAQ_SCHEDULE
    // event pairs bracketing fused-kernel launches while timing is on;
    // launches [t_read, t_next) have not been reported yet
    std::vector<hipEvent_t> ev_start, ev_stop;
    uint64_t t_next = 0, t_read = 0;
    hipStream_t capture = nullptr;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

constexpr size_t kMaxTimed = 1 << 14;  // event pairs kept between reads

// Records the start event of a timed launch; returns its slot.
int timing_begin(daq_ctx *ctx, hipStream_t stream, size_t *slot) {
    const size_t i = (size_t)(ctx->t_next % kMaxTimed);
    if (i >= ctx->ev_start.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        HIP_TRY(hipEventCreate(&a));
        hipError_t e = hipEventCreate(&b);
        if (e != hipSuccess) {
            (void)hipEventDestroy(a);
            return hip_fail(e, "hipEventCreate");
        }
        ctx->ev_start.push_back(a);
        ctx->ev_stop.push_back(b);
    }
    *slot = i;
    HIP_TRY(hipEventRecord(ctx->ev_start[i], stream));
    return DAQ_OK;
}

int timing_end(daq_ctx *ctx, hipStream_t stream, size_t slot) {
    HIP_TRY(hipEventRecord(ctx->ev_stop[slot], stream));
    ctx->t_next++;
    if (ctx->t_next - ctx->t_read > kMaxTimed) ctx->t_read = ctx->t_next - kMaxTimed;
    return DAQ_OK;
}

void free_graphs(Scratch *s) {
    if (s->g_prep) (void)hipGraphExecDestroy(s->g_prep);
    if (s->g_chop) (void)hipGraphExecDestroy(s->g_chop);
    if (s->g_all) (void)hipGraphExecDestroy(s->g_all);
    s->g_prep = s->g_chop = s->g_all = nullptr;
    s->key = GraphKey{};
}

void free_scratch(Scratch *s) {
    free_graphs(s);
    for (int k = 0; k < daqk::kMaxParts; k++) {
        if (s->part_stream[k]) (void)hipStreamSynchronize(s->part_stream[k]);
        if (s->part_stream[k]) (void)hipStreamDestroy(s->part_stream[k]);
        if (s->ev_scan[k]) (void)hipEventDestroy(s->ev_scan[k]);
        if (s->ev_join[k]) (void)hipEventDestroy(s->ev_join[k]);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    (void)hipFree(s->tile_state);
    (void)hipFree(s->ticket);
    (void)hipFree(s->thr_eff);
    (void)hipFree(s->hdr);
    (void)hipFree(s->tile_pref);
    (void)hipFree(s->mask);
    (void)hipFree(s->q_ped);
    (void)hipFree(s->z_gofs);
    for (int i = 0; i < kRing; i++) {
        if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
        if (s->ring_host[i]) (void)hipHostFree(s->ring_host[i]);
    }
    delete s;
}

Scratch *scratch_for(daq_ctx *ctx, hipStream_t stream) {
    for (Scratch *s : ctx->scratch)
        if (s->stream == stream) return s;
    Scratch *s = new Scratch();
    s->stream = stream;
    ctx->scratch.push_back(s);
    return s;
}

// Grows the scratch of one stream; waits for that stream first because the
// old buffers may still be in use by queued work or captured graphs.
int ensure_scratch(Scratch *s, int64_t tiles, int32_t fills, int64_t mask_bytes) {
    if (!s->ticket) HIP_TRY(hipMalloc(&s->ticket, 64));
    if (tiles <= s->tile_cap && fills <= s->fill_cap && s->ring_host[0] && mask_bytes <= s->mask_cap)
        return DAQ_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    free_graphs(s);
    daqlog::say(2, "scratch of stream %p grows for %lld tiles, %d fills, %lld mask bytes", (void *)s->stream,
                (long long)tiles, fills, (long long)mask_bytes);
    if (tiles > s->tile_cap) {
        int64_t cap = std::max<int64_t>(tiles + tiles / 2, 4096);
        (void)hipFree(s->tile_state);
        (void)hipFree(s->tile_pref);
        s->tile_state = nullptr;
        s->tile_pref = nullptr;
        s->tile_cap = 0;
        HIP_TRY(hipMalloc(&s->tile_state, (size_t)cap * sizeof(uint64_t)));
        HIP_TRY(hipMalloc(&s->tile_pref, (size_t)cap * sizeof(uint64_t)));
        s->tile_cap = cap;
    }
    if (mask_bytes > s->mask_cap) {
        const int64_t cap = std::max<int64_t>(mask_bytes + mask_bytes / 2, 1 << 20);
        (void)hipFree(s->mask);
        s->mask = nullptr;
        s->mask_cap = 0;
        HIP_TRY(hipMalloc(&s->mask, (size_t)cap));
        s->mask_cap = cap;
    }
    if (fills > s->fill_cap || !s->ring_host[0]) {
        int32_t cap = std::max<int32_t>(fills + fills / 2, 64);
        (void)hipFree(s->thr_eff);
        (void)hipFree(s->hdr);
        s->thr_eff = nullptr;
        s->table = nullptr;
        s->hdr = nullptr;
        s->fill_cap = 0;
        HIP_TRY(hipMalloc(&s->thr_eff, (size_t)cap * sizeof(int64_t)));
        HIP_TRY(hipMalloc(&s->hdr, sizeof(BatchHdr) + (size_t)cap * sizeof(FillDev)));
        s->table = reinterpret_cast<FillDev *>(s->hdr + 1);
        s->last_desc.clear();
        for (int i = 0; i < kRing; i++) {
            if (s->ring_used[i]) HIP_TRY(hipEventSynchronize(s->ring_ev[i]));
            if (s->ring_host[i]) (void)hipHostFree(s->ring_host[i]);
            s->ring_host[i] = nullptr;
            s->ring_used[i] = false;
            HIP_TRY(hipHostMalloc(&s->ring_host[i], sizeof(BatchHdr) + (size_t)cap * sizeof(FillDev),
                                  hipHostMallocDefault));
            if (!s->ring_ev[i]) HIP_TRY(hipEventCreateWithFlags(&s->ring_ev[i], hipEventDisableTiming));
        }
        s->fill_cap = cap;
    }
    return DAQ_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int check_fill(const daq_fill *f) {
    if (!f) return DAQ_EINVAL;
    if (f->reserved != 0) return DAQ_EINVAL;
    if (f->n_samples < 0 || f->row_stride < f->n_samples) return DAQ_EINVAL;
    if (f->n_samples > DAQ_MAX_SAMPLES) return DAQ_ERANGE;
    if (f->n_channels < 1 || f->ped_samples < 1 || f->pre < 0 || f->post < 0) return DAQ_EINVAL;
    if (f->n_channels > DAQ_MAX_CHANNELS || f->pre > DAQ_MAX_WINDOW || f->post > DAQ_MAX_WINDOW)
        return DAQ_ERANGE;
    if (f->row_stride > DAQ_MAX_SAMPLES + 8) return DAQ_ERANGE;
    if (f->n_samples > 0 && !f->raw) return DAQ_EINVAL;
    if ((f->row_stride % daqk::kVec) != 0 || !aligned16(f->raw)) return DAQ_EALIGN;
    return DAQ_OK;
}

int check_out(const daq_fill_out *o) {
    if (!o || !o->counts) return DAQ_EINVAL;
    if (o->capacity < 0 || (o->capacity > 0 && !o->islands)) return DAQ_EINVAL;
    if (o->out && o->out_stride < 0) return DAQ_EINVAL;
    return DAQ_OK;
}

int64_t tiles_of(const daq_fill &f, const daq_schedule &sc) {
    const int64_t T = daqk::tile_shape(f.pre, f.post, f.n_channels, sc.threads, sc.variant).tout;
    return (f.n_samples + T - 1) / T;
}

// Scratch of one fill under the split variant: island-mask bits (with
// guards), the (start, offset) run table for the worst-case island count and
// the island of every chunk start, each part 16-byte aligned.
struct SplitLayout {
    int64_t runs = 0, cmap = 0, bytes = 0;
};
SplitLayout split_layout_of(const daq_fill &f, const daq_schedule &sc) {
    const int64_t tout = daqk::tile_shape(f.pre, f.post, f.n_channels, sc.threads, sc.variant).tout;
    const int64_t data = tiles_of(f, sc) * tout / daqk::kVec;
    SplitLayout L;
    L.runs = (data + 2 * daqk::kMaskGuard + 15) / 16 * 16;
    const int64_t isl = std::max<int64_t>(daq_max_islands(f.n_samples, f.pre, f.post), 0);
    L.cmap = L.runs + (8 * isl + 15) / 16 * 16;
    const int64_t chunks = (f.n_samples + daqk::kCopyChunk - 1) / daqk::kCopyChunk + 2;
    L.bytes = L.cmap + (4 * chunks + 15) / 16 * 16;
    return L;
}

FillDev make_desc(const daq_fill &f, const daq_fill_out &o, int64_t tile_base, const daq_schedule &sc) {
    const daqk::TileShape ts = daqk::tile_shape(f.pre, f.post, f.n_channels, sc.threads, sc.variant);
    FillDev d{};
    d.raw = f.raw;
    d.n = f.n_samples;
    d.stride = f.row_stride;
    d.C = f.n_channels;
    d.np = f.ped_samples;
    d.thr = f.threshold;
    d.pre = f.pre;
    d.post = f.post;
    d.gl = ts.gl;
    d.gr = ts.gr;
    d.wide = ts.wide;
    d.mode = ts.mode;
    d.tout = ts.tout;
    d.tile_base = tile_base;
    d.n_tiles = tiles_of(f, sc);
    d.isl = o.islands;
    d.cap = o.capacity;
    d.counts = o.counts;
    d.ped = o.ped;
    d.out = o.out;
    d.out_stride = o.out ? o.out_stride : 0;
    return d;
}

int chop_grid(const daq_ctx *ctx, const daq_schedule &s, int64_t total_tiles) {
    int64_t g = s.wgs_per_cu > 0 ? (int64_t)s.wgs_per_cu * ctx->n_cu : total_tiles;
    g = std::min<int64_t>(std::max<int64_t>(g, 1), total_tiles > 0 ? total_tiles : 1);
    return (int)std::min<int64_t>(g, 1 << 30);
}

bool all_calorimeters(const daq_fill *fills, int32_t n) {
    for (int32_t i = 0; i < n; i++)
        if (fills[i].n_channels != daqk::kResidentChannels) return false;
    return true;
}

// Streams and events for cutting a split launch into `parts` fill groups.
int ensure_parts(Scratch *sc, int parts) {
    if (!sc->ev_fork) HIP_TRY(hipEventCreateWithFlags(&sc->ev_fork, hipEventDisableTiming));
    for (int k = 0; k < parts; k++) {
        if (k > 0 && !sc->part_stream[k]) HIP_TRY(hipStreamCreateWithFlags(&sc->part_stream[k], hipStreamNonBlocking));
        if (!sc->ev_scan[k]) HIP_TRY(hipEventCreateWithFlags(&sc->ev_scan[k], hipEventDisableTiming));
        if (!sc->ev_join[k]) HIP_TRY(hipEventCreateWithFlags(&sc->ev_join[k], hipEventDisableTiming));
    }
    return DAQ_OK;
}

// Work-groups of the edge pass: one wave per tile, so no more than the
// tiles need (tiles < 0: not known, as in a captured graph that may be
// replayed for any batch its scratch holds), and at most the scan's grid.
int edge_grid(int grid, int64_t tiles, int threads) {
    if (tiles < 0) return grid;
    const int64_t waves = threads / 64;
    return (int)std::max<int64_t>(1, std::min<int64_t>(grid, (tiles + waves - 1) / waves));
}

int launch_main(const daq_ctx *ctx, Scratch *sc, const KArgs &a, const daq_schedule &s, int grid,
                int64_t tiles, hipStream_t stream) {
    if (s.variant == daqk::kVariantPipe) {
        HIP_TRY(daqk::launch_pipe(a, s.threads, grid, stream));
        return DAQ_OK;
    }
    if (s.variant == daqk::kVariantSplit) {
        const int parts = (a.table && s.parts > 1) ? std::min(s.parts, daqk::kMaxParts) : 1;
        const int eg = edge_grid(grid, tiles, s.threads);
        if (parts == 1) {
            KArgs a1 = a;
            a1.part = 0;
            a1.parts = 1;
            HIP_TRY(daqk::launch_scan(a1, s.threads, grid, stream));
            HIP_TRY(daqk::launch_emit(a1, s.threads, eg, daqk::kCopyWgsPerCu * ctx->n_cu, stream));
            return DAQ_OK;
        }
        // fill group k runs on its own stream; its scan starts when group
        // k-1's scan has finished, so group k's scan overlaps the edge and
        // copy passes of group k-1
        int rc = ensure_parts(sc, parts);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(sc->ev_fork, stream));
        for (int k = 0; k < parts; k++) {
            hipStream_t sk = k == 0 ? stream : sc->part_stream[k];
            KArgs ak = a;
            ak.part = k;
            ak.parts = parts;
            if (k > 0) {
                HIP_TRY(hipStreamWaitEvent(sk, sc->ev_fork, 0));
                HIP_TRY(hipStreamWaitEvent(sk, sc->ev_scan[k - 1], 0));
            }
            HIP_TRY(daqk::launch_scan(ak, s.threads, grid, sk));
            HIP_TRY(hipEventRecord(sc->ev_scan[k], sk));
            HIP_TRY(daqk::launch_emit(ak, s.threads, eg, daqk::kCopyWgsPerCu * ctx->n_cu, sk));
            if (k > 0) HIP_TRY(hipEventRecord(sc->ev_join[k], sk));
        }
        for (int k = 1; k < parts; k++) HIP_TRY(hipStreamWaitEvent(stream, sc->ev_join[k], 0));
        return DAQ_OK;
    }
    (void)ctx;
    (void)sc;
    HIP_TRY(daqk::launch_chop(a, s.threads, s.variant, grid, stream));
    return DAQ_OK;
}

// Whether a launch needs k_prepare first: the split schedule's scan computes
// the pedestals itself unless the Q-method rides along (its bins are cleared
// by k_prepare).
bool needs_prepare(const daq_schedule &s, const KArgs &a) {
    return s.variant != daqk::kVariantSplit || a.q_fused != 0;
}

int prepare_blocks(const KArgs &a, int64_t total_tiles) {
    int prep_blocks = (int)std::min<int64_t>(kPrepareBlocks, std::max<int64_t>(1, (total_tiles + 2047) / 2048));
    prep_blocks = std::max(prep_blocks, std::min(a.n_fills, kPrepareBlocks));
    return std::min(prep_blocks, std::max(a.n_fills, 64));
}

int launch_pair(daq_ctx *ctx, Scratch *sc, const KArgs &a, int64_t total_tiles, hipStream_t stream,
                const daq_schedule &s) {
    // a launch without tiles only clears the counts and pedestals (k_prepare)
    if (needs_prepare(s, a) || total_tiles == 0) HIP_TRY(daqk::launch_prepare(a, prepare_blocks(a, total_tiles), stream));
    if (total_tiles == 0) return DAQ_OK;
    size_t slot = 0;
    if (ctx->timing) {
        int rc = timing_begin(ctx, stream, &slot);
        if (rc) return rc;
    }
    int rc = launch_main(ctx, sc, a, s, chop_grid(ctx, s, total_tiles), total_tiles, stream);
    if (rc) return rc;
    if (ctx->timing) return timing_end(ctx, stream, slot);
    return DAQ_OK;
}

// Captures the two kernels of a table-driven launch (sizes read from the
// device header) into two graph execs bound to this scratch.
int capture_graphs(daq_ctx *ctx, Scratch *s, const daq_schedule &sc) {
    free_graphs(s);
    if (!ctx->capture) HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    KArgs a{};
    a.table = s->table;
    a.hdr = s->hdr;
    a.tile_state = s->tile_state;
    a.ticket = s->ticket;
    a.thr_eff = s->thr_eff;
    a.tile_pref = s->tile_pref;
    hipGraph_t g = nullptr;
    // graphs never carry the Q-method: only schedules other than the split
    // one need k_prepare
    const bool prep = needs_prepare(sc, a);
    hipError_t e = hipSuccess, e2 = hipSuccess;
    if (prep) {
        // prepare: grid covers the largest table this scratch holds
        HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        e = daqk::launch_prepare(a, kPrepareBlocks, ctx->capture);
        e2 = hipStreamEndCapture(ctx->capture, &g);
        if (e != hipSuccess) return hip_fail(e, "launch_prepare (capture)");
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&s->g_prep, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    }
    HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    const int rc0 = launch_main(ctx, s, a, sc, sc.wgs_per_cu * ctx->n_cu, -1, ctx->capture);
    e2 = hipStreamEndCapture(ctx->capture, &g);
    if (rc0) return rc0;
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->g_chop, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    // prepare (if any) and main pass in one graph: one launch, no gap between the two
    HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    e = prep ? daqk::launch_prepare(a, kPrepareBlocks, ctx->capture) : hipSuccess;
    const int rc1 = e == hipSuccess ? launch_main(ctx, s, a, sc, sc.wgs_per_cu * ctx->n_cu, -1, ctx->capture) : DAQ_OK;
    e2 = hipStreamEndCapture(ctx->capture, &g);
    if (e != hipSuccess) return hip_fail(e, "launch_prepare (capture)");
    if (rc1) return rc1;
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&s->g_all, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    s->key.threads = sc.threads;
    s->key.wgs = sc.wgs_per_cu;
    s->key.variant = sc.variant;
    s->key.parts = sc.parts;
    s->key.table = s->table;
    s->key.state = s->tile_state;
    daqlog::say(2, "graphs captured for schedule %d/%d/%d/%d on stream %p", sc.threads, sc.wgs_per_cu, sc.variant,
                sc.parts, (void *)s->stream);
    return DAQ_OK;
}

// The fused pass over n fills. n == 1 without `force_table` passes the one
// descriptor in the kernel arguments; otherwise the descriptors go through a
// pinned staging slot into the device table (and graphs may be replayed).
int check_q_out(const daq_fill &f, const daq_q_out &o);
bool q_acc_overlap(const daq_fill *fills, const daq_q_out *outs, int32_t n);

// qouts (optional): the Q-method runs inside the split schedule's scan pass,
// on the same read of the raw samples (plain launches, no graph).
int run_fused(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs, int32_t n,
              hipStream_t stream, bool force_table, const daq_q_out *qouts = nullptr) {
    if (!ctx || n < 0 || (n > 0 && (!fills || !outs))) return DAQ_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        int rc = check_fill(&fills[i]);
        if (rc) return rc;
        rc = check_out(&outs[i]);
        if (rc) return rc;
        if (qouts) {
            rc = check_q_out(fills[i], qouts[i]);
            if (rc) return rc;
            if (qouts[i].ped && outs[i].ped) return DAQ_EINVAL;
        }
    }
    if (qouts && q_acc_overlap(fills, qouts, n)) return DAQ_EINVAL;
    if (n == 0) return DAQ_OK;
    DeviceGuard guard(ctx->device);
    daq_schedule sc = ctx->sched;
    if (qouts && sc.variant != daqk::kVariantSplit) sc = daq_schedule{256, 16, daqk::kVariantSplit, 0};
    // the register variant keeps exactly 54 rows per thread: calls with other
    // channel counts run the re-read variant
    if (sc.variant == daqk::kVariantResident && !all_calorimeters(fills, n)) sc.variant = daqk::kVariantReload;
    int64_t total = 0, mask_total = 0, max_chunks = 0;
    std::vector<int64_t> base((size_t)n), moff((size_t)n, -1);
    std::vector<SplitLayout> lay((size_t)n);
    // the pipe variant uses the split variant's run table and chunk map
    const bool split = sc.variant == daqk::kVariantSplit || sc.variant == daqk::kVariantPipe;
    int64_t raw_bytes = 0;
    for (int32_t i = 0; i < n; i++) {
        base[(size_t)i] = total;
        total += tiles_of(fills[i], sc);
        raw_bytes += 2 * (int64_t)fills[i].n_channels * fills[i].n_samples;
        if (split) {
            moff[(size_t)i] = mask_total;
            lay[(size_t)i] = split_layout_of(fills[i], sc);
            mask_total += lay[(size_t)i].bytes;
            max_chunks = std::max<int64_t>(max_chunks, (fills[i].n_samples + daqk::kCopyChunk - 1) /
                                                           daqk::kCopyChunk);
        }
    }
    Scratch *s = scratch_for(ctx, stream);
    // tile words double as per-fill words (pipe variant): at least one per fill
    int rc = ensure_scratch(s, std::max<int64_t>(total, n), n, mask_total);
    if (rc) return rc;
    // fused Q-method: the accumulator update needs the pedestals in memory
    std::vector<int64_t> poff((size_t)n, -1);
    if (qouts) {
        int64_t ped_need = 0;
        for (int32_t i = 0; i < n; i++)
            if (!outs[i].ped && !qouts[i].ped) {
                poff[(size_t)i] = ped_need;
                ped_need += fills[i].n_channels;
            }
        if (ped_need > s->q_ped_cap) {
            HIP_TRY(hipStreamSynchronize(stream));
            (void)hipFree(s->q_ped);
            s->q_ped = nullptr;
            s->q_ped_cap = 0;
            const int64_t cap = std::max<int64_t>(ped_need + ped_need / 2, 4096);
            HIP_TRY(hipMalloc(&s->q_ped, (size_t)cap * sizeof(int32_t)));
            s->q_ped_cap = cap;
        }
    }
    auto desc = [&](int32_t i) {
        FillDev d = make_desc(fills[i], outs[i], base[(size_t)i], sc);
        d.mbits = split ? s->mask + moff[(size_t)i] + daqk::kMaskGuard : nullptr;
        d.runs = split ? reinterpret_cast<int32_t *>(s->mask + moff[(size_t)i] + lay[(size_t)i].runs) : nullptr;
        d.cmap = split ? reinterpret_cast<int32_t *>(s->mask + moff[(size_t)i] + lay[(size_t)i].cmap) : nullptr;
        if (qouts) {
            const daq_q_out &q = qouts[i];
            if (!d.ped) d.ped = q.ped ? q.ped : s->q_ped + poff[(size_t)i];
            d.qsum = q.qsum;
            d.acc = q.acc;
            d.acc_stride = q.acc ? q.acc_stride : 0;
        }
        return d;
    };
    KArgs a{};
    a.tile_state = s->tile_state;
    a.ticket = s->ticket;
    a.thr_eff = s->thr_eff;
    a.tile_pref = s->tile_pref;
    a.n_fills = n;
    a.total_tiles = total;
    a.stream_loads = raw_bytes > kStreamLoadBytes ? 1 : 0;
    a.copy_slots = split ? max_chunks * n : 0;
    a.q_fused = qouts ? 1 : 0;
    if (n == 1 && !force_table) {
        a.one = desc(0);
        return launch_pair(ctx, s, a, total, stream, sc);
    }
    // stage the descriptors
    const int rs = s->ring_pos;
    s->ring_pos = (s->ring_pos + 1) % kRing;
    if (s->ring_used[rs]) HIP_TRY(hipEventSynchronize(s->ring_ev[rs]));
    BatchHdr *h = reinterpret_cast<BatchHdr *>(s->ring_host[rs]);
    FillDev *tab = reinterpret_cast<FillDev *>(h + 1);
    h->n_fills = n;
    h->stream_loads = a.stream_loads;
    h->total_tiles = total;
    h->copy_slots = a.copy_slots;
    h->pad2 = 0;
    for (int32_t i = 0; i < n; i++) tab[i] = desc(i);
    // one upload of header and table, skipped when the device already holds
    // exactly these bytes (the same batch launched again)
    const size_t bytes = sizeof(BatchHdr) + (size_t)n * sizeof(FillDev);
    const uint8_t *img = reinterpret_cast<const uint8_t *>(h);
    if (s->last_desc.size() != bytes || std::memcmp(s->last_desc.data(), img, bytes) != 0) {
        HIP_TRY(hipMemcpyAsync(s->hdr, h, bytes, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipEventRecord(s->ring_ev[rs], stream));
        s->ring_used[rs] = true;
        s->last_desc.assign(img, img + bytes);
    }
    a.table = s->table;
    a.hdr = s->hdr;
    const bool use_graph = ctx->graphs && sc.wgs_per_cu > 0 && !qouts;
    if (!use_graph) return launch_pair(ctx, s, a, total, stream, sc);
    GraphKey want;
    want.threads = sc.threads;
    want.wgs = sc.wgs_per_cu;
    want.variant = sc.variant;
    want.parts = sc.parts;
    want.table = s->table;
    want.state = s->tile_state;
    if (!s->g_chop || !(s->key == want)) {
        rc = capture_graphs(ctx, s, sc);
        if (rc) return rc;
    }
    if (!ctx->timing) {
        HIP_TRY(hipGraphLaunch(s->g_all, stream));
        return DAQ_OK;
    }
    if (s->g_prep) HIP_TRY(hipGraphLaunch(s->g_prep, stream));
    size_t slot = 0;
    if (ctx->timing) {
        rc = timing_begin(ctx, stream, &slot);
        if (rc) return rc;
    }
    HIP_TRY(hipGraphLaunch(s->g_chop, stream));
    if (ctx->timing) return timing_end(ctx, stream, slot);
    return DAQ_OK;
}

// ---- autotune ---------------------------------------------------------------

// Poison of every output buffer before a candidate's first run: records and
// counts all bits set (each field reads -1), pedestals and packed rows 0x5A
// bytes. A candidate that leaves an output unwritten then differs from the
// reference instead of inheriting the previous candidate's bytes.
__global__ void k_poison_outputs(const FillDev *tab, int n) {
    const int f = blockIdx.y;
    if (f >= n) return;
    const FillDev d = tab[f];
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    if (gtid == 0 && d.counts) {
        d.counts->n_islands = -1;
        d.counts->total_len = -1;
        d.counts->status = -1;
        d.counts->reserved = -1;
    }
    int64_t *isl = reinterpret_cast<int64_t *>(d.isl);
    for (int64_t i = gtid; i < 3 * d.cap; i += gsz) isl[i] = -1;
    if (d.ped)
        for (int64_t i = gtid; i < d.C; i += gsz) d.ped[i] = 0x5A5A5A5A;
    if (d.out) {
        const int64_t total = (int64_t)d.C * d.out_stride;  // the rows are contiguous
        int64_t head = 0;
        if (((uintptr_t)d.out & 15u) == 0) {
            uint4 *o16 = reinterpret_cast<uint4 *>(d.out);
            const uint4 v = make_uint4(0x5A5A5A5Au, 0x5A5A5A5Au, 0x5A5A5A5Au, 0x5A5A5A5Au);
            for (int64_t i = gtid; i < total / 8; i += gsz) o16[i] = v;
            head = total / 8 * 8;
        }
        for (int64_t i = head + gtid; i < total; i += gsz) d.out[i] = (int16_t)0x5A5A;
    }
}

// Where the reference copy of one fill's outputs sits.
struct RefFill {
    const daq_counts *counts;
    const int64_t *isl;
    const int32_t *ped;
    const int16_t *out;
};

// Counts the elements of fill blockIdx.y's defined outputs that differ from
// the reference: counts, records [0, min(n, cap)), pedestals, and every
// packed row up to min(total_len, out_stride).
__global__ void k_compare_outputs(const FillDev *tab, const RefFill *ref, int n, unsigned long long *bad) {
    const int f = blockIdx.y;
    if (f >= n) return;
    const FillDev d = tab[f];
    const RefFill r = ref[f];
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    const daq_counts c = *d.counts, rc = *r.counts;
    if (c.n_islands != rc.n_islands || c.total_len != rc.total_len || c.status != rc.status ||
        c.reserved != rc.reserved) {
        if (gtid == 0) atomicAdd(&bad[f], 1ull);
        return;
    }
    unsigned long long miss = 0;
    const int64_t nrec = c.n_islands < d.cap ? (c.n_islands < 0 ? 0 : c.n_islands) : d.cap;
    const int64_t *isl = reinterpret_cast<const int64_t *>(d.isl);
    for (int64_t i = gtid; i < 3 * nrec; i += gsz) miss += isl[i] != r.isl[i];
    if (d.ped)
        for (int64_t i = gtid; i < d.C; i += gsz) miss += d.ped[i] != r.ped[i];
    if (d.out) {
        const int64_t len = c.total_len < d.out_stride ? (c.total_len < 0 ? 0 : c.total_len) : d.out_stride;
        const int64_t items = (int64_t)d.C * len;
        for (int64_t i = gtid; i < items; i += gsz) {
            const int64_t row = i / (len > 0 ? len : 1), k = i - row * len;
            miss += d.out[row * d.out_stride + k] != r.out[row * d.out_stride + k];
        }
    }
    for (int dd = 32; dd > 0; dd >>= 1) miss += __shfl_xor(miss, dd, 64);
    if ((threadIdx.x & 63) == 0 && miss) atomicAdd(&bad[f], miss);
}

constexpr int kCheckBlocks = 256;  // blocks per fill of the poison and compare kernels

// The reference copy of a batch's outputs (the first candidate's), in one
// device allocation owned by the autotune call.
struct RefCopy {
    uint8_t *buf = nullptr;
    RefFill *d_ref = nullptr;
    unsigned long long *d_bad = nullptr;
    std::vector<RefFill> host;
    ~RefCopy() {
        (void)hipFree(buf);
        (void)hipFree(d_ref);
        (void)hipFree(d_bad);
    }
};

int64_t up256(int64_t b) { return (b + 255) / 256 * 256; }

int poison_outputs(Scratch *s, int32_t n, hipStream_t stream) {
    hipLaunchKernelGGL(k_poison_outputs, dim3(kCheckBlocks, n), dim3(256), 0, stream, s->table, n);
    HIP_TRY(hipGetLastError());
    return DAQ_OK;
}

// Copies every output buffer of the batch (whole buffers) into `rf`.
int snapshot_outputs(const daq_fill *fills, const daq_fill_out *outs, int32_t n, hipStream_t stream, RefCopy &rf) {
    int64_t bytes = 0;
    for (int32_t i = 0; i < n; i++) {
        const int64_t C = fills[i].n_channels;
        bytes += up256(sizeof(daq_counts)) + up256(24 * outs[i].capacity) + up256(4 * C) +
                 (outs[i].out ? up256(2 * C * outs[i].out_stride) : 0);
    }
    HIP_TRY(hipMalloc(&rf.buf, (size_t)std::max<int64_t>(bytes, 256)));
    HIP_TRY(hipMalloc(&rf.d_ref, (size_t)n * sizeof(RefFill)));
    HIP_TRY(hipMalloc(&rf.d_bad, (size_t)n * sizeof(unsigned long long)));
    rf.host.assign((size_t)n, RefFill{});
    int64_t o = 0;
    for (int32_t i = 0; i < n; i++) {
        const daq_fill_out &q = outs[i];
        const int64_t C = fills[i].n_channels;
        RefFill &r = rf.host[(size_t)i];
        uint8_t *b = rf.buf + o;
        r.counts = reinterpret_cast<const daq_counts *>(b);
        HIP_TRY(hipMemcpyAsync(b, q.counts, sizeof(daq_counts), hipMemcpyDeviceToDevice, stream));
        b += up256(sizeof(daq_counts));
        r.isl = reinterpret_cast<const int64_t *>(b);
        if (q.capacity > 0)
            HIP_TRY(hipMemcpyAsync(b, q.islands, (size_t)(24 * q.capacity), hipMemcpyDeviceToDevice, stream));
        b += up256(24 * q.capacity);
        r.ped = reinterpret_cast<const int32_t *>(b);
        if (q.ped) HIP_TRY(hipMemcpyAsync(b, q.ped, (size_t)(4 * C), hipMemcpyDeviceToDevice, stream));
        b += up256(4 * C);
        r.out = reinterpret_cast<const int16_t *>(b);
        if (q.out) {
            HIP_TRY(hipMemcpyAsync(b, q.out, (size_t)(2 * C * q.out_stride), hipMemcpyDeviceToDevice, stream));
            b += up256(2 * C * q.out_stride);
        }
        o = b - rf.buf;
    }
    HIP_TRY(hipMemcpyAsync(rf.d_ref, rf.host.data(), (size_t)n * sizeof(RefFill), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return DAQ_OK;
}

// Compares the batch's current outputs with the reference copy, element by
// element; *same is false when any fill differs.
int compare_outputs(Scratch *s, int32_t n, hipStream_t stream, RefCopy &rf, bool *same) {
    HIP_TRY(hipMemsetAsync(rf.d_bad, 0, (size_t)n * sizeof(unsigned long long), stream));
    hipLaunchKernelGGL(k_compare_outputs, dim3(kCheckBlocks, n), dim3(256), 0, stream, s->table, rf.d_ref, n,
                       rf.d_bad);
    HIP_TRY(hipGetLastError());
    std::vector<unsigned long long> bad((size_t)n, 0);
    HIP_TRY(hipMemcpyAsync(bad.data(), rf.d_bad, (size_t)n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *same = true;
    for (unsigned long long b : bad) *same = *same && b == 0;
    return DAQ_OK;
}

std::string shape_key(const daq_ctx *ctx, const daq_fill *fills, int32_t n) {
    int64_t tot = 0, mx = 0;
    int cmax = 0, wmax = 0;
    for (int32_t i = 0; i < n; i++) {
        tot += fills[i].n_samples;
        mx = std::max<int64_t>(mx, fills[i].n_samples);
        cmax = std::max(cmax, fills[i].n_channels);
        wmax = std::max(wmax, fills[i].pre + fills[i].post);
    }
    int lg = 0;
    while ((int64_t)1 << (lg + 1) <= std::max<int64_t>(tot, 1)) lg++;
    std::ostringstream o;
    std::string name = ctx->name;
    std::replace(name.begin(), name.end(), ' ', '_');
    o << name << " n" << n << " C" << cmax << " log2N" << lg << " w" << (wmax <= 64 ? 64 : wmax);
    return o.str();
}

// ---- scratch of the no-allocation entry point ----------------------------------
//
// One static device array per GPU (each device holds its own copy at its own
// address). Host code never passes `scratch` itself to a kernel or a copy: on
// the host that name is only a stand-in for the symbol. Its device address is
// looked up once per device, at the first daq_ctx_create on it, and kept in
// g_noalloc_ptr.
static __device__ __align__(256) uint8_t scratch[DAQ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint8_t *g_noalloc_ptr[kMaxDevices] = {};

// With `device` current: looks up the device address of the scratch array.
int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return DAQ_OK;  // such devices cannot use the entry point
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return DAQ_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[device] = static_cast<uint8_t *>(p);
    return DAQ_OK;
}

// DAQ_SCHEDULE="threads,wgs_per_cu,variant,parts[,graphs]" fixes a new
// context's schedule (and, with the fifth field, whether launches replay
// captured graphs); daq_autotune then keeps it instead of timing the menu.
// A value that does not parse, or that daq_ctx_set_schedule would refuse,
// fails the context's creation and says why on stderr at every log level.
int schedule_from_env(daq_ctx *c) {
    const char *env = std::getenv("DAQ_SCHEDULE");
    if (!env || !*env) return DAQ_OK;
    daq_schedule s{};
    int graphs = -1, used = 0;
    const int got = std::sscanf(env, "%d,%d,%d,%d%n,%d%n", &s.threads, &s.wgs_per_cu, &s.variant, &s.parts, &used,
                                &graphs, &used);
    if (got < 4 || env[used] != '\0' || (got == 5 && graphs != 0 && graphs != 1) ||
        daq_ctx_set_schedule(c, &s) != DAQ_OK) {
        daqlog::say(0, "DAQ_SCHEDULE=\"%s\" refused: expected threads,wgs_per_cu,variant,parts[,graphs] "
                       "that daq_ctx_set_schedule accepts, graphs 0 or 1", env);
        return DAQ_EINVAL;
    }
    if (got == 5) c->graphs = graphs == 1;
    c->pinned = true;
    return DAQ_OK;
}

uint8_t *noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

// Descriptors of up to kPutFills fills travel as kernel arguments into the
// table in the scratch array (no host staging buffer, no copy call).
constexpr int kPutFills = 16;
struct PutDescArgs {
    FillDev d[kPutFills];
    BatchHdr hdr;
    FillDev *dst;      // table entry of d[0]
    BatchHdr *dst_hdr; // written when write_hdr
    int32_t count, write_hdr;
};
static_assert(sizeof(PutDescArgs) <= 3584, "kernel arguments of the descriptor upload (explicit arguments well below 4 KB)");

__global__ void k_put_descs(PutDescArgs a) {
    constexpr int W = (int)(sizeof(FillDev) / 16);  // 16-byte words per descriptor
    const int i = (int)threadIdx.x;
    if (i < a.count * W) {
        const uint4 *src = reinterpret_cast<const uint4 *>(&a.d[0]);
        reinterpret_cast<uint4 *>(a.dst)[i] = src[i];
    }
    if (a.write_hdr && i == 0) *a.dst_hdr = a.hdr;
}

// Layout of one no-allocation call inside the scratch array (byte offsets).
struct NoAllocLayout {
    int64_t ticket = 0, thr_eff = 0, hdr = 0, tile_state = 0, tile_pref = 0, fills = 0, bytes = 0;
    int64_t total_tiles = 0, max_chunks = 0;
};

int64_t up16(int64_t b) { return (b + 15) / 16 * 16; }

// Validated fills only.
NoAllocLayout noalloc_layout(const daq_fill *fills, int32_t n, const daq_schedule &sc) {
    NoAllocLayout L;
    int64_t tiles = 0, per_fill = 0;
    for (int32_t i = 0; i < n; i++) {
        tiles += tiles_of(fills[i], sc);
        per_fill += up16(split_layout_of(fills[i], sc).bytes);
        L.max_chunks = std::max<int64_t>(L.max_chunks, (fills[i].n_samples + daqk::kCopyChunk - 1) / daqk::kCopyChunk);
    }
    L.total_tiles = tiles;
    int64_t o = 0;
    L.ticket = o;
    o += 256;
    L.thr_eff = o;
    o = up256(o + 8 * (int64_t)std::max(n, 1));
    L.hdr = o;
    o = up256(o + (int64_t)sizeof(BatchHdr) + (int64_t)n * (int64_t)sizeof(FillDev));
    L.tile_state = o;
    o = up256(o + 8 * std::max<int64_t>(tiles, n));
    L.tile_pref = o;
    o = up256(o + 8 * std::max<int64_t>(tiles, n));
    L.fills = o;
    o += per_fill;
    L.bytes = o;
    return L;
}

daq_schedule noalloc_schedule(const daq_ctx *ctx) {
    daq_schedule sc{512, 8, daqk::kVariantSplit, 0};
    if (ctx->sched.variant == daqk::kVariantSplit) {
        sc.threads = ctx->sched.threads;
        sc.wgs_per_cu = ctx->sched.wgs_per_cu > 0 ? ctx->sched.wgs_per_cu : 16;
    }
    return sc;
}

}  // namespace

// ---- C ABI --------------------------------------------------------------------

extern "C" {

const char *daq_version(void) { return "libdaqisland 1.0 (gfx950)"; }

const char *daq_strerror(int code) {
    switch (code) {
        case DAQ_OK: return "ok";
        case DAQ_EINVAL: return "invalid argument";
        case DAQ_EALIGN: return "raw base not 16-byte aligned or row stride not a multiple of 8";
        case DAQ_EHIP: return "HIP runtime error";
        case DAQ_ENOMEM: return "out of memory";
        case DAQ_EAGAIN: return "resource busy, try again";
        case DAQ_ERANGE: return "size exceeds a documented limit";
        case DAQ_EMISMATCH: return "autotune candidates produced different results";
        case DAQ_ETIMEDOUT: return "batch outlived the server's batch time-out";
        default: return "unknown error";
    }
}

int daq_last_hip_error(void) { return g_last_hip; }

int64_t daq_max_islands(int64_t n_samples, int32_t pre, int32_t post) {
    if (pre < 0 || post < 0) return -1;
    if (n_samples <= 0) return 0;
    return (n_samples - 1) / ((int64_t)pre + (int64_t)post + 2) + 1;
}

int daq_ctx_create(daq_ctx **out, int device) {
    if (!out) return DAQ_EINVAL;
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return DAQ_EINVAL;
    DeviceGuard guard(device);
    daq_ctx *c = new daq_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    c->n_cu = prop.multiProcessorCount;
    c->name = prop.gcnArchName;
    int rc = noalloc_init(device);
    if (rc == DAQ_OK) rc = schedule_from_env(c);
    if (rc != DAQ_OK) {
        delete c;
        return rc;
    }
    daqlog::say(2, "context on device %d: %s, %s, %d compute units, schedule %d/%d/%d/%d%s", device, prop.name,
                prop.gcnArchName, c->n_cu, c->sched.threads, c->sched.wgs_per_cu, c->sched.variant, c->sched.parts,
                c->pinned ? " (DAQ_SCHEDULE)" : "");
    *out = c;
    return DAQ_OK;
}

void daq_ctx_destroy(daq_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    for (Scratch *s : ctx->scratch) {
        (void)hipStreamSynchronize(s->stream);
        free_scratch(s);
    }
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    for (hipEvent_t e : ctx->ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->ev_stop) (void)hipEventDestroy(e);
    delete ctx;
}

int daq_ctx_get_device(daq_ctx *ctx, int *device) {
    if (!ctx || !device) return DAQ_EINVAL;
    *device = ctx->device;
    return DAQ_OK;
}

int daq_find_islands(daq_ctx *ctx, const daq_fill *fill, daq_island *d_islands, int64_t capacity,
                     daq_counts *d_counts, int32_t *d_ped, void *stream) {
    daq_fill_out o{};
    o.islands = d_islands;
    o.capacity = capacity;
    o.counts = d_counts;
    o.ped = d_ped;
    o.out = nullptr;
    o.out_stride = 0;
    return run_fused(ctx, fill, &o, 1, (hipStream_t)stream, false);
}

int daq_gather_islands(daq_ctx *ctx, const daq_fill *fill, const daq_island *d_islands, int64_t capacity,
                       daq_counts *d_counts, int16_t *d_out, int64_t out_stride, void *stream) {
    if (!ctx) return DAQ_EINVAL;
    int rc = check_fill(fill);
    if (rc) return rc;
    if (!d_counts || !d_out || out_stride < 0 || capacity < 0 || (capacity > 0 && !d_islands))
        return DAQ_EINVAL;
    if (capacity == 0 || fill->n_samples == 0) return DAQ_OK;
    DeviceGuard guard(ctx->device);
    GatherArgs g{};
    g.raw = fill->raw;
    g.stride = fill->row_stride;
    g.C = fill->n_channels;
    g.isl = d_islands;
    g.cap = capacity;
    g.counts = d_counts;
    g.out = d_out;
    g.out_stride = out_stride;
    const int64_t most = std::min<int64_t>(fill->n_samples, out_stride);
    int grid = (int)std::min<int64_t>((int64_t)ctx->n_cu * 4, std::max<int64_t>(1, (most + 2047) / 2048));
    HIP_TRY(daqk::launch_gather(g, grid, (hipStream_t)stream));
    return DAQ_OK;
}

int daq_chop_fill(daq_ctx *ctx, const daq_fill *fill, const daq_fill_out *out, void *stream) {
    return run_fused(ctx, fill, out, 1, (hipStream_t)stream, false);
}

namespace {

int check_q_out(const daq_fill &f, const daq_q_out &o) {
    if (o.acc) {
        if (o.acc_stride < f.n_samples || (o.acc_stride % 4) != 0) return DAQ_EINVAL;
        if (!aligned16(o.acc)) return DAQ_EALIGN;
    }
    if (o.qsum && ((uintptr_t)o.qsum & 7u) != 0) return DAQ_EALIGN;
    return DAQ_OK;
}

// Accumulators of one call must not overlap: each fill adds to its own rows.
bool q_acc_overlap(const daq_fill *fills, const daq_q_out *outs, int32_t n) {
    std::vector<std::pair<uintptr_t, uintptr_t>> iv;
    for (int32_t i = 0; i < n; i++) {
        const daq_q_out &o = outs[i];
        if (!o.acc || fills[i].n_samples == 0) continue;
        const uintptr_t lo = (uintptr_t)o.acc;
        const uintptr_t hi = lo + (uintptr_t)(((int64_t)fills[i].n_channels - 1) * o.acc_stride +
                                               fills[i].n_samples) * sizeof(int32_t);
        iv.emplace_back(lo, hi);
    }
    std::sort(iv.begin(), iv.end());
    for (size_t k = 1; k < iv.size(); k++)
        if (iv[k].first < iv[k - 1].second) return true;
    return false;
}

// The Q-method over n fills: k_prepare (pedestals, thr = 0 so the effective
// threshold is the pedestal sum), then k_q_pass over tiles of 8 x threads
// samples. Plain launches; the descriptors go through the staging ring.
int run_qmethod(daq_ctx *ctx, const daq_fill *fills, const daq_q_out *outs, int32_t n, hipStream_t stream) {
    if (!ctx || n < 0 || (n > 0 && (!fills || !outs))) return DAQ_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        int rc = check_fill(&fills[i]);
        if (rc) return rc;
        rc = check_q_out(fills[i], outs[i]);
        if (rc) return rc;
    }
    if (q_acc_overlap(fills, outs, n)) return DAQ_EINVAL;
    if (n == 0) return DAQ_OK;
    DeviceGuard guard(ctx->device);
    const int threads = ctx->sched.threads == 512 ? 512 : 256;
    const int64_t T = (int64_t)threads * daqk::kVec;  // samples per tile, no halo
    int64_t total = 0, raw_bytes = 0, ped_need = 0;
    std::vector<int64_t> base((size_t)n), poff((size_t)n, -1);
    for (int32_t i = 0; i < n; i++) {
        base[(size_t)i] = total;
        total += (fills[i].n_samples + T - 1) / T;
        raw_bytes += 2 * (int64_t)fills[i].n_channels * fills[i].n_samples;
        if (!outs[i].ped) {
            poff[(size_t)i] = ped_need;
            ped_need += fills[i].n_channels;
        }
    }
    Scratch *s = scratch_for(ctx, stream);
    int rc = ensure_scratch(s, std::max<int64_t>(total, n), n, 0);
    if (rc) return rc;
    if (ped_need > s->q_ped_cap) {
        HIP_TRY(hipStreamSynchronize(stream));
        (void)hipFree(s->q_ped);
        s->q_ped = nullptr;
        s->q_ped_cap = 0;
        const int64_t cap = std::max<int64_t>(ped_need + ped_need / 2, 4096);
        HIP_TRY(hipMalloc(&s->q_ped, (size_t)cap * sizeof(int32_t)));
        s->q_ped_cap = cap;
    }
    auto desc = [&](int32_t i) {
        const daq_fill &f = fills[i];
        const daq_q_out &o = outs[i];
        FillDev d{};
        d.raw = f.raw;
        d.n = f.n_samples;
        d.stride = f.row_stride;
        d.C = f.n_channels;
        d.np = f.ped_samples;
        d.tout = T;
        d.tile_base = base[(size_t)i];
        d.n_tiles = (f.n_samples + T - 1) / T;
        d.ped = o.ped ? o.ped : s->q_ped + poff[(size_t)i];
        d.qsum = o.qsum;
        d.acc = o.acc;
        d.acc_stride = o.acc ? o.acc_stride : 0;
        return d;
    };
    KArgs a{};
    a.tile_state = s->tile_state;
    a.ticket = s->ticket;
    a.thr_eff = s->thr_eff;
    a.tile_pref = s->tile_pref;
    a.n_fills = n;
    a.total_tiles = total;
    a.stream_loads = raw_bytes > kStreamLoadBytes ? 1 : 0;
    if (n == 1) {
        a.one = desc(0);
    } else {
        const int rs = s->ring_pos;
        s->ring_pos = (s->ring_pos + 1) % kRing;
        if (s->ring_used[rs]) HIP_TRY(hipEventSynchronize(s->ring_ev[rs]));
        BatchHdr *h = reinterpret_cast<BatchHdr *>(s->ring_host[rs]);
        FillDev *tab = reinterpret_cast<FillDev *>(h + 1);
        h->n_fills = n;
        h->stream_loads = a.stream_loads;
        h->total_tiles = total;
        h->copy_slots = 0;
        h->pad2 = 0;
        for (int32_t i = 0; i < n; i++) tab[i] = desc(i);
        const size_t bytes = sizeof(BatchHdr) + (size_t)n * sizeof(FillDev);
        const uint8_t *img = reinterpret_cast<const uint8_t *>(h);
        if (s->last_desc.size() != bytes || std::memcmp(s->last_desc.data(), img, bytes) != 0) {
            HIP_TRY(hipMemcpyAsync(s->hdr, h, bytes, hipMemcpyHostToDevice, stream));
            HIP_TRY(hipEventRecord(s->ring_ev[rs], stream));
            s->ring_used[rs] = true;
            s->last_desc.assign(img, img + bytes);
        }
        a.table = s->table;
        a.hdr = s->hdr;
    }
    int prep_blocks = (int)std::min<int64_t>(kPrepareBlocks, std::max<int64_t>(1, (total + 2047) / 2048));
    prep_blocks = std::max(prep_blocks, std::min(n, kPrepareBlocks));
    prep_blocks = std::min(prep_blocks, std::max(n, 64));
    HIP_TRY(daqk::launch_prepare(a, prep_blocks, stream));
    if (total == 0) return DAQ_OK;
    const int wgs = ctx->sched.wgs_per_cu > 0 ? ctx->sched.wgs_per_cu : 8;
    const int grid = (int)std::min<int64_t>((int64_t)wgs * ctx->n_cu, total);
    size_t slot = 0;
    if (ctx->timing) {
        rc = timing_begin(ctx, stream, &slot);
        if (rc) return rc;
    }
    HIP_TRY(daqk::launch_q(a, threads, grid, stream));
    if (ctx->timing) return timing_end(ctx, stream, slot);
    return DAQ_OK;
}

}  // namespace

int64_t daq_packed12_stride(int64_t n_samples) {
    if (n_samples < 0) return -1;
    return ((3 * n_samples + 1) / 2 + 3) / 4 * 4;
}

int daq_unpack12(daq_ctx *ctx, const uint8_t *d_packed, int64_t packed_stride, int32_t n_channels,
                 int64_t n_samples, int16_t *d_raw, int64_t row_stride, void *stream) {
    if (!ctx || n_channels < 1 || n_samples < 0) return DAQ_EINVAL;
    if (n_samples > DAQ_MAX_SAMPLES || n_channels > DAQ_MAX_CHANNELS) return DAQ_ERANGE;
    if (n_samples == 0) return DAQ_OK;
    if (!d_packed || !d_raw || packed_stride < (3 * n_samples + 1) / 2 || row_stride < n_samples)
        return DAQ_EINVAL;
    if (((uintptr_t)d_packed & 3u) != 0 || (packed_stride % 4) != 0 || !aligned16(d_raw) ||
        (row_stride % daqk::kVec) != 0)
        return DAQ_EALIGN;
    DeviceGuard guard(ctx->device);
    const int64_t items = (n_samples + daqk::kVec - 1) / daqk::kVec * n_channels;
    const int64_t grid = std::min<int64_t>((items + 255) / 256, (int64_t)16 * ctx->n_cu);
    HIP_TRY(daqk::launch_unpack12(d_packed, packed_stride, n_channels, n_samples, d_raw, row_stride,
                                  (int)std::max<int64_t>(grid, 1), (hipStream_t)stream));
    return DAQ_OK;
}

namespace {

bool aligned_to(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

// Block groups (8 blocks of one row) of a fill whose rows hold max_len samples.
int64_t z_groups(const daq_z_fill &z) {
    const int64_t nb = (z.max_len + DAQ_Z_BLOCK - 1) / DAQ_Z_BLOCK;
    return (nb + 7) / 8 * z.n_channels;
}

int check_z_fill(const daq_z_fill &z) {
    if (!z.packed || !z.counts || !z.hdr || !z.n_words || z.stride < 0 || z.max_len < 0 || z.words_cap < 0 ||
        z.n_channels < 1 || z.reserved != 0 || (z.words_cap > 0 && !z.words))
        return DAQ_EINVAL;
    if (z.n_channels > DAQ_MAX_CHANNELS || z.max_len > DAQ_MAX_SAMPLES) return DAQ_ERANGE;
    if (z.stride < z.max_len) return DAQ_EINVAL;
    if (!aligned16(z.packed) || (z.stride % daqk::kVec) != 0) return DAQ_EALIGN;
    if (!aligned_to(z.counts, 8) || !aligned_to(z.hdr, 4) || !aligned_to(z.offsets, 8) ||
        !aligned_to(z.words, 4) || !aligned_to(z.n_words, 8))
        return DAQ_EALIGN;
    return DAQ_OK;
}

}  // namespace

#ifndef DAQ_Z_WGS_PER_CU
#define DAQ_Z_WGS_PER_CU 8  // compression work-groups per CU, shared by the launch's fills
#endif

int daq_compress_batch(daq_ctx *ctx, const daq_z_fill *fills, int32_t n, void *stream_) {
    if (!ctx || n < 0 || (n > 0 && !fills)) return DAQ_EINVAL;
    if (n == 0) return DAQ_OK;
    const hipStream_t stream = (hipStream_t)stream_;
    for (int32_t i = 0; i < n; i++) {
        const int rc = check_z_fill(fills[i]);
        if (rc) return rc;
    }
    // Work-groups per fill of each launch: the resident count (8 per CU)
    // shared by its fills, at most kZMaxGrid, fewer for short streams.
    auto grid_of = [&](int32_t i0, int32_t m) {
        int64_t most = 1;
        for (int32_t j = 0; j < m; j++) most = std::max(most, z_groups(fills[i0 + j]));
        const int64_t wide =
            std::min<int64_t>(daqk::kZMaxGrid, std::max<int64_t>(1, (int64_t)DAQ_Z_WGS_PER_CU * ctx->n_cu / m));
        return (int)std::max<int64_t>(1, std::min<int64_t>(wide, (most + daqk::kZWaves - 1) / daqk::kZWaves));
    };
    int64_t need = 0;  // one word per wave of a launch (launches run in stream order)
    for (int32_t i0 = 0; i0 < n; i0 += daqk::kZMaxFills) {
        const int32_t m = std::min<int32_t>(n - i0, daqk::kZMaxFills);
        need = std::max<int64_t>(need, (int64_t)m * grid_of(i0, m) * daqk::kZWaves);
    }
    DeviceGuard guard(ctx->device);
    Scratch *s = scratch_for(ctx, stream);
    if (need > s->z_gofs_cap) {
        HIP_TRY(hipStreamSynchronize(stream));
        (void)hipFree(s->z_gofs);
        s->z_gofs = nullptr;
        s->z_gofs_cap = 0;
        const int64_t cap = std::max<int64_t>(need, 4096);
        HIP_TRY(hipMalloc(&s->z_gofs, (size_t)cap * sizeof(int64_t)));
        s->z_gofs_cap = cap;
    }
    size_t slot = 0;
    if (ctx->timing) {
        const int rc = timing_begin(ctx, stream, &slot);
        if (rc) return rc;
    }
    for (int32_t i0 = 0; i0 < n; i0 += daqk::kZMaxFills) {
        daqk::ZArgs a{};
        a.n = std::min<int32_t>(n - i0, daqk::kZMaxFills);
        const int grid = grid_of(i0, a.n);
        for (int32_t j = 0; j < a.n; j++) {
            const daq_z_fill &z = fills[i0 + j];
            daqk::ZFillDev &d = a.f[j];
            d.packed = z.packed;
            d.stride = z.stride;
            d.counts = z.counts;
            d.max_len = z.max_len;
            d.hdr = z.hdr;
            d.offsets = z.offsets;
            d.gofs = s->z_gofs + (int64_t)j * grid * daqk::kZWaves;
            d.words = z.words;
            d.cap = z.words_cap;
            d.n_words = z.n_words;
            d.C = z.n_channels;
        }
        HIP_TRY(daqk::launch_z(a, grid, stream));
    }
    if (ctx->timing) return timing_end(ctx, stream, slot);
    return DAQ_OK;
}

#ifndef DAQ_UNZ_WGS_PER_CU
#define DAQ_UNZ_WGS_PER_CU 32  // decoding work-groups per CU, shared by the launch's streams (latency-bound: more in flight)
#endif

int daq_decompress_batch(daq_ctx *ctx, const daq_z_stream *streams, int32_t n, void *stream_) {
    if (!ctx || n < 0 || (n > 0 && !streams)) return DAQ_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        const daq_z_stream &z = streams[i];
        if (!z.hdr || !z.offsets || !z.out || z.n_samples < 0 || z.n_words < 0 || z.n_channels < 1 ||
            z.reserved != 0 || (z.n_words > 0 && !z.words) || z.out_stride < z.n_samples)
            return DAQ_EINVAL;
        if (z.n_channels > DAQ_MAX_CHANNELS || z.n_samples > DAQ_MAX_SAMPLES) return DAQ_ERANGE;
        if (!aligned16(z.out) || (z.out_stride % daqk::kVec) != 0 || !aligned_to(z.hdr, 4) ||
            !aligned_to(z.offsets, 8) || !aligned_to(z.words, 4))
            return DAQ_EALIGN;
    }
    if (n == 0) return DAQ_OK;
    DeviceGuard guard(ctx->device);
    for (int32_t i0 = 0; i0 < n; i0 += daqk::kZMaxFills) {
        daqk::ZDecArgs a{};
        a.n = std::min<int32_t>(n - i0, daqk::kZMaxFills);
        int64_t most = 1;
        for (int32_t j = 0; j < a.n; j++) {
            const daq_z_stream &z = streams[i0 + j];
            daqk::ZStreamDev &d = a.f[j];
            d.hdr = z.hdr;
            d.offsets = z.offsets;
            d.words = z.words;
            d.n_words = z.n_words;
            d.out = z.out;
            d.out_stride = z.out_stride;
            d.L = z.n_samples;
            d.C = z.n_channels;
            const int64_t nb = (z.n_samples + DAQ_Z_BLOCK - 1) / DAQ_Z_BLOCK;
            most = std::max<int64_t>(most, (nb + 7) / 8 * z.n_channels);
        }
        const int64_t wide = std::max<int64_t>(1, (int64_t)DAQ_UNZ_WGS_PER_CU * ctx->n_cu / a.n);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wide, (most + daqk::kZWaves - 1) / daqk::kZWaves));
        HIP_TRY(daqk::launch_unz(a, grid, (hipStream_t)stream_));
    }
    return DAQ_OK;
}

int daq_qmethod_batch(daq_ctx *ctx, const daq_fill *fills, const daq_q_out *outs, int32_t n, void *stream) {
    return run_qmethod(ctx, fills, outs, n, (hipStream_t)stream);
}

int daq_process_batch(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs, int32_t n,
                      void *stream) {
    return run_fused(ctx, fills, outs, n, (hipStream_t)stream, true);
}

int64_t daq_noalloc_scratch_bytes(const daq_fill *fills, int32_t n) {
    if (n < 0 || (n > 0 && !fills)) return DAQ_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        const int rc = check_fill(&fills[i]);
        if (rc) return rc;
    }
    int64_t most = 0;
    for (int threads : {256, 512})
        most = std::max(most, noalloc_layout(fills, n, daq_schedule{threads, 16, daqk::kVariantSplit, 0}).bytes);
    return most;
}

int daq_process_batch_noalloc(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs, int32_t n,
                              void *stream_) {
    if (!ctx || n < 0 || (n > 0 && (!fills || !outs))) return DAQ_EINVAL;
    for (int32_t i = 0; i < n; i++) {
        int rc = check_fill(&fills[i]);
        if (rc) return rc;
        rc = check_out(&outs[i]);
        if (rc) return rc;
    }
    if (n == 0) return DAQ_OK;
    const daq_schedule sc = noalloc_schedule(ctx);
    const NoAllocLayout L = noalloc_layout(fills, n, sc);
    if (L.bytes > DAQ_NOALLOC_SCRATCH_BYTES) return DAQ_ERANGE;
    DeviceGuard guard(ctx->device);
    uint8_t *base = noalloc_ptr(ctx->device);
    if (!base) return DAQ_EINVAL;
    const hipStream_t stream = (hipStream_t)stream_;
    int64_t raw_bytes = 0;
    for (int32_t i = 0; i < n; i++) raw_bytes += 2 * (int64_t)fills[i].n_channels * fills[i].n_samples;
    BatchHdr *d_hdr = reinterpret_cast<BatchHdr *>(base + L.hdr);
    FillDev *d_table = reinterpret_cast<FillDev *>(d_hdr + 1);
    KArgs a{};
    a.table = d_table;
    a.hdr = d_hdr;
    a.tile_state = reinterpret_cast<uint64_t *>(base + L.tile_state);
    a.ticket = reinterpret_cast<uint32_t *>(base + L.ticket);
    a.thr_eff = reinterpret_cast<int64_t *>(base + L.thr_eff);
    a.tile_pref = reinterpret_cast<uint64_t *>(base + L.tile_pref);
    a.n_fills = n;
    a.total_tiles = L.total_tiles;
    a.stream_loads = raw_bytes > kStreamLoadBytes ? 1 : 0;
    a.copy_slots = L.max_chunks * n;
    a.part = 0;
    a.parts = 1;
    // descriptors, kPutFills per launch; the header with the first group
    PutDescArgs put{};
    put.hdr.n_fills = n;
    put.hdr.stream_loads = a.stream_loads;
    put.hdr.total_tiles = L.total_tiles;
    put.hdr.copy_slots = a.copy_slots;
    put.dst_hdr = d_hdr;
    int64_t tile_base = 0, foff = L.fills;
    for (int32_t i0 = 0; i0 < n; i0 += kPutFills) {
        put.count = std::min<int32_t>(kPutFills, n - i0);
        put.write_hdr = i0 == 0 ? 1 : 0;
        put.dst = d_table + i0;
        for (int32_t k = 0; k < put.count; k++) {
            const daq_fill &f = fills[i0 + k];
            const SplitLayout sl = split_layout_of(f, sc);
            FillDev d = make_desc(f, outs[i0 + k], tile_base, sc);
            d.mbits = base + foff + daqk::kMaskGuard;
            d.runs = reinterpret_cast<int32_t *>(base + foff + sl.runs);
            d.cmap = reinterpret_cast<int32_t *>(base + foff + sl.cmap);
            put.d[k] = d;
            tile_base += d.n_tiles;
            foff += up16(sl.bytes);
        }
        hipLaunchKernelGGL(k_put_descs, dim3(1), dim3(kPutFills * sizeof(FillDev) / 16), 0, stream, put);
        HIP_TRY(hipGetLastError());
    }
    if (L.total_tiles == 0) {  // only counts and pedestals to clear
        HIP_TRY(daqk::launch_prepare(a, prepare_blocks(a, 0), stream));
        return DAQ_OK;
    }
    const int grid = chop_grid(ctx, sc, L.total_tiles);
    HIP_TRY(daqk::launch_scan(a, sc.threads, grid, stream));
    HIP_TRY(daqk::launch_emit(a, sc.threads, edge_grid(grid, L.total_tiles, sc.threads),
                              daqk::kCopyWgsPerCu * ctx->n_cu, stream));
    return DAQ_OK;
}

int daq_process_batch_q(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs, const daq_q_out *qouts,
                        int32_t n, void *stream) {
    if (n > 0 && !qouts) return DAQ_EINVAL;
    return run_fused(ctx, fills, outs, n, (hipStream_t)stream, true, qouts);
}

int daq_ctx_set_schedule(daq_ctx *ctx, const daq_schedule *s) {
    if (!ctx || !s) return DAQ_EINVAL;
    if ((s->threads != 128 && s->threads != 256 && s->threads != 512) || s->wgs_per_cu < 0 || s->wgs_per_cu > 16 ||
        s->variant < daqk::kVariantReload || s->variant > daqk::kVariantLast || s->parts < 0 ||
        s->parts > daqk::kMaxParts || (s->parts > 1 && s->variant != daqk::kVariantSplit))
        return DAQ_EINVAL;
    if (s->variant == daqk::kVariantStream && s->threads != daqk::kStreamThreads) return DAQ_EINVAL;
    if ((s->variant == daqk::kVariantSplit || s->variant == daqk::kVariantPipe) && s->threads == 128)
        return DAQ_EINVAL;
    ctx->sched = *s;
    return DAQ_OK;
}

int daq_ctx_get_schedule(daq_ctx *ctx, daq_schedule *s) {
    if (!ctx || !s) return DAQ_EINVAL;
    *s = ctx->sched;
    return DAQ_OK;
}

int daq_ctx_set_graphs(daq_ctx *ctx, int enable) {
    if (!ctx) return DAQ_EINVAL;
    ctx->graphs = enable != 0;
    return DAQ_OK;
}

int daq_ctx_get_graphs(daq_ctx *ctx, int *enable) {
    if (!ctx || !enable) return DAQ_EINVAL;
    *enable = ctx->graphs ? 1 : 0;
    return DAQ_OK;
}

int daq_ctx_set_timing(daq_ctx *ctx, int enable) {
    if (!ctx) return DAQ_EINVAL;
    ctx->timing = enable != 0;
    ctx->t_read = ctx->t_next;
    return DAQ_OK;
}

int daq_ctx_kernel_times(daq_ctx *ctx, float *ms, int32_t max) {
    if (!ctx || max < 0 || (max > 0 && !ms)) return DAQ_EINVAL;
    DeviceGuard guard(ctx->device);
    int32_t n = 0;
    while (ctx->t_read < ctx->t_next && n < max) {
        const size_t i = (size_t)(ctx->t_read % kMaxTimed);
        HIP_TRY(hipEventSynchronize(ctx->ev_stop[i]));
        HIP_TRY(hipEventElapsedTime(&ms[n], ctx->ev_start[i], ctx->ev_stop[i]));
        n++;
        ctx->t_read++;
    }
    return n;
}

int daq_ctx_kernel_time(daq_ctx *ctx, float *ms) {
    if (!ctx || !ms) return DAQ_EINVAL;
    if (ctx->t_next == 0 || ctx->t_read >= ctx->t_next) return DAQ_EINVAL;
    DeviceGuard guard(ctx->device);
    const size_t i = (size_t)((ctx->t_next - 1) % kMaxTimed);
    HIP_TRY(hipEventSynchronize(ctx->ev_stop[i]));
    HIP_TRY(hipEventElapsedTime(ms, ctx->ev_start[i], ctx->ev_stop[i]));
    ctx->t_read = ctx->t_next;
    return DAQ_OK;
}

int daq_autotune(daq_ctx *ctx, const daq_fill *fills, const daq_fill_out *outs, int32_t n, void *stream,
                 const char *cache_path, daq_schedule *best) {
    if (!ctx || n <= 0 || !fills || !outs) return DAQ_EINVAL;
    if (ctx->pinned) {
        daqlog::say(2, "autotune: schedule %d/%d/%d/%d fixed by DAQ_SCHEDULE, not tuned", ctx->sched.threads,
                    ctx->sched.wgs_per_cu, ctx->sched.variant, ctx->sched.parts);
        if (best) *best = ctx->sched;
        return DAQ_OK;
    }
    hipStream_t st = (hipStream_t)stream;
    const std::string key = shape_key(ctx, fills, n);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find('|');
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            daq_schedule s{};
            float ms = 0.f;
            int graphs = 1;
            const int got = sscanf(line.c_str() + bar + 1, "%d %d %d %d %f %d", &s.threads, &s.wgs_per_cu, &s.variant,
                                   &s.parts, &ms, &graphs);
            if (got >= 4 && daq_ctx_set_schedule(ctx, &s) == DAQ_OK) {
                if (got == 6) ctx->graphs = graphs != 0;
                daqlog::say(2, "autotune: schedule %d/%d/%d/%d (graphs %d) from %s", s.threads, s.wgs_per_cu,
                            s.variant, s.parts, ctx->graphs ? 1 : 0, cache_path);
                if (best) *best = s;
                return DAQ_OK;
            }
        }
    }
    std::vector<daq_schedule> cand;
    const bool calo = all_calorimeters(fills, n);
    const int V0 = daqk::kVariantReload, V1 = daqk::kVariantResident, V2 = daqk::kVariantStream;
    const int V3 = daqk::kVariantReload18, V4 = daqk::kVariantReload27, V5 = daqk::kVariantSplit;
    // the library's default first: it is the reference every other candidate
    // is compared with. The persistent variant is not on the menu (it never
    // won, and its bounded waits may give up); daq_ctx_set_schedule selects it.
    const daq_schedule menu[] = {{512, 8, V5, 0},  {256, 16, V5, 0}, {512, 4, V5, 0},  {512, 8, V5, 2},
                                 {256, 16, V5, 2}, {256, 16, V5, 3}, {256, 16, V5, 4},
                                 {256, 8, V5, 0},  {256, 8, V5, 2},  {256, 4, V0, 0},
                                 {256, 8, V0, 0},  {512, 2, V0, 0},  {256, 2, V2, 0},  {256, 4, V3, 0},
                                 {256, 3, V4, 0},  {128, 8, V0, 0},  {256, 1, V1, 0}};
    for (const daq_schedule &m : menu)
        if (((m.variant != V1 && m.variant != V2) || calo) && (m.parts <= 1 || n >= 2 * m.parts)) cand.push_back(m);
    const daq_schedule saved = ctx->sched;
    const bool saved_timing = ctx->timing;
    ctx->timing = true;
    DeviceGuard guard(ctx->device);
    RefCopy ref;
    float best_ms = 1e30f;
    daq_schedule best_s = saved;
    int rc = DAQ_OK;
    for (size_t k = 0; k < cand.size() && rc == DAQ_OK; k++) {
        ctx->sched = cand[k];
        // the descriptor table is staged by the first run; poison through it
        // once it exists, then run again from poisoned outputs
        rc = run_fused(ctx, fills, outs, n, st, true);  // warm-up (and capture)
        if (rc) break;
        Scratch *s = scratch_for(ctx, st);
        rc = poison_outputs(s, n, st);
        if (!rc) rc = run_fused(ctx, fills, outs, n, st, true);
        if (!rc) {
            float ms0 = 0.f;  // untimed: discard the two runs' timings
            rc = daq_ctx_kernel_time(ctx, &ms0);
        }
        if (rc) break;
        if (k == 0) {
            rc = snapshot_outputs(fills, outs, n, st, ref);
            if (rc) break;
        } else {
            bool same = false;
            rc = compare_outputs(s, n, st, ref, &same);
            if (rc) break;
            if (!same) {
                daqlog::say(1, "autotune: schedule %d/%d/%d/%d wrote outputs that differ from %d/%d/%d/%d's",
                            cand[k].threads, cand[k].wgs_per_cu, cand[k].variant, cand[k].parts, cand[0].threads,
                            cand[0].wgs_per_cu, cand[0].variant, cand[0].parts);
                rc = DAQ_EMISMATCH;
                break;
            }
        }
        // the median of ten timed launches (differences between the best
        // schedules are a few percent)
        constexpr int reps = 10;
        float t[reps];
        for (int r = 0; r < reps && rc == DAQ_OK; r++) {
            rc = run_fused(ctx, fills, outs, n, st, true);
            t[r] = 0.f;
            if (!rc) rc = daq_ctx_kernel_time(ctx, &t[r]);
        }
        if (rc) break;
        std::sort(t, t + reps);
        const float med = 0.5f * (t[reps / 2 - 1] + t[reps / 2]);
        daqlog::say(2, "autotune: schedule %d/%d/%d/%d median %.4f ms", cand[k].threads, cand[k].wgs_per_cu,
                    cand[k].variant, cand[k].parts, med);
        if (med < best_ms) {
            best_ms = med;
            best_s = cand[k];
        }
    }
    // the winner replayed from its captured graph against plain launches of
    // the same kernels (graph replay costs a few microseconds per launch on
    // some runtimes): the context keeps the faster mode
    const bool saved_graphs = ctx->graphs;
    float mode_ms[2] = {best_ms, best_ms};
    if (!rc) {
        ctx->sched = best_s;
        for (int g = 0; g < 2 && rc == DAQ_OK; g++) {
            ctx->graphs = g == 1;
            constexpr int reps = 10;
            float t[reps];
            rc = run_fused(ctx, fills, outs, n, st, true);  // warm-up (and capture)
            if (!rc) rc = daq_ctx_kernel_time(ctx, &t[0]);
            for (int r = 0; r < reps && rc == DAQ_OK; r++) {
                rc = run_fused(ctx, fills, outs, n, st, true);
                t[r] = 0.f;
                if (!rc) rc = daq_ctx_kernel_time(ctx, &t[r]);
            }
            if (rc) break;
            std::sort(t, t + reps);
            mode_ms[g] = 0.5f * (t[reps / 2 - 1] + t[reps / 2]);
        }
    }
    ctx->timing = saved_timing;
    ctx->t_read = ctx->t_next;
    if (rc) {
        ctx->sched = saved;
        ctx->graphs = saved_graphs;
        return rc;
    }
    ctx->sched = best_s;
    ctx->graphs = mode_ms[1] <= mode_ms[0];
    daqlog::say(2, "autotune: kept %d/%d/%d/%d with %s (plain launches %.4f ms, graph replay %.4f ms)",
                best_s.threads, best_s.wgs_per_cu, best_s.variant, best_s.parts,
                ctx->graphs ? "graph replay" : "plain launches", mode_ms[0], mode_ms[1]);
    if (best) *best = best_s;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << "|" << best_s.threads << " " << best_s.wgs_per_cu << " " << best_s.variant << " "
          << best_s.parts << " " << (ctx->graphs ? mode_ms[1] : mode_ms[0]) << " " << (ctx->graphs ? 1 : 0) << "\n";
    }
    return DAQ_OK;
}

}  // extern "C"
