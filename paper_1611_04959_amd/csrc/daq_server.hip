// daq_server.hip -- the serving loop of libdaqisland (include/daq.h).
//
// Admission by HBM budget: every submitted fill gets a slot in the caller's
// device arena (daqk::Arena does the bookkeeping) or is refused with
// DAQ_EAGAIN. Continuous batching: n_streams worker threads each own a HIP
// stream and a private context; a free worker takes all queued fills (up to
// max_batch, oldest first) and launches them as one batch, so fills that
// arrive while other batches run are launched on another stream and overlap
// with them on the device. A worker waits for its own batch, copies the
// per-fill counts to the host in one transfer and publishes completions.
//
// Deadtime accounting (the abstract asks for deadtime-free records): a
// fill's arrival time (given with daq_submit_fill_at by callers that retry
// after DAQ_EAGAIN) starts its latency; fills admitted later than the
// admission deadline count as late, and the time from a refused submit to the
// next admission adds to the server's deadtime. A watchdog bounds each
// worker's wait for its batch: past the batch time-out the batch's fills
// complete with DAQ_ETIMEDOUT and the worker goes on, while their slots stay
// held until the device has finished with them.
//
// Built on the public calls of the library only (daq_process_batch and the
// context calls); the server adds host threads, the arena and one small
// kernel that collects the counts of a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>
#include "arena.h"
#include "daq.h"
#include "daq_log.h"

namespace {

constexpr int kMaxStreams = 8;
constexpr int kMaxBatch = 256;
constexpr uint64_t kAlign = daqk::Arena::kAlign;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint64_t up(uint64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Parts of one slot, as byte offsets from the slot's start.
struct SlotLayout {
    uint64_t counts = 0, ped = 0, islands = 0, out = 0, raw = 0, packed = 0, bytes = 0;
    int64_t capacity = 0, out_stride = 0;
};

int check_submit_fill(const daq_fill *f, int32_t flags) {
    if (!f || f->reserved != 0) return DAQ_EINVAL;
    if (flags & ~(DAQ_SUBMIT_HOST_RAW | DAQ_SUBMIT_HOST_PACKED12)) return DAQ_EINVAL;
    if ((flags & DAQ_SUBMIT_HOST_RAW) && (flags & DAQ_SUBMIT_HOST_PACKED12)) return DAQ_EINVAL;
    if (f->n_samples < 0 || f->row_stride < f->n_samples) return DAQ_EINVAL;
    if (f->n_samples > DAQ_MAX_SAMPLES) return DAQ_ERANGE;
    if (f->n_channels < 1 || f->ped_samples < 1 || f->pre < 0 || f->post < 0) return DAQ_EINVAL;
    if (f->n_channels > DAQ_MAX_CHANNELS || f->pre > DAQ_MAX_WINDOW || f->post > DAQ_MAX_WINDOW)
        return DAQ_ERANGE;
    if (f->row_stride > DAQ_MAX_SAMPLES + 8) return DAQ_ERANGE;
    if (f->n_samples > 0 && !f->raw) return DAQ_EINVAL;
    if (f->row_stride % 8 != 0) return DAQ_EALIGN;
    if (!(flags & (DAQ_SUBMIT_HOST_RAW | DAQ_SUBMIT_HOST_PACKED12)) && ((uintptr_t)f->raw & 15u) != 0)
        return DAQ_EALIGN;
    return DAQ_OK;
}

SlotLayout layout_of(const daq_fill &f, int32_t flags) {
    SlotLayout L;
    const uint64_t C = (uint64_t)f.n_channels;
    L.capacity = daq_max_islands(f.n_samples, f.pre, f.post);
    L.out_stride = (f.n_samples + 7) / 8 * 8;
    uint64_t o = 0;
    L.counts = o;
    o += up(sizeof(daq_counts));
    L.ped = o;
    o += up(C * sizeof(int32_t));
    L.islands = o;
    o += up((uint64_t)L.capacity * sizeof(daq_island));
    L.out = o;
    o += up(C * (uint64_t)L.out_stride * sizeof(int16_t));
    L.raw = o;
    if (flags & (DAQ_SUBMIT_HOST_RAW | DAQ_SUBMIT_HOST_PACKED12)) o += up(C * (uint64_t)f.row_stride * sizeof(int16_t));
    L.packed = o;
    if (flags & DAQ_SUBMIT_HOST_PACKED12) o += up(C * (uint64_t)daq_packed12_stride(f.n_samples));
    L.bytes = o;
    return L;
}

static_assert(sizeof(daq_completion) == 128, "daq_completion layout");
static_assert(sizeof(daq_server_stats) == 104, "daq_server_stats layout");

// Gathers the counts of a batch into one array (one copy to the host).
struct CountPtrs {
    const daq_counts *p[kMaxBatch];
};

__global__ void k_collect_counts(CountPtrs ptrs, int n, daq_counts *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = *ptrs.p[i];
}

// kHeld: completed with DAQ_ETIMEDOUT while the device may still use the slot.
enum class State { kQueued, kRunning, kDone, kHeld };

struct Job {
    uint64_t ticket = 0, tag = 0;
    int32_t flags = 0;
    daq_fill fill{};        // raw: device rows the kernels read
    const int16_t *host_raw = nullptr;
    const uint8_t *host_packed = nullptr;  // 12-bit words, rows daq_packed12_stride(N) bytes apart
    uint8_t *dev_packed = nullptr;         // their place in the slot
    daq_fill_out out{};
    uint64_t offset = 0;    // slot offset in the arena
    int64_t t_submit = 0;   // arrival (steady clock)
    State state = State::kQueued;
    bool released = false;  // kHeld: released by the caller, slot freed when the device is done
};

struct Worker {
    std::thread th;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    daq_ctx *ctx = nullptr;
    daq_counts *d_counts = nullptr;  // kMaxBatch, device
    daq_counts *h_counts = nullptr;  // kMaxBatch, pinned host
    std::vector<Job *> held;         // timed-out fills whose launches may still run
};

}  // namespace

struct daq_server {
    int device = 0;
    daq_schedule sched{};
    uint8_t *arena_base = nullptr;
    int32_t max_batch = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    daqk::Arena arena;
    std::deque<Job *> queue;                       // admitted, not launched
    std::deque<daq_completion> done;               // finished, not polled
    std::unordered_map<uint64_t, Job *> jobs;      // every unreleased fill
    uint64_t next_ticket = 1;
    bool stop = false;
    int32_t running = 0;
    daq_server_stats stats{};
    std::vector<Worker> workers;
    std::atomic<int64_t> admit_deadline_ns{10'000'000};  // 10 ms: fill spacing in a burst
    std::atomic<int64_t> batch_timeout_ns{10'000'000'000};
    int64_t dead_since = -1;  // first refused submit of the current dead period, or -1
};

namespace {

// Waits for `ev` at most limit_ns (yielding for the first 2 ms, then
// sleeping 50 us between polls); *timed_out when it did not complete.
hipError_t wait_event(hipEvent_t ev, int64_t limit_ns, bool *timed_out) {
    const int64_t t0 = now_ns();
    *timed_out = false;
    for (;;) {
        const hipError_t q = hipEventQuery(ev);
        if (q != hipErrorNotReady) return q;
        const int64_t dt = now_ns() - t0;
        if (dt >= limit_ns) {
            *timed_out = true;
            return hipSuccess;
        }
        if (dt < 2'000'000) std::this_thread::yield();
        else std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

// With srv->mu held: once the worker's last launch has finished, its held
// (timed-out) fills are done with: released ones give their slots back, the
// others become ordinary finished fills.
void reclaim_held(daq_server *srv, Worker *w) {
    if (w->held.empty() || hipEventQuery(w->done) != hipSuccess) return;
    for (Job *j : w->held) {
        if (j->released) {
            srv->arena.release(j->offset);
            srv->jobs.erase(j->ticket);
            delete j;
        } else {
            j->state = State::kDone;
        }
    }
    w->held.clear();
}

void worker_loop(daq_server *srv, Worker *w) {
    (void)hipSetDevice(srv->device);
    std::vector<Job *> batch;
    std::vector<daq_fill> fills;
    std::vector<daq_fill_out> outs;
    for (;;) {
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (;;) {
                reclaim_held(srv, w);
                if (srv->stop || !srv->queue.empty()) break;
                if (w->held.empty()) srv->cv_work.wait(lk);
                else srv->cv_work.wait_for(lk, std::chrono::milliseconds(1));
            }
            if (srv->stop) return;
            while (!srv->queue.empty() && (int32_t)batch.size() < srv->max_batch) {
                Job *j = srv->queue.front();
                srv->queue.pop_front();
                j->state = State::kRunning;
                batch.push_back(j);
            }
            srv->running += (int32_t)batch.size();
            srv->stats.batches++;
        }
        const int n = (int)batch.size();
        // profiler ranges (roctx; no cost without a profiler attached): the
        // batch, and inside it the host-fed copies, the launch, the wait and
        // the publication of the completions
        roctxRangePushA("daq_server batch");
        fills.resize((size_t)n);
        outs.resize((size_t)n);
        int rc = DAQ_OK;
        hipError_t he = hipSuccess;
        roctxRangePushA("daq_server ingest");
        for (int i = 0; i < n; i++) {
            Job *j = batch[(size_t)i];
            fills[(size_t)i] = j->fill;
            outs[(size_t)i] = j->out;
            if (j->host_raw && he == hipSuccess) {
                const size_t bytes = (size_t)j->fill.n_channels * (size_t)j->fill.row_stride * sizeof(int16_t);
                he = hipMemcpyAsync(const_cast<int16_t *>(j->fill.raw), j->host_raw, bytes,
                                    hipMemcpyHostToDevice, w->stream);
            }
            if (j->host_packed && he == hipSuccess && j->fill.n_samples > 0) {
                const int64_t pst = daq_packed12_stride(j->fill.n_samples);
                he = hipMemcpyAsync(j->dev_packed, j->host_packed, (size_t)j->fill.n_channels * (size_t)pst,
                                    hipMemcpyHostToDevice, w->stream);
                if (he == hipSuccess &&
                    daq_unpack12(w->ctx, j->dev_packed, pst, j->fill.n_channels, j->fill.n_samples,
                                 const_cast<int16_t *>(j->fill.raw), j->fill.row_stride, w->stream) != DAQ_OK)
                    he = hipErrorUnknown;
            }
        }
        roctxRangePop();
        const int64_t t_launch = now_ns();
        bool timed_out = false;
        roctxRangePushA("daq_server launch");
        if (he == hipSuccess) rc = daq_process_batch(w->ctx, fills.data(), outs.data(), n, w->stream);
        else rc = DAQ_EHIP;
        roctxRangePop();
        roctxRangePushA("daq_server wait");
        if (rc == DAQ_OK) {
            CountPtrs cp{};
            for (int i = 0; i < n; i++) cp.p[i] = outs[(size_t)i].counts;
            hipLaunchKernelGGL(k_collect_counts, dim3(1), dim3(kMaxBatch), 0, w->stream, cp, n, w->d_counts);
            he = hipGetLastError();
            if (he == hipSuccess)
                he = hipMemcpyAsync(w->h_counts, w->d_counts, (size_t)n * sizeof(daq_counts),
                                    hipMemcpyDeviceToHost, w->stream);
            if (he == hipSuccess) he = hipEventRecord(w->done, w->stream);
            if (he == hipSuccess) {
                const int64_t limit = srv->batch_timeout_ns.load(std::memory_order_relaxed);
                if (limit > 0) he = wait_event(w->done, limit, &timed_out);
                else he = hipEventSynchronize(w->done);
                if (timed_out)
                    daqlog::say(1, "server: a batch of %d fills outlived the %lld ns time-out; its slots stay held "
                                   "until the device is done with them", n, (long long)limit);
            }
            if (he != hipSuccess) {
                daqlog::say(1, "server: waiting for a batch of %d fills failed: %s", n, hipGetErrorName(he));
                rc = DAQ_EHIP;
            } else if (timed_out) {
                rc = DAQ_ETIMEDOUT;
            }
        } else {
            daqlog::say(1, "server: a batch of %d fills failed to launch: status %d, HIP error %d", n, rc,
                        (int)he);
            // the copies above may be in flight: wait for the stream before
            // the slots can be handed back
            (void)hipStreamSynchronize(w->stream);
        }
        roctxRangePop();
        const int64_t t_ready = now_ns();
        roctxRangePushA("daq_server publish");
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int i = 0; i < n; i++) {
            Job *j = batch[(size_t)i];
            daq_completion c{};
            c.tag = j->tag;
            c.ticket = j->ticket;
            if (rc == DAQ_OK) c.counts = w->h_counts[i];
            c.out = j->out;
            c.raw = j->fill.raw;
            c.status = rc;
            c.batch_fills = n;
            c.t_submit_ns = j->t_submit;
            c.t_launch_ns = t_launch;
            c.t_ready_ns = t_ready;
            if (timed_out) {
                j->state = State::kHeld;
                w->held.push_back(j);
            } else {
                j->state = State::kDone;
            }
            srv->done.push_back(c);
        }
        srv->running -= n;
        srv->stats.completed += (uint64_t)n;
        if (timed_out) srv->stats.timed_out += (uint64_t)n;
        srv->cv_done.notify_all();
        roctxRangePop();  // publish
        roctxRangePop();  // batch
    }
}

void free_worker(Worker &w) {
    if (w.ctx) daq_ctx_destroy(w.ctx);
    if (w.d_counts) (void)hipFree(w.d_counts);
    if (w.h_counts) (void)hipHostFree(w.h_counts);
    if (w.done) (void)hipEventDestroy(w.done);
    if (w.stream) (void)hipStreamDestroy(w.stream);
    w = Worker{};
}

}  // namespace

extern "C" {

int daq_server_slot_bytes(const daq_fill *fill, int32_t flags, uint64_t *bytes) {
    if (!bytes) return DAQ_EINVAL;
    const int rc = check_submit_fill(fill, flags);
    if (rc) return rc;
    *bytes = layout_of(*fill, flags).bytes;
    return DAQ_OK;
}

int daq_server_create(daq_server **out, daq_ctx *ctx, void *d_arena, size_t arena_bytes, int32_t n_streams,
                      int32_t max_batch) {
    if (!out || !ctx || !d_arena || arena_bytes < kAlign) return DAQ_EINVAL;
    if (((uintptr_t)d_arena % kAlign) != 0) return DAQ_EALIGN;
    if (n_streams < 1 || n_streams > kMaxStreams || max_batch < 1 || max_batch > kMaxBatch) return DAQ_EINVAL;
    *out = nullptr;
    daq_server *srv = new daq_server();
    int dev = 0;
    hipError_t he = hipSuccess;
    int graphs = 1;
    int rc = daq_ctx_get_device(ctx, &dev);
    if (rc == DAQ_OK) rc = daq_ctx_get_schedule(ctx, &srv->sched);
    if (rc == DAQ_OK) rc = daq_ctx_get_graphs(ctx, &graphs);
    if (rc == DAQ_OK && (he = hipSetDevice(dev)) != hipSuccess) rc = DAQ_EHIP;
    srv->device = dev;
    srv->arena_base = static_cast<uint8_t *>(d_arena);
    srv->arena.reset(arena_bytes);
    srv->max_batch = max_batch;
    srv->stats.arena_bytes = srv->arena.size();
    srv->workers.resize((size_t)n_streams);
    for (int i = 0; rc == DAQ_OK && i < n_streams; i++) {
        Worker &w = srv->workers[(size_t)i];
        rc = daq_ctx_create(&w.ctx, dev);
        if (rc == DAQ_OK) rc = daq_ctx_set_schedule(w.ctx, &srv->sched);
        if (rc == DAQ_OK) rc = daq_ctx_set_graphs(w.ctx, graphs);
        if (rc == DAQ_OK && (he = hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking)) != hipSuccess)
            rc = DAQ_EHIP;
        if (rc == DAQ_OK && (he = hipEventCreateWithFlags(&w.done, hipEventDisableTiming)) != hipSuccess)
            rc = DAQ_EHIP;
        if (rc == DAQ_OK && (he = hipMalloc(&w.d_counts, kMaxBatch * sizeof(daq_counts))) != hipSuccess)
            rc = he == hipErrorOutOfMemory ? DAQ_ENOMEM : DAQ_EHIP;
        if (rc == DAQ_OK &&
            (he = hipHostMalloc(&w.h_counts, kMaxBatch * sizeof(daq_counts), hipHostMallocDefault)) != hipSuccess)
            rc = he == hipErrorOutOfMemory ? DAQ_ENOMEM : DAQ_EHIP;
    }
    if (rc != DAQ_OK) {
        for (Worker &w : srv->workers) free_worker(w);
        delete srv;
        return rc;
    }
    for (Worker &w : srv->workers) w.th = std::thread(worker_loop, srv, &w);
    daqlog::say(2, "server on device %d: %d workers, batches of up to %d fills, arena of %llu bytes", dev, n_streams,
                max_batch, (unsigned long long)srv->arena.size());
    *out = srv;
    return DAQ_OK;
}

int daq_submit_fill(daq_server *srv, const daq_fill *fill, int32_t flags, uint64_t tag, uint64_t *ticket) {
    return daq_submit_fill_at(srv, fill, flags, tag, 0, ticket);
}

int daq_submit_fill_at(daq_server *srv, const daq_fill *fill, int32_t flags, uint64_t tag, int64_t t_arrive_ns,
                       uint64_t *ticket) {
    if (!srv || !ticket) return DAQ_EINVAL;
    int rc = check_submit_fill(fill, flags);
    if (rc) return rc;
    const SlotLayout L = layout_of(*fill, flags);
    Job *j = new Job();
    std::unique_lock<std::mutex> lk(srv->mu);
    if (L.bytes > srv->arena.size()) {
        delete j;
        return DAQ_ERANGE;
    }
    const int64_t now = now_ns();
    const int64_t off = srv->arena.alloc(L.bytes);
    if (off < 0) {
        srv->stats.rejected++;
        if (srv->dead_since < 0) {
            srv->dead_since = now;
            roctxMarkA("daq_server deadtime begins");  // the budget refuses fills from here on
            daqlog::say(2, "server: deadtime begins, %llu of %llu arena bytes in use",
                        (unsigned long long)srv->arena.in_use(), (unsigned long long)srv->arena.size());
        }
        delete j;
        return DAQ_EAGAIN;
    }
    if (srv->dead_since >= 0) {
        srv->stats.deadtime_ns += (uint64_t)(now - srv->dead_since);
        srv->dead_since = -1;
    }
    const int64_t t_arr = (t_arrive_ns > 0 && t_arrive_ns <= now) ? t_arrive_ns : now;
    const uint64_t wait = (uint64_t)(now - t_arr);
    if (wait > srv->stats.admit_wait_max_ns) srv->stats.admit_wait_max_ns = wait;
    const int64_t deadline = srv->admit_deadline_ns.load(std::memory_order_relaxed);
    if (deadline > 0 && (int64_t)wait > deadline) srv->stats.late++;
    uint8_t *base = srv->arena_base + off;
    j->ticket = srv->next_ticket++;
    j->tag = tag;
    j->flags = flags;
    j->fill = *fill;
    if (flags & DAQ_SUBMIT_HOST_RAW) {
        j->host_raw = fill->raw;
        j->fill.raw = reinterpret_cast<const int16_t *>(base + L.raw);
    }
    if (flags & DAQ_SUBMIT_HOST_PACKED12) {
        j->host_packed = reinterpret_cast<const uint8_t *>(fill->raw);
        j->dev_packed = base + L.packed;
        j->fill.raw = reinterpret_cast<const int16_t *>(base + L.raw);
    }
    j->out.counts = reinterpret_cast<daq_counts *>(base + L.counts);
    j->out.ped = reinterpret_cast<int32_t *>(base + L.ped);
    j->out.islands = reinterpret_cast<daq_island *>(base + L.islands);
    j->out.capacity = L.capacity;
    j->out.out = reinterpret_cast<int16_t *>(base + L.out);
    j->out.out_stride = L.out_stride;
    j->offset = (uint64_t)off;
    j->t_submit = t_arr;
    srv->jobs[j->ticket] = j;
    srv->queue.push_back(j);
    srv->stats.submitted++;
    *ticket = j->ticket;
    lk.unlock();
    srv->cv_work.notify_one();
    return DAQ_OK;
}

int daq_poll(daq_server *srv, daq_completion *out, int32_t max, int32_t timeout_us) {
    if (!srv || max < 0 || (max > 0 && !out) || timeout_us < 0) return DAQ_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && timeout_us > 0 && max > 0)
        srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !srv->done.empty(); });
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    return k;
}

int daq_release(daq_server *srv, uint64_t ticket) {
    if (!srv) return DAQ_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return DAQ_EINVAL;
    Job *j = it->second;
    if (j->state == State::kHeld) {
        if (j->released) return DAQ_EINVAL;
        j->released = true;  // the worker frees the slot once the device is done
        srv->stats.released++;
        return DAQ_OK;
    }
    if (j->state != State::kDone) return DAQ_EAGAIN;
    srv->arena.release(j->offset);
    srv->jobs.erase(it);
    delete j;
    srv->stats.released++;
    return DAQ_OK;
}

int daq_server_set_limits(daq_server *srv, int64_t admit_deadline_us, int64_t batch_timeout_us) {
    if (!srv || admit_deadline_us < 0 || batch_timeout_us < 0) return DAQ_EINVAL;
    const int64_t big = INT64_MAX / 1000;
    srv->admit_deadline_ns.store(admit_deadline_us > big ? INT64_MAX : admit_deadline_us * 1000);
    srv->batch_timeout_ns.store(batch_timeout_us > big ? INT64_MAX : batch_timeout_us * 1000);
    return DAQ_OK;
}

int daq_server_get_stats(daq_server *srv, daq_server_stats *st) {
    if (!srv || !st) return DAQ_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *st = srv->stats;
    st->arena_in_use = srv->arena.in_use();
    st->arena_peak = srv->arena.peak();
    st->pending = (int32_t)srv->queue.size();
    st->running = srv->running;
    return DAQ_OK;
}

void daq_server_destroy(daq_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (Worker &w : srv->workers)
        if (w.th.joinable()) w.th.join();
    for (Worker &w : srv->workers) {
        if (w.stream) (void)hipStreamSynchronize(w.stream);
        w.held.clear();  // owned by srv->jobs
        free_worker(w);
    }
    for (auto &kv : srv->jobs) delete kv.second;
    const daq_server_stats &t = srv->stats;
    daqlog::say(2, "server shut down: %llu admitted, %llu refused, %llu completed in %llu batches, %llu late, "
                   "%llu timed out, %.3f ms of deadtime, arena peak %llu bytes",
                (unsigned long long)t.submitted, (unsigned long long)t.rejected, (unsigned long long)t.completed,
                (unsigned long long)t.batches, (unsigned long long)t.late, (unsigned long long)t.timed_out,
                t.deadtime_ns / 1e6, (unsigned long long)srv->arena.peak());
    delete srv;
}

}  // extern "C"
