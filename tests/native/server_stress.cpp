// Host-side stress of the serving loop, for sanitizer builds of the library
// (AddressSanitizer and UndefinedBehaviorSanitizer on host code only):
// several submitter threads and one poller drive a server with three workers
// and a budget that refuses fills now and then, the watchdog limit is changed
// while batches run, and every completion is checked against the same fill's
// first result. Uses include/daq.h and HIP's C runtime API only.
//
//   server_stress SECONDS
//
// Exit status 0 when every completion matched, 1 on a mismatch, 3 on a
// library or runtime error (printed).
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "daq.h"

namespace {

constexpr int kFills = 8;
constexpr int32_t kC = 54;
constexpr int64_t kN = 100000;

#define CHECK_HIP(x)                                                  \
    do {                                                              \
        hipError_t e_ = (x);                                          \
        if (e_ != hipSuccess) {                                       \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); \
            return 3;                                                 \
        }                                                             \
    } while (0)

// A fill with a baseline of 1800 and negative pulses at fill-dependent
// spacing, so that every fill has islands of its own count.
std::vector<int16_t> make_fill(int f) {
    std::vector<int16_t> x((size_t)kC * kN, 1800);
    const int64_t gap = 900 + 137 * f;
    for (int64_t t0 = 500; t0 + 40 < kN; t0 += gap)
        for (int c = 0; c < 4; c++)
            for (int k = 0; k < 30; k++) x[(size_t)(c + 3 * f % 40) * kN + t0 + k] = (int16_t)(1800 - 400 + 10 * k);
    return x;
}

}  // namespace

int main(int argc, char **argv) {
    const double seconds = argc > 1 ? std::atof(argv[1]) : 2.0;
    daq_ctx *ctx = nullptr;
    if (daq_ctx_create(&ctx, 0) != DAQ_OK) {
        std::fprintf(stderr, "daq_ctx_create failed\n");
        return 3;
    }
    std::vector<void *> raw(kFills, nullptr);
    for (int f = 0; f < kFills; f++) {
        const std::vector<int16_t> x = make_fill(f);
        CHECK_HIP(hipMalloc(&raw[(size_t)f], x.size() * sizeof(int16_t)));
        CHECK_HIP(hipMemcpy(raw[(size_t)f], x.data(), x.size() * sizeof(int16_t), hipMemcpyHostToDevice));
    }
    std::vector<daq_fill> fills(kFills);
    for (int f = 0; f < kFills; f++) fills[(size_t)f] = daq_fill{(const int16_t *)raw[(size_t)f], kN, kN, kC, 100, -200, 8, 24, 0};
    uint64_t slot = 0;
    if (daq_server_slot_bytes(&fills[0], 0, &slot) != DAQ_OK) return 3;
    // room for about six fills: submitters see DAQ_EAGAIN regularly
    const size_t arena_bytes = (size_t)slot * 6 + 4096;
    void *arena = nullptr;
    CHECK_HIP(hipMalloc(&arena, arena_bytes));
    daq_server *srv = nullptr;
    if (daq_server_create(&srv, ctx, arena, arena_bytes, 3, 4) != DAQ_OK) {
        std::fprintf(stderr, "daq_server_create failed\n");
        return 3;
    }

    std::atomic<bool> stop{false};
    std::atomic<int64_t> submitted{0}, refused{0}, completed{0}, mismatched{0}, errors{0};
    std::mutex mu;
    std::vector<int64_t> first_islands(kFills, -1), first_len(kFills, -1);

    auto submitter = [&](int id) {
        uint64_t k = (uint64_t)id * 7919u;
        while (!stop.load()) {
            const int f = (int)(k++ % kFills);
            uint64_t ticket = 0;
            const int rc = daq_submit_fill(srv, &fills[(size_t)f], 0, (uint64_t)f, &ticket);
            if (rc == DAQ_OK) {
                submitted++;
            } else if (rc == DAQ_EAGAIN) {
                refused++;
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else {
                errors++;
                return;
            }
        }
    };
    auto poller = [&]() {
        daq_completion c[32];
        while (!stop.load() || completed.load() < submitted.load()) {
            const int n = daq_poll(srv, c, 32, 1000);
            if (n < 0) {
                errors++;
                return;
            }
            for (int i = 0; i < n; i++) {
                const int f = (int)c[i].tag;
                if (c[i].status == DAQ_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    if (first_islands[(size_t)f] < 0) {
                        first_islands[(size_t)f] = c[i].counts.n_islands;
                        first_len[(size_t)f] = c[i].counts.total_len;
                    } else if (first_islands[(size_t)f] != c[i].counts.n_islands ||
                               first_len[(size_t)f] != c[i].counts.total_len) {
                        mismatched++;
                    }
                } else if (c[i].status != DAQ_ETIMEDOUT) {
                    errors++;
                }
                int rc = daq_release(srv, c[i].ticket);
                // a timed-out fill's slot comes back once the device is done
                while (rc == DAQ_EAGAIN) {
                    std::this_thread::sleep_for(std::chrono::microseconds(100));
                    rc = daq_release(srv, c[i].ticket);
                }
                if (rc != DAQ_OK) errors++;
                completed++;
            }
        }
    };
    auto watchdog = [&]() {
        // alternate a tight batch time-out (some batches give up and hold
        // their slots) with a normal one, while the others run
        int k = 0;
        while (!stop.load()) {
            daq_server_set_limits(srv, 10000, (k++ % 4 == 0) ? 1 : 10000000);
            daq_server_stats st;
            daq_server_get_stats(srv, &st);
            std::this_thread::sleep_for(std::chrono::milliseconds(20));
        }
        daq_server_set_limits(srv, 10000, 10000000);
    };

    std::vector<std::thread> th;
    for (int i = 0; i < 3; i++) th.emplace_back(submitter, i);
    std::thread pt(poller), wt(watchdog);
    std::this_thread::sleep_for(std::chrono::duration<double>(seconds));
    stop = true;
    for (auto &t : th) t.join();
    wt.join();
    pt.join();
    daq_server_stats st;
    daq_server_get_stats(srv, &st);
    daq_server_destroy(srv);
    (void)hipFree(arena);
    for (void *p : raw) (void)hipFree(p);
    daq_ctx_destroy(ctx);
    std::printf("submitted %lld refused %lld completed %lld mismatched %lld errors %lld timed_out %llu batches %llu\n",
                (long long)submitted.load(), (long long)refused.load(), (long long)completed.load(),
                (long long)mismatched.load(), (long long)errors.load(), (unsigned long long)st.timed_out,
                (unsigned long long)st.batches);
    if (errors.load()) return 3;
    return mismatched.load() ? 1 : 0;
}
