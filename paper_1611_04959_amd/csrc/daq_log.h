// daq_log.h -- diagnostic lines of libdaqisland on stderr.
//
// The environment variable DAQ_LOG sets how much the library says, read once
// per process:
//   0 or unset  nothing;
//   1           failures: a HIP call that failed (with the call), a batch
//               the server's watchdog gave up on, a batch that failed;
//   2           also the library's decisions: context creation (device,
//               architecture, compute units), a schedule taken from
//               DAQ_SCHEDULE, every schedule the tuner timed and the one it
//               kept, graph captures, scratch growth, server creation and
//               shutdown (with its counters), the start of a deadtime period.
// Each line starts with "[daq] " and is written with one stdio call, so lines
// of different threads do not interleave.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <cstdlib>

namespace daqlog {

inline int level() {
    static const int lv = [] {
        const char *s = std::getenv("DAQ_LOG");
        if (!s || !*s) return 0;
        const int v = std::atoi(s);
        return v < 0 ? 0 : v;
    }();
    return lv;
}

// Writes one line when DAQ_LOG is at least `lv`; lv 0 always writes.
__attribute__((format(printf, 2, 3))) inline void say(int lv, const char *fmt, ...) {
    if (lv > 0 && level() < lv) return;
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[daq] %s\n", buf);
}

}  // namespace daqlog
