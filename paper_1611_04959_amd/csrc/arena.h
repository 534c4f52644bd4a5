// arena.h -- first-fit sub-allocator over a caller-owned byte range.
//
// The serving loop keeps every admitted fill's outputs (and, for host-fed
// fills, its raw samples) resident in one device arena whose size is the HBM
// budget. This class only does the bookkeeping of offsets: it never touches
// the memory, so it is plain host C++ and is tested on the CPU.
//
// Blocks are aligned to kAlign bytes. Free ranges are kept sorted by offset
// and merged with their neighbours on release, so a budget that has been
// fully released is again one free range.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace daqk {

class Arena {
public:
    static constexpr uint64_t kAlign = 256;

    explicit Arena(uint64_t bytes = 0) { reset(bytes); }

    void reset(uint64_t bytes) {
        free_.clear();
        used_.clear();
        size_ = bytes / kAlign * kAlign;
        in_use_ = 0;
        peak_ = 0;
        if (size_) free_[0] = size_;
    }

    // Rounded size of a request.
    static uint64_t round(uint64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // Offset of a new block of n bytes (n > 0), or -1 when no free range is
    // large enough. First fit in offset order.
    int64_t alloc(uint64_t n) {
        if (n == 0) return -1;
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const uint64_t off = it->first, left = it->second - n;
            free_.erase(it);
            if (left) free_[off + n] = left;
            used_[off] = n;
            in_use_ += n;
            if (in_use_ > peak_) peak_ = in_use_;
            return (int64_t)off;
        }
        return -1;
    }

    // Returns a block to the free ranges. False for an offset that is not the
    // start of a live block (nothing changes then).
    bool release(uint64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        uint64_t n = u->second;
        used_.erase(u);
        in_use_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return true;
            }
        }
        free_[off] = n;
        return true;
    }

    uint64_t size() const { return size_; }
    uint64_t in_use() const { return in_use_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto &f : free_)
            if (f.second > m) m = f.second;
        return m;
    }
    size_t free_ranges() const { return free_.size(); }
    size_t live_blocks() const { return used_.size(); }

private:
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    std::map<uint64_t, uint64_t> used_;  // offset -> bytes
    uint64_t size_ = 0, in_use_ = 0, peak_ = 0;
};

}  // namespace daqk
