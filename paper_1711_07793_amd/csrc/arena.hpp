// First-fit allocator over one preallocated range [0, size): the serving
// engine's HBM budget.  Host-only bookkeeping (offsets, no memory access), so
// it builds with any C++17 compiler and is unit-tested on the CPU.
#pragma once

#include <stdint.h>

#include <iterator>
#include <map>

namespace rbsm {

class Arena {
  public:
    static constexpr int64_t kAlign = 256;

    explicit Arena(int64_t size = 0) { reset(size); }

    void reset(int64_t size) {
        free_.clear();
        size_ = size > 0 ? size : 0;
        used_ = 0;
        peak_ = 0;
        if (size_ > 0) free_[0] = size_;
    }

    static int64_t round_up(int64_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // Offset of a block of at least `bytes` (rounded up to kAlign), or -1 when
    // no free run is large enough.  The lowest-addressed fitting run is used.
    int64_t alloc(int64_t bytes) {
        const int64_t want = round_up(bytes > 0 ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < want) continue;
            const int64_t off = it->first, rest = it->second - want;
            free_.erase(it);
            if (rest > 0) free_[off + want] = rest;
            used_ += want;
            if (used_ > peak_) peak_ = used_;
            return off;
        }
        return -1;
    }

    // Return a block obtained from alloc(bytes); merges with free neighbours.
    void release(int64_t off, int64_t bytes) {
        int64_t start = off, len = round_up(bytes > 0 ? bytes : 1);
        used_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(start);
        if (next != free_.end() && start + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }

    int64_t size() const { return size_; }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    int64_t largest_free() const {
        int64_t m = 0;
        for (const auto &kv : free_)
            if (kv.second > m) m = kv.second;
        return m;
    }
    size_t free_runs() const { return free_.size(); }

  private:
    std::map<int64_t, int64_t> free_;  // offset -> length, disjoint, non-adjacent
    int64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace rbsm
