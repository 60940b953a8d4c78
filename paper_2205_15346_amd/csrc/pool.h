// First-fit sub-allocator over one device allocation (host-side bookkeeping only).
//
// The serving engine takes all job workspaces from one pool allocated at start-up, so
// admitting or retiring a job never calls the device allocator (whose free synchronises the
// device).  Offsets are aligned to kAlign; freed ranges coalesce with their neighbours.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace te {

class PoolAlloc {
  public:
    static constexpr uint64_t kAlign = 256;

    PoolAlloc() = default;
    explicit PoolAlloc(uint64_t bytes) { reset(bytes); }

    void reset(uint64_t bytes) {
        free_.clear();
        live_.clear();
        size_ = bytes / kAlign * kAlign;
        used_ = peak_ = 0;
        if (size_ > 0) free_[0] = size_;
    }

    static uint64_t round(uint64_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

    // first fit; false if no free range is large enough
    bool alloc(uint64_t bytes, uint64_t* off) {
        const uint64_t need = round(bytes == 0 ? 1 : bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const uint64_t rest = it->second - need;
            const uint64_t next = it->first + need;
            free_.erase(it);
            if (rest > 0) free_[next] = rest;
            live_[*off] = need;
            used_ += need;
            if (used_ > peak_) peak_ = used_;
            return true;
        }
        return false;
    }

    bool fits(uint64_t bytes) const {
        const uint64_t need = round(bytes == 0 ? 1 : bytes);
        for (const auto& f : free_)
            if (f.second >= need) return true;
        return false;
    }

    // returns false (and changes nothing) unless (off, bytes) is a live allocation
    bool release(uint64_t off, uint64_t bytes) {
        const uint64_t len = round(bytes == 0 ? 1 : bytes);
        auto live = live_.find(off);
        if (live == live_.end() || live->second != len) return false;
        live_.erase(live);
        auto next = free_.lower_bound(off);
        uint64_t start = off, length = len;
        if (next != free_.end() && next->first == off + len) {
            length += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                length += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = length;
        used_ -= len;
        return true;
    }

    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    size_t ranges() const { return free_.size(); }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto& f : free_)
            if (f.second > m) m = f.second;
        return m;
    }

  private:
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    std::map<uint64_t, uint64_t> live_;  // allocated offset -> length
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace te
