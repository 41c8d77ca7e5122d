// First-fit sub-allocator over one contiguous range (offsets only; no
// device calls), used by the request server for its HBM admission budget.
// Blocks are rounded up to 256 bytes; freed neighbours coalesce.  Not
// thread-safe: the server calls it under its own lock.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace grav {

class Arena {
  public:
    static constexpr size_t kAlign = 256;
    static size_t round(size_t bytes) { return (((bytes ? bytes : 1) + kAlign - 1) / kAlign) * kAlign; }

    explicit Arena(size_t size) : size_(size / kAlign * kAlign) {
        if (size_) free_[0] = size_;
    }
    // first free range that fits; false (nothing changed) if none does
    bool alloc(size_t bytes, size_t *off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    // give back a range returned by alloc (same size argument)
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

  private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, disjoint, coalesced
};

}  // namespace grav
