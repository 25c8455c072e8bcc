// First-fit free list over a byte range [0, size), in granules of kAlign
// bytes: the bookkeeping of the request server's device arena.  Plain C++
// (no device code), so that it is tested on the host by itself.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace fdbb {

class FreeList {
public:
    static constexpr size_t kAlign = 256;

    static size_t round(size_t bytes) { return std::max(kAlign, (bytes + kAlign - 1) / kAlign * kAlign); }

    // Start with one free block covering `bytes` rounded up to a granule.
    void reset(size_t bytes)
    {
        size_ = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ = 0;
        free_.clear();
        if (size_) free_[0] = size_;
    }

    // Offset of a block of `bytes` (rounded up to a granule) at the lowest
    // address that fits, or SIZE_MAX when no free block is large enough.
    size_t alloc(size_t bytes)
    {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_ += bytes;
                return off;
            }
        }
        return SIZE_MAX;
    }

    // Give back a block that alloc(bytes) returned at `off`; it merges with
    // free neighbours.
    void release(size_t off, size_t bytes)
    {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_blocks() const { return free_.size(); }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    size_t size_ = 0;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, no two adjacent
};

}  // namespace fdbb
