// au_arena.h -- first-fit allocator over an address range, used by the
// server to carve its device arena and pinned staging area.  Host-only
// bookkeeping (no HIP); offsets and sizes are rounded up to 256 bytes, and
// freed neighbours are merged.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace au {

inline size_t arena_round(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) in 256-byte granules; host bookkeeping only.
class Arena {
public:
    void init(size_t size)
    {
        free_.clear();
        size_ = size & ~(size_t)255;
        if (size_) free_[0] = size_;
        in_use_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = arena_round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o2 = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = arena_round(bytes ? bytes : 1);
        in_use_ -= bytes;
        auto nx = free_.lower_bound(off);
        size_t o = off, len = bytes;
        if (nx != free_.end() && o + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == o) {
                o = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[o] = len;
    }
    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, in_use_ = 0, peak_ = 0;
};

}  // namespace au
