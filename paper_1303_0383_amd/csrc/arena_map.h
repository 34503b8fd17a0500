// arena_map.h -- first-fit allocation of offsets in a device arena (the
// serving engine's pieces each take one region).  Host-only C++; no HIP.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace lagp_rt {

// Free blocks by offset; callers allocate multiples of 256 bytes, and a
// released block merges with free neighbours on either side.
class ArenaMap {
    std::map<size_t, size_t> free_;   // offset -> bytes
public:
    void reset(size_t bytes)
    {
        free_.clear();
        const size_t b = bytes & ~(size_t)255;
        if (b) free_[0] = b;
    }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t blocks() const { return free_.size(); }
    // The lowest-offset free block that holds `bytes` (> 0) gives its front.
    bool alloc(size_t bytes, size_t* off)
    {
        if (bytes == 0) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o = it->first;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            return true;
        }
        return false;
    }
    // Return [off, off + bytes), a region alloc() handed out.
    void release(size_t off, size_t bytes)
    {
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
};

}  // namespace lagp_rt
