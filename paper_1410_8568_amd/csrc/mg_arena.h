// First-fit allocator over the byte range [0, size) of the solve server's HBM
// arena, with coalescing frees.  Host-only (no HIP), so its admission logic can
// be tested on the CPU.  Offsets and sizes are multiples of 256 bytes.
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

namespace mgrt {

class Arena {
   public:
    void reset(size_t size) {
        free_.clear();
        size_ = size & ~(size_t)255;
        if (size_) free_[0] = size_;
    }
    // Lowest-offset free range that fits; false if none does.
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
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
    size_t free_bytes() const {
        size_t s = 0;
        for (auto& kv : free_) s += kv.second;
        return s;
    }
    size_t largest_free() const {
        size_t s = 0;
        for (auto& kv : free_) s = kv.second > s ? kv.second : s;
        return s;
    }
    size_t size() const { return size_; }
    size_t fragments() const { return free_.size(); }

   private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0;
};

}  // namespace mgrt
