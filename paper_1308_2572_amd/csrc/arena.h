// First-fit allocator with coalescing, used by the quote server to admit
// quotes against the caller's device arena (offsets only; it never touches
// memory, so it is plain C++ and unit-tested on the CPU).
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace ara {

class Arena {
   public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t o = it->first, rem = it->second - n;
                free_.erase(it);
                if (rem) free_[o + n] = rem;
                *off = o;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }
    size_t size() const { return size_; }

   private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0;
};

}  // namespace ara
