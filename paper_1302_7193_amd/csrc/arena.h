// Host-side bookkeeping of the serving runtime: a first-fit sub-allocator
// over one device arena and the FIFO admission rule.  No HIP calls here
// (compiled by g++ in the CPU tests).
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace pcg {

// First-fit allocator over [0, size) with 256-byte granularity; free blocks
// coalesce with their neighbours.  Offsets, not pointers.
class Arena {
public:
    static constexpr size_t kAlign = 256;

    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size)
    {
        free_.clear();
        used_.clear();
        size_ = size & ~(kAlign - 1);
        if (size_) free_[0] = size_;
        in_use_ = 0;
    }

    // Returns false when no free block is large enough.
    bool alloc(size_t bytes, size_t* offset)
    {
        const size_t need = round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            used_[off] = need;
            in_use_ += need;
            *offset = off;
            return true;
        }
        return false;
    }

    // Returns false for an offset that is not allocated.
    bool release(size_t offset)
    {
        auto u = used_.find(offset);
        if (u == used_.end()) return false;
        size_t off = offset, len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }
    static size_t round(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

private:
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;   // offset -> length
    size_t size_ = 0;
    size_t in_use_ = 0;
};

// Admission rule: the oldest queued request is admitted when a worker slot is
// free, its device bytes keep the admitted total within the budget, and the
// arena has a block for it.  Strict FIFO: a request that does not fit holds
// back the ones behind it (no starvation of large requests).
inline bool admissible(size_t budget, size_t admitted_bytes, size_t need, int active,
                       int max_active)
{
    return active < max_active && need <= budget && admitted_bytes + need <= budget;
}

}  // namespace pcg
