// sched.hpp -- the run server's host-side policy, free of HIP so that it can
// be checked on its own: the first-fit allocator of the device arena, the
// admission rule and the latency percentiles.
#pragma once
#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>
#include <vector>

namespace clgc {

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator over [0, size) in 256-byte units: alloc takes the
// lowest-addressed free range that fits, release returns a range and merges
// it with free neighbours, so that freed memory is whole again.
class Heap {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = align256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align256(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t free_ranges() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;  // offset -> length of each free range
    size_t size_ = 0, used_ = 0;
};

// Admission of the queue's head: FIFO, so a run that does not fit blocks the
// ones behind it (no run is overtaken, and a large run cannot starve).  It is
// admitted when its precision group has room for one more run in a batched
// launch and the arena a free range of its bytes, which it then holds.
inline bool admit_head(Heap& heap, size_t bytes, int group_runs, int max_group_runs, size_t* off)
{
    if (group_runs >= max_group_runs) return false;
    return heap.alloc(bytes, off);
}

// q-quantile (0 <= q <= 1) with linear interpolation between order statistics
inline double percentile(std::vector<float> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace clgc
