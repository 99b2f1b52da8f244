// First-fit range allocator of the serving scheduler's device pool: plain C++,
// no device code, so it can be unit-tested on the host.  Private to the library.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace dsdp {
namespace host {

// First-fit allocator over [0, total) with coalescing of freed ranges.
struct RangeAlloc {
    std::map<size_t, size_t> free_;   // offset -> length
    size_t total = 0, used = 0;
    void init(size_t n)
    {
        free_.clear();
        if (n) free_[0] = n;
        total = n;
        used = 0;
    }
    bool alloc(size_t n, size_t &off)
    {
        if (n == 0) n = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                used += n;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        if (n == 0) n = 1;
        used -= n;
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
};

}  // namespace host
}  // namespace dsdp
