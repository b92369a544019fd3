// The symmetric-heap allocator (host side; see hostalloc.hpp).
#include "hostalloc.hpp"

#include <iterator>

namespace vshmem {

void SymAllocator::reset(uint64_t capacity)
{
    free_.clear();
    live_.clear();
    cap_ = capacity;
    used_ = 0;
    if (capacity) free_[0] = capacity;
}

uint64_t SymAllocator::alloc(uint64_t size, uint64_t align)
{
    if (size == 0) return UINT64_MAX;
    size = (size + kMinAlign - 1) & ~(kMinAlign - 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        uint64_t off = it->first, len = it->second;
        uint64_t a = (off + align - 1) & ~(align - 1);
        if (a < off || a - off > len || len - (a - off) < size) continue;
        uint64_t end = off + len;
        free_.erase(it);
        if (a > off) free_[off] = a - off;
        if (a + size < end) free_[a + size] = end - (a + size);
        live_[a] = size;
        used_ += size;
        return a;
    }
    return UINT64_MAX;
}

bool SymAllocator::free(uint64_t off)
{
    auto it = live_.find(off);
    if (it == live_.end()) return false;
    uint64_t len = it->second;
    live_.erase(it);
    used_ -= len;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {   // merge with the next hole
        len += nx->second;
        nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {                           // merge with the previous hole
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += len;
            return true;
        }
    }
    free_[off] = len;
    return true;
}

}  // namespace vshmem
