// Caching allocators owned by a context.  Plans draw their workspace from
// here and hand it back on spk_free, so repeated plan/solve/free cycles of
// the same shape cost no hipMalloc/hipFree (each of which synchronises the
// device and costs up to milliseconds for large blocks).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <iterator>
#include <map>
#include <unordered_map>

namespace spk {

template <bool Pinned>
class CachingPool {
  public:
    explicit CachingPool(size_t cache_cap = 0) : cap_(cache_cap) {}
    CachingPool(const CachingPool &) = delete;
    CachingPool &operator=(const CachingPool &) = delete;
    ~CachingPool() { trim(); }

    void set_cap(size_t cap) { cap_ = cap; }

    // Budget mode: blocks are reused only at their exact (rounded) size, and
    // the cap bounds everything the pool holds (blocks in use plus cached
    // ones), so the device memory held never exceeds the cap.  get() fails
    // with hipErrorOutOfMemory when a request would pass it.
    void set_budget_mode(bool on) { budget_ = on; }

    // A block of at least `bytes` (reusing a cached block no larger than
    // twice the request; in budget mode only one of the same size), or a
    // fresh allocation.
    hipError_t get(size_t bytes, void **out) {
        bytes = round(bytes);
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && (budget_ ? it->first == bytes : it->first <= 2 * bytes)) {
            *out = it->second;
            cached_ -= it->first;
            in_use_ += it->first;
            free_.erase(it);
            return hipSuccess;
        }
        if (budget_) {
            if (in_use_ + bytes > cap_) return hipErrorOutOfMemory;
            // give back cached blocks until the new one fits under the cap
            while (!free_.empty() && in_use_ + cached_ + bytes > cap_) {
                auto victim = std::prev(free_.end());   // the largest first
                cached_ -= victim->first;
                size_.erase(victim->second);
                raw_free(victim->second);
                free_.erase(victim);
            }
        }
        void *p = nullptr;
        hipError_t e = raw_alloc(&p, bytes);
        if (e != hipSuccess) {
            trim();   // give the cache back and retry once
            e = raw_alloc(&p, bytes);
            if (e != hipSuccess) return e;
        }
        size_[p] = bytes;
        in_use_ += bytes;
        *out = p;
        return hipSuccess;
    }

    // Return a block obtained from get(); it stays cached while the cache
    // is below its cap.  The caller guarantees no queued work still uses it.
    void put(void *p) {
        if (!p) return;
        auto s = size_.find(p);
        if (s == size_.end()) return;
        const size_t bytes = s->second;
        in_use_ -= bytes;
        if (cached_ + bytes + (budget_ ? in_use_ : 0) > cap_) {
            size_.erase(s);
            raw_free(p);
            return;
        }
        free_.emplace(bytes, p);
        cached_ += bytes;
    }

    void trim() {
        for (auto &kv : free_) {
            size_.erase(kv.second);
            raw_free(kv.second);
        }
        free_.clear();
        cached_ = 0;
    }

    size_t in_use() const { return in_use_; }
    size_t cached() const { return cached_; }
    // Size of a block get(bytes) hands out (requests are rounded up to 256 bytes).
    static size_t block_bytes(size_t bytes) { return round(bytes); }

  private:
    static size_t round(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }
    static hipError_t raw_alloc(void **p, size_t bytes) {
        if (Pinned) return hipHostMalloc(p, bytes, hipHostMallocDefault);
        return hipMalloc(p, bytes);
    }
    static void raw_free(void *p) {
        if (Pinned) (void)hipHostFree(p);
        else (void)hipFree(p);
    }

    std::multimap<size_t, void *> free_;
    std::unordered_map<void *, size_t> size_;
    size_t in_use_ = 0, cached_ = 0, cap_;
    bool budget_ = false;
};

using DevicePool = CachingPool<false>;
using PinnedPool = CachingPool<true>;

}  // namespace spk
