// Device-memory arena: one hipMalloc at construction, first-fit sub-allocation
// with 256-byte alignment and coalescing frees.  Thread-safe.  Used by the
// request server so that admitting, building and retiring cells never calls
// hipMalloc or hipFree (hipFree waits for the whole device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>

namespace pbcjk {

class Arena {
public:
    static constexpr size_t kAlign = 256;

    // Returns hipSuccess or the hipMalloc error.
    hipError_t init(size_t bytes)
    {
        cap_ = round_up(bytes);
        hipError_t e = hipMalloc((void **)&base_, cap_);
        if (e != hipSuccess) {
            base_ = nullptr;
            cap_ = 0;
            return e;
        }
        free_.clear();
        free_[0] = cap_;
        return hipSuccess;
    }
    ~Arena()
    {
        if (base_) (void)hipFree(base_);
    }

    // nullptr when no free block is large enough.
    void *alloc(size_t n)
    {
        n = round_up(n ? n : 1);
        std::lock_guard<std::mutex> lk(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            used_[off] = n;
            in_use_ += n;
            if (in_use_ > peak_) peak_ = in_use_;
            return base_ + off;
        }
        return nullptr;
    }

    // Returns false for a pointer this arena did not hand out.
    bool release(void *p)
    {
        if (!p) return true;
        std::lock_guard<std::mutex> lk(mu_);
        const size_t off = (size_t)((char *)p - base_);
        auto u = used_.find(off);
        if ((char *)p < base_ || u == used_.end()) return false;
        size_t sz = u->second, start = off;
        used_.erase(u);
        in_use_ -= sz;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && nx->first == off + sz) {
            sz += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                sz += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = sz;
        return true;
    }

    bool owns(const void *p) const
    {
        return base_ && (const char *)p >= base_ && (const char *)p < base_ + cap_;
    }
    size_t capacity() const { return cap_; }
    size_t in_use()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return in_use_;
    }
    size_t peak()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return peak_;
    }
    size_t largest_free()
    {
        std::lock_guard<std::mutex> lk(mu_);
        size_t m = 0;
        for (auto &f : free_)
            if (f.second > m) m = f.second;
        return m;
    }
    static size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

private:
    char *base_ = nullptr;
    size_t cap_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;          // offset -> size
    std::unordered_map<size_t, size_t> used_;  // offset -> size
    std::mutex mu_;
};

}  // namespace pbcjk
