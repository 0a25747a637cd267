// rp_arena.h -- host-side bookkeeping of the serving form's device arena
// (internal to librp, host code only, no HIP calls).
//
// Best-fit allocator over one region of `size` bytes: blocks are rounded up
// to 256 bytes, the smallest free block that fits is split, and a freed block
// merges with free neighbours on both sides, so freeing everything leaves one
// block again.  Offsets only; the caller adds them to the region's address.
#pragma once

#include <algorithm>
#include <cstdint>
#include <map>
#include <set>
#include <utility>

namespace rpserve {

constexpr uint64_t ALIGN = 256;

class Arena {
public:
    void reset(uint64_t size)
    {
        size_ = size;
        by_off_.clear();
        by_len_.clear();
        if (size)
            insert(0, size);
        in_use_ = peak_ = 0;
    }
    static uint64_t rounded(uint64_t bytes)
    {
        return std::max<uint64_t>(ALIGN, (bytes + ALIGN - 1) / ALIGN * ALIGN);
    }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        const uint64_t len = rounded(bytes);
        auto it = by_len_.lower_bound({len, 0});
        if (it == by_len_.end())
            return false;
        const uint64_t o = it->second, l = it->first;
        erase(o, l);
        if (l > len)
            insert(o + len, l - len);
        *off = o;
        in_use_ += len;
        peak_ = std::max(peak_, in_use_);
        return true;
    }
    void free(uint64_t off, uint64_t bytes)
    {
        uint64_t len = rounded(bytes);
        in_use_ -= len;
        auto nx = by_off_.lower_bound(off);
        if (nx != by_off_.end() && off + len == nx->first) {
            const uint64_t o = nx->first, l = nx->second;
            erase(o, l);
            len += l;
        }
        auto pv = by_off_.lower_bound(off);
        if (pv != by_off_.begin()) {
            --pv;
            if (pv->first + pv->second == off) {
                const uint64_t o = pv->first, l = pv->second;
                erase(o, l);
                off = o;
                len += l;
            }
        }
        insert(off, len);
    }
    uint64_t in_use() const { return in_use_; }
    uint64_t peak() const { return peak_; }
    uint64_t size() const { return size_; }
    size_t free_blocks() const { return by_off_.size(); }
    uint64_t largest_free() const { return by_len_.empty() ? 0 : by_len_.rbegin()->first; }

private:
    void insert(uint64_t o, uint64_t l)
    {
        by_off_[o] = l;
        by_len_.insert({l, o});
    }
    void erase(uint64_t o, uint64_t l)
    {
        by_off_.erase(o);
        by_len_.erase({l, o});
    }
    uint64_t size_ = 0, in_use_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> by_off_;
    std::set<std::pair<uint64_t, uint64_t>> by_len_;
};

}  // namespace rpserve
