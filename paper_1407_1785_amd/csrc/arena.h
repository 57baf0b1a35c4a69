// First-fit allocator of one device allocation (host-side bookkeeping
// only, no device calls): the HBM arena from which the batched and served
// solves take one block per running problem.  Blocks are 256-byte aligned;
// freed blocks merge with free neighbours.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace tsvd {

class Arena {
public:
    void reset(char* base, size_t cap) {
        base_ = base;
        cap_ = cap;
        used_ = 0;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool take(size_t bytes, size_t* off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        bytes = round(bytes);
        used_ -= bytes;
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
    char* base() const { return base_; }
    size_t cap() const { return cap_; }
    size_t used() const { return used_; }
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }

private:
    char* base_ = nullptr;
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

}  // namespace tsvd
