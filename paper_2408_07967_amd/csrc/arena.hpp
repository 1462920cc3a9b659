// Host-side pieces of the render server's admission control, free of HIP so
// they can be exercised on their own: a first-fit allocator over one device
// allocation (offsets only) and the FIFO-with-bounded-bypass admission rule.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace fgs {

constexpr size_t kArenaAlign = 256;

inline size_t arena_align(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size): free ranges in a map ordered by offset,
// coalesced on release.  Sizes are rounded up to kArenaAlign.
class Arena {
  public:
    void init(size_t bytes) {
        size_ = bytes / kArenaAlign * kArenaAlign;
        free_.clear();
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = arena_align(bytes);
        if (bytes == 0) bytes = kArenaAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    // bytes: the size passed to alloc
    void release(size_t off, size_t bytes) {
        bytes = arena_align(bytes);
        if (bytes == 0) bytes = kArenaAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest_free() const {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }
    size_t free_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

// Admission over the waiting requests in arrival order (FIFO).  try_admit(w)
// admits w if its buffers can be reserved now.  The oldest request that does
// not fit blocks every later one once it has been overtaken max_bypass times;
// until then later requests that fit go ahead, each counting one bypass of
// it.  bypassed(w) is the per-request counter (kept across calls).  Returns
// the number of requests admitted.
template <class W, class TryAdmit, class Bypassed>
int admit_fifo_bounded_bypass(const std::vector<W> &waiting, int max_bypass, TryAdmit try_admit,
                              Bypassed bypassed, int64_t *bypasses) {
    int admitted = 0;
    W blocked{};
    bool have_blocked = false;
    for (const W &w : waiting) {
        if (have_blocked && bypassed(blocked) >= max_bypass) break;
        if (!try_admit(w)) {
            if (!have_blocked) {
                blocked = w;
                have_blocked = true;
            }
            continue;
        }
        if (have_blocked) {
            bypassed(blocked) += 1;
            *bypasses += 1;
        }
        ++admitted;
    }
    return admitted;
}

}  // namespace fgs
