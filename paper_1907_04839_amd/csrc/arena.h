// First-fit allocator over one preallocated device region: host-side
// bookkeeping only, no device calls, so it is testable on the CPU.  The
// serving layer admits a registration when its footprint fits here.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace lddmm {

class Arena {
 public:
  static constexpr size_t kAlign = 256;

  explicit Arena(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    size_ = bytes - bytes % kAlign;
    free_.clear();
    used_.clear();
    if (size_) free_[0] = size_;
  }

  static size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

  // Offset of a block of at least `bytes`, or npos when nothing fits.
  size_t alloc(size_t bytes) {
    const size_t need = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      return off;
    }
    return npos;
  }

  // Returns a block; neighbouring free blocks are merged.  False if `off` was
  // not allocated.
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  size_t size() const { return size_; }
  size_t used_bytes() const {
    size_t s = 0;
    for (const auto& kv : used_) s += kv.second;
    return s;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  size_t blocks() const { return used_.size(); }

  static constexpr size_t npos = static_cast<size_t>(-1);

 private:
  size_t size_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> used_;
};

}  // namespace lddmm
