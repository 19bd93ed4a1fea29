// cg_arena.h - first-fit allocator over one device region (the caller's
// arena tensor or a region the library allocated).  Host-only bookkeeping:
// no device call, so it is also built and tested without a GPU.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>

namespace cgr {

// Blocks are carved first-fit in address order with 256-byte granularity;
// a released block coalesces with free neighbours on both sides.
class Arena {
 public:
  static constexpr size_t kAlign = 256;

  void init(char* base, size_t size) {
    base_ = base;
    size_ = size / kAlign * kAlign;
    free_.clear();
    used_.clear();
    in_use_ = 0;
    if (size_) free_[0] = size_;
  }

  // nullptr when no free block is large enough.
  void* alloc(size_t n) {
    n = (n ? n : 1) + kAlign - 1;
    n -= n % kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, sz = it->second;
        free_.erase(it);
        if (sz > n) free_[off + n] = sz - n;
        used_[off] = n;
        in_use_ += n;
        return base_ + off;
      }
    }
    return nullptr;
  }

  // Pointers that alloc() did not return (or already released) are ignored.
  void release(void* p) {
    if (!p) return;
    const size_t off = (size_t)((char*)p - base_);
    auto it = used_.find(off);
    if (it == used_.end()) return;
    size_t start = off, n = it->second;
    used_.erase(it);
    in_use_ -= n;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        pv->second += n;
        return;
      }
    }
    free_[start] = n;
  }

  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  char* base() const { return base_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  std::map<size_t, size_t> used_;  // offset -> bytes
};

}  // namespace cgr
