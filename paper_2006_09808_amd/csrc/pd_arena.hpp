// pd_arena.hpp - first-fit allocator over the caller's device memory (the
// arena whose size is a context's HBM budget).  Host bookkeeping only: it
// hands out byte offsets, 256-byte aligned, and never touches the memory.
// Freed blocks merge with free neighbours, so the free list always holds
// maximal runs and an allocation fails only if no single run is large enough.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace pdh {

constexpr size_t kArenaAlign = 256;
inline size_t arena_align(size_t x) { return (x + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

class Arena {
 public:
  void init(char* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = arena_align(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        size_t o = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[o + bytes] = len - bytes;
        used_ += bytes;
        *off = o;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = arena_align(std::max<size_t>(bytes, 1));
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
  char* ptr(size_t off) const { return base_ + off; }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

}  // namespace pdh
