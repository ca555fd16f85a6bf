// dd_pool.hpp -- host bookkeeping of a device memory pool: first-fit
// allocation of byte ranges, free ranges merged with their neighbours on
// release.  Plain C++ (no HIP), so that it can be checked on any host.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace dd {

constexpr size_t POOL_ALIGN = 256;

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Ranges are multiples of POOL_ALIGN bytes; alloc of 0 bytes takes none.
class RangeAlloc {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes, POOL_ALIGN);
    if (bytes == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[o + bytes] = rest;
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes, POOL_ALIGN);
    if (bytes == 0) return;
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

  // Sum of the free bytes and number of free ranges (for checks).
  size_t free_bytes() const {
    size_t n = 0;
    for (const auto& kv : free_) n += kv.second;
    return n;
  }
  size_t ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace dd
