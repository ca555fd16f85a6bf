// Randomised check of the server's pool bookkeeping (dd_pool.hpp) against a
// byte map: live ranges are disjoint and inside the pool, free + live bytes
// always equal the pool, and releasing everything leaves one free range.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2403_16665_amd/csrc/dd_pool.hpp"

int main() {
  const size_t pool = (size_t)1 << 20;
  std::mt19937_64 rng(20240325);
  struct Live { size_t off, bytes; };
  for (int round = 0; round < 20; ++round) {
    dd::RangeAlloc a;
    a.reset(pool);
    std::vector<unsigned char> owner(pool, 0);
    std::vector<Live> live;
    size_t live_bytes = 0, fails = 0;
    for (int step = 0; step < 4000; ++step) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        const size_t want = rng() % (96 * 1024);
        size_t off = 0;
        if (!a.alloc(want, &off)) {
          ++fails;
          // a failed request must really not fit any free range
          if (a.free_bytes() >= dd::round_up(want, dd::POOL_ALIGN) && a.ranges() == 1) {
            std::printf("FAIL: refused %zu with one free range of %zu\n", want, a.free_bytes());
            return 1;
          }
          continue;
        }
        const size_t b = dd::round_up(want, dd::POOL_ALIGN);
        if (b == 0) continue;
        if (off % dd::POOL_ALIGN || off + b > pool) {
          std::printf("FAIL: range [%zu, %zu) outside the pool\n", off, off + b);
          return 1;
        }
        for (size_t i = off; i < off + b; ++i) {
          if (owner[i]) {
            std::printf("FAIL: overlap at byte %zu\n", i);
            return 1;
          }
          owner[i] = 1;
        }
        live.push_back({off, want});
        live_bytes += b;
      } else {
        const size_t k = rng() % live.size();
        const Live l = live[k];
        live[k] = live.back();
        live.pop_back();
        const size_t b = dd::round_up(l.bytes, dd::POOL_ALIGN);
        for (size_t i = l.off; i < l.off + b; ++i) owner[i] = 0;
        a.release(l.off, l.bytes);
        live_bytes -= b;
      }
      if (a.free_bytes() + live_bytes != pool) {
        std::printf("FAIL: free %zu + live %zu != pool\n", a.free_bytes(), live_bytes);
        return 1;
      }
    }
    for (const Live& l : live) a.release(l.off, l.bytes);
    if (a.ranges() != 1 || a.free_bytes() != pool) {
      std::printf("FAIL: after releasing all: %zu ranges, %zu bytes\n", a.ranges(), a.free_bytes());
      return 1;
    }
    std::printf("round %d ok (%zu refusals)\n", round, fails);
  }
  std::printf("OK\n");
  return 0;
}
