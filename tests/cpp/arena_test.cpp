// CPU test of the serving arena (first-fit, coalescing): no GPU involved.
#include "arena.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); std::exit(1); } \
  } while (0)

int main() {
  using lddmm::Arena;
  Arena a(1 << 20);
  CHECK(a.size() == (1u << 20));
  const size_t x = a.alloc(1000), y = a.alloc(5000), z = a.alloc(256);
  CHECK(x == 0 && y == 1024 && z == 1024 + 5120);
  CHECK(a.used_bytes() == 1024 + 5120 + 256);
  CHECK(a.alloc(1 << 20) == Arena::npos);            // does not fit
  CHECK(a.release(y));
  CHECK(!a.release(y));                               // double free refused
  CHECK(a.alloc(4000) == 1024);                       // first fit reuses the hole
  CHECK(a.release(x) && a.release(1024) && a.release(z));
  CHECK(a.used_bytes() == 0 && a.largest_free() == (1u << 20));   // fully coalesced
  // random alloc/free against a shadow model: blocks never overlap, all coalesce back
  std::mt19937 rng(7);
  std::vector<std::pair<size_t, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 2) {
      const size_t want = 1 + rng() % 40000, off = a.alloc(want);
      if (off == Arena::npos) continue;
      const size_t len = Arena::round_up(want);
      CHECK(off % Arena::kAlign == 0 && off + len <= a.size());
      for (auto& b : live) CHECK(off + len <= b.first || b.first + b.second <= off);
      live.emplace_back(off, len);
    } else {
      const size_t k = rng() % live.size();
      CHECK(a.release(live[k].first));
      live.erase(live.begin() + k);
    }
  }
  for (auto& b : live) CHECK(a.release(b.first));
  CHECK(a.used_bytes() == 0 && a.largest_free() == a.size() && a.blocks() == 0);
  std::printf("arena ok\n");
  return 0;
}
