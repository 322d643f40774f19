// Host unit test of the arena allocator (paper_2006_09808_amd/csrc/pd_arena.hpp)
// against a brute-force model: a map of which 256-byte granules are taken.
// Random allocate/release sequences; every allocation must be aligned, in
// range, disjoint from the live ones, and at the lowest offset whose free run
// fits (first fit over maximal runs); an allocation fails exactly when no free
// run is long enough; releasing everything leaves one run of the whole arena.
// Prints "ok <operations>" or the first violation, exit status 0 / 1.
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "pd_arena.hpp"

namespace {

struct Model {
  std::vector<char> used;   // one entry per granule
  explicit Model(size_t granules) : used(granules, 0) {}
  // lowest start of a free run of n granules, or -1
  long first_fit(size_t n) const {
    size_t run = 0;
    for (size_t g = 0; g < used.size(); ++g) {
      run = used[g] ? 0 : run + 1;
      if (run == n) return (long)(g + 1 - n);
    }
    return -1;
  }
  void mark(size_t g0, size_t n, char v) {
    for (size_t g = g0; g < g0 + n; ++g) used[g] = v;
  }
};

int fail(const char* what, long a, long b) {
  std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

}  // namespace

int main() {
  const size_t G = pdh::kArenaAlign;
  long ops = 0;
  for (int trial = 0; trial < 40; ++trial) {
    std::mt19937_64 rng(1234 + trial);
    const size_t granules = 64 + rng() % 512;
    const size_t size = granules * G + (trial % 3 == 0 ? 100 : 0);   // a ragged tail is never handed out
    pdh::Arena a;
    a.init(nullptr, size);
    Model m(granules);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    for (int step = 0; step < 600; ++step, ++ops) {
      const bool do_alloc = live.empty() || (rng() % 100) < 55;
      if (do_alloc) {
        // sizes from one byte to a quarter of the arena, often not multiples of 256
        const size_t bytes = 1 + rng() % (size / 4);
        const size_t n = (bytes + G - 1) / G;
        size_t off = 0;
        const bool ok = a.alloc(bytes, &off);
        const long want = m.first_fit(n);
        if (ok != (want >= 0)) return fail("alloc success differs from the model", (long)ok, want);
        if (!ok) continue;
        if (off % G) return fail("unaligned offset", (long)off, 0);
        if (off / G != (size_t)want) return fail("not the first fit", (long)(off / G), want);
        if (off + n * G > size) return fail("out of range", (long)off, (long)n);
        m.mark(off / G, n, 1);
        live.push_back({off, bytes});
      } else {
        const size_t k = rng() % live.size();
        a.release(live[k].off, live[k].bytes);
        m.mark(live[k].off / G, (live[k].bytes + G - 1) / G, 0);
        live.erase(live.begin() + (long)k);
      }
      size_t in_use = 0;
      for (char u : m.used) in_use += (size_t)u;
      if (a.used() != in_use * G) return fail("used() differs from the model", (long)a.used(), (long)(in_use * G));
    }
    for (auto& l : live) a.release(l.off, l.bytes);
    size_t off = 0;
    if (a.used() != 0) return fail("bytes still in use after releasing all", (long)a.used(), 0);
    if (!a.alloc(granules * G, &off) || off != 0) return fail("arena not one run after releasing all", (long)off, 0);
  }
  std::printf("ok %ld\n", ops);
  return 0;
}
