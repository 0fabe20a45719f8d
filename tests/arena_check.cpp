// Randomised check of the serving pool's first-fit allocator against a
// brute-force page map: allocations never overlap and stay in range, freed
// space is coalesced (one free block once everything is released), the
// first-fit choice is the lowest free range that fits, and the byte counts
// match.  Exit status 0 on success.
#include <cstdio>
#include <random>
#include <vector>

#include "arena.h"

int main() {
  using ens_host::Arena;
  const size_t PAGE = 256, PAGES = 4096;
  std::mt19937_64 rng(12345);
  for (int round = 0; round < 20; ++round) {
    Arena a;
    a.reset(PAGES * PAGE);
    std::vector<int> owner(PAGES, -1);
    struct Blk { size_t off, bytes; bool live; };
    std::vector<Blk> blocks;
    for (int step = 0; step < 4000; ++step) {
      const bool do_alloc = blocks.empty() || rng() % 3 != 0;
      if (do_alloc) {
        const size_t bytes = 1 + rng() % (PAGE * 64);
        const size_t pages = (bytes + PAGE - 1) / PAGE;
        // brute force: lowest start with `pages` free pages
        size_t want = PAGES;
        for (size_t s = 0, run = 0; s < PAGES; ++s) {
          run = owner[s] < 0 ? run + 1 : 0;
          if (run == pages) { want = s + 1 - pages; break; }
        }
        size_t off = 0;
        const bool ok = a.alloc(bytes, &off);
        if (ok != (want < PAGES)) { std::printf("fit mismatch\n"); return 1; }
        if (!ok) continue;
        if (off != want * PAGE) { std::printf("not first fit\n"); return 1; }
        for (size_t p = 0; p < pages; ++p) {
          if (owner[off / PAGE + p] >= 0) { std::printf("overlap\n"); return 1; }
          owner[off / PAGE + p] = (int)blocks.size();
        }
        blocks.push_back({off, bytes, true});
      } else {
        const size_t k = rng() % blocks.size();
        if (!blocks[k].live) continue;
        a.release(blocks[k].off, blocks[k].bytes);
        for (size_t p = 0; p < (blocks[k].bytes + PAGE - 1) / PAGE; ++p)
          owner[blocks[k].off / PAGE + p] = -1;
        blocks[k].live = false;
      }
      size_t used = 0;
      for (int o : owner) used += o >= 0 ? PAGE : 0;
      if (used != a.used()) { std::printf("used mismatch\n"); return 1; }
    }
    for (auto& b : blocks)
      if (b.live) a.release(b.off, b.bytes);
    if (a.used() != 0 || a.free_blocks() != 1 || a.largest_free() != PAGES * PAGE) {
      std::printf("not coalesced\n");
      return 1;
    }
  }
  std::printf("ok\n");
  return 0;
}
