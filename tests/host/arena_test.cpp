// Randomised check of the request server's arena allocator against a
// brute-force occupancy map: blocks never overlap or leave the arena,
// largest() equals the longest free run, and freeing everything coalesces
// back into one block.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "arena.h"

int main() {
  const size_t size = 4096;
  wpcd::Arena a;
  a.reset(size);
  std::vector<int> owner(size, -1);
  struct Blk { size_t off, len; };
  std::vector<Blk> live;
  std::mt19937_64 rng(7);
  for (int step = 0; step < 200000; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t len = 1 + rng() % 300;
      // brute force: first free run of length >= len
      size_t want = SIZE_MAX, run = 0;
      for (size_t i = 0; i < size; ++i) {
        run = owner[i] < 0 ? run + 1 : 0;
        if (run == len) { want = i + 1 - len; break; }
      }
      const size_t got = a.alloc(len);
      if (got != want) { printf("step %d: alloc(%zu) = %zu, first fit is %zu\n", step, len, got, want); return 1; }
      if (got != SIZE_MAX) {
        for (size_t i = got; i < got + len; ++i) owner[i] = step;
        live.push_back({got, len});
      }
    } else {
      const size_t k = rng() % live.size();
      for (size_t i = live[k].off; i < live[k].off + live[k].len; ++i) owner[i] = -1;
      a.release(live[k].off, live[k].len);
      live[k] = live.back();
      live.pop_back();
    }
    size_t best = 0, run = 0, used = 0;
    for (size_t i = 0; i < size; ++i) {
      run = owner[i] < 0 ? run + 1 : 0;
      best = run > best ? run : best;
      used += owner[i] >= 0;
    }
    if (a.largest() != best || a.used() != used) {
      printf("step %d: largest %zu vs %zu, used %zu vs %zu\n", step, a.largest(), best, a.used(), used);
      return 1;
    }
  }
  for (auto& b : live) a.release(b.off, b.len);
  if (a.free_blocks() != 1 || a.largest() != size || a.used() != 0) { printf("no full coalescing\n"); return 1; }
  printf("arena ok\n");
  return 0;
}
