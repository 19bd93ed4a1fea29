// Drives the library's device-memory arena (host-only bookkeeping) from a
// script on stdin, for the CPU tests:
//   init <bytes>      a <id> <bytes>      r <id>      q
// prints the offset of every allocation (-1 when refused) and, for q, the
// bytes in use, the largest free block and the number of free blocks.
#include <cstdio>
#include <cstring>
#include <map>

#include "cg_arena.h"

int main() {
  cgr::Arena arena;
  static char region[1];  // only addresses relative to it are used
  std::map<long, void*> live;
  char op[16];
  while (std::scanf("%15s", op) == 1) {
    if (!std::strcmp(op, "init")) {
      unsigned long long n;
      std::scanf("%llu", &n);
      arena.init(region, (size_t)n);
    } else if (!std::strcmp(op, "a")) {
      long id;
      unsigned long long n;
      std::scanf("%ld %llu", &id, &n);
      void* p = arena.alloc((size_t)n);
      if (p) live[id] = p;
      std::printf("%lld\n", p ? (long long)((char*)p - region) : -1LL);
    } else if (!std::strcmp(op, "r")) {
      long id;
      std::scanf("%ld", &id);
      auto it = live.find(id);
      if (it != live.end()) {
        arena.release(it->second);
        live.erase(it);
      }
    } else if (!std::strcmp(op, "q")) {
      std::printf("%zu %zu %zu\n", arena.in_use(), arena.largest_free(), arena.free_blocks());
    }
  }
  return 0;
}
