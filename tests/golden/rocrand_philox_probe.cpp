// Prints rocRAND's Philox4x32-10 draws (header-only engine, host side) for
// (seed, subsequence, offset) triples read from stdin, one per line.  Used by
// the oracle tests as an independent known-answer source for the draw
// "output t mod 4 of Philox4x32-10 with key = seed, counter = (t/4, 0, i, 0)",
// which is rocRAND's engine(seed, subsequence = i, offset = t).next().
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    std::printf("%u\n", e.next());
  }
  return 0;
}
