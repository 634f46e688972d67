// Host-only probe: prints rocRAND's Philox4x32-10 output words for
// (seed, subsequence, offset) triples read from stdin.  rocRAND is used as
// an independent black-box implementation of the generator (Salmon et al.,
// SC'11) to pin the oracle's Philox; nothing here runs on a GPU.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, off, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
