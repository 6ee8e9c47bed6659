// Test helper: prints rocRAND's Philox4x32-10 output block for each
// (seed, subsequence, offset) triple read from stdin.  rocRAND's engine maps
// seed -> key (lo, hi), subsequence -> counter words 2..3 and offset/4 ->
// counter words 0..1, so offset = 4 * t, subsequence = pid reproduces the
// counter (t, 0, pid lo, pid hi).  Runs on the host only; used to pin the
// oracle's independent Philox implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, sub, off;
  while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
    rocrand_device::philox4x32_10_engine eng(seed, sub, off);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
