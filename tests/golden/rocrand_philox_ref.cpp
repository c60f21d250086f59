// External reference for the oracle's Philox4x32-10: rocRAND's host-callable
// implementation.  Reads "c0 c1 c2 c3 seed" lines on stdin (decimal) and prints the
// generator's 4-word output block for counter (c0, c1, c2, c3) under key = seed.
// rocRAND maps (offset / 4) to counter words 0-1 and the subsequence to words 2-3.
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long c0, c1, c2, c3, seed;
  while (std::scanf("%llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
    rocrand_state_philox4x32_10 st;
    const unsigned long long offset = 4ull * (c0 | (c1 << 32));
    const unsigned long long subseq = c2 | (c3 << 32);
    rocrand_init(seed, subseq, offset, &st);
    uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
