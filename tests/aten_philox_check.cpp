// Prints Philox4x32-10 outputs from ATen's independent host implementation,
// one line of four words per (seed, c0, c1, c2, c3) line read from stdin.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    // ATen's counter is (offset_lo, offset_hi, subsequence_lo, subsequence_hi)
    at::Philox4_32 eng(seed, c2 | (c3 << 32), c0 | (c1 << 32));
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
