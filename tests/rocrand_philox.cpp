// Prints rocRAND's Philox4x32-10 block for each (c0 c1 c2 c3 k0 k1) line on stdin.
// rocRAND is an implementation independent of this repository; its engine is
// header-only and host-callable, so this runs on a machine without a GPU.
// Engine layout: key = (seed lo, seed hi); counter = (offset/4 as 64 bits,
// subsequence as 64 bits).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 s;
    const unsigned long long seed = k0 | (k1 << 32);
    const unsigned long long subsequence = c2 | (c3 << 32);
    const unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_init(seed, subsequence, offset, &s);
    const uint4 r = rocrand4(&s);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
