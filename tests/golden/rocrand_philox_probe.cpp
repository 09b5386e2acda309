// Host-only probe: prints rocRAND's Philox4x32-10 block for counter
// (j, i, g, s) and key (seed lo, seed hi), one query per stdin line
// "seed j i g s".  rocRAND's engine lays its counter out as
// (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi), so the
// query maps to subsequence g | s<<32 and offset 4*(j | i<<32).
// Used by tests/test_oracle_philox.py as an independent library reference.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long seed, j, i, g, s;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &j, &i, &g, &s) == 5) {
    rocrand_device::philox4x32_10_engine e(seed, g | (s << 32), 4ull * (j | (i << 32)));
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
