// Test helper: prints rocRAND's Philox-4x32-10 output blocks (host-side use of
// the rocRAND device API) for (seed, subsequence, offset) triples read from
// stdin, one block per line.  An independent implementation used only to
// check the oracle's own Philox.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long seed, subseq, offset;
  while (std::scanf("%llu %llu %llu", &seed, &subseq, &offset) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, offset, &st);
    uint4 v = rocrand4(&st);
    std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
  }
  return 0;
}
