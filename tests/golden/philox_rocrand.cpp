// Prints the first n outputs (four words each) of rocRAND's header-only
// philox4x32_10 engine for a 64-bit seed, subsequence 0, offset 0: the
// generator's words for counters (0, 0, 0, 0), (1, 0, 0, 0), ... under the
// key (seed low word, seed high word).  Host code only; used by a CPU test
// as an independent implementation of the generator.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const unsigned long long seed = strtoull(argv[1], nullptr, 0);
  const int n = atoi(argv[2]);
  rocrand_device::philox4x32_10_engine e(seed, 0, 0);
  for (int i = 0; i < n; ++i) {
    const uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
