// Host-side reference for the Philox4x32-10 pin: evaluates rocRAND's own
// philox4x32_10 bijection (a library routine, independent of the oracle) on
// counter/key lines read from stdin ("c0 c1 c2 c3 k0 k1", decimal) and prints
// the four output words per line.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct PhiloxRef : rocrand_device::philox4x32_10_engine {
  uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  PhiloxRef ref;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = ref.eval(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
