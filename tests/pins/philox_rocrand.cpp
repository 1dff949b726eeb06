// Known-answer generator for the Philox4x32-10 pin: runs rocRAND's own
// philox4x32_10 engine (from the ROCm headers, compiled here) on the host.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the
// four output words of the block function for each.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  probe p;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr{c0, c1, c2, c3};
    uint2 key{k0, k1};
    uint4 o = p.block(ctr, key);
    std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
