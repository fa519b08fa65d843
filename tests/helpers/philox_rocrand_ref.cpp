// Test helper: prints Philox4x32-10 outputs computed by ROCm's rocRAND engine
// (an implementation independent of the oracle) for counter/key lines read
// from stdin: "c0 c1 c2 c3 k0 k1" in hex, one query per line.  Host only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct PhiloxProbe : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  PhiloxProbe p;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = p.rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
