// Host-only check program: evaluates Philox4x32-10 with the open-source
// rocRAND implementation, as an independent reference for the oracle.
// Usage: philox_rocrand c0 c1 c2 c3 k0 k1 (hex); prints four hex words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
struct Peek : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
  unsigned c[4], k[2];
  for (int i = 0; i < 4; ++i) c[i] = strtoul(argv[1+i], 0, 16);
  for (int i = 0; i < 2; ++i) k[i] = strtoul(argv[5+i], 0, 16);
  Peek e;
  uint4 r = e.run(uint4{c[0], c[1], c[2], c[3]}, uint2{k[0], k[1]});
  printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
}
