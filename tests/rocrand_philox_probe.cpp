// Host-only probe: prints Philox4x32-10 blocks computed by rocRAND's open-source
// engine for (counter, key) lines read from stdin.  Used by the oracle tests
// as an independent implementation to compare against.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
struct Probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main(int argc, char** argv) {
  unsigned v[6];
  Probe p;
  while (scanf("%x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
    uint4 c = {v[0], v[1], v[2], v[3]}; uint2 k = {v[4], v[5]};
    uint4 o = p.run(c, k);
    printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
  return 0;
}
