// Host-only cross-check of Philox4x32-10 against rocRAND's header implementation
// (test dependency only; reads "ctr0 ctr1 ctr2 ctr3 key0 key1" hex lines, prints the 4 output words).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c0,c1,c2,c3,k0,k1; probe p;
  while (scanf("%x %x %x %x %x %x", &c0,&c1,&c2,&c3,&k0,&k1) == 6) {
    uint4 r = p.run(uint4{c0,c1,c2,c3}, uint2{k0,k1});
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
}
