// Third-party Philox4x32-10 (rocRAND header implementation) used only to pin
// the oracle generator: reads "ctr0 ctr1 ctr2 ctr3 key0 key1" hex lines from
// stdin and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct P : rocrand_device::philox4x32_10_engine {
  uint4 tr(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  P p; unsigned a,b,c,d,e,f;
  while (scanf("%x %x %x %x %x %x", &a,&b,&c,&d,&e,&f) == 6) {
    uint4 o = p.tr(uint4{a,b,c,d}, uint2{e,f});
    printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
  }
}
