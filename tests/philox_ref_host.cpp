// Host-only reference for Philox4x32-10: reads "c0 c1 c2 c3 k0 k1" lines (hex)
// from stdin and prints the four output words, using rocRAND's open-source
// header as an implementation independent of the oracle's.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Ref : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Ref r;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = r.apply(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
