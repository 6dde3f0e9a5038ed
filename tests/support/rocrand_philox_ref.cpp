// Independent Philox4x32-10 reference for the oracle's pin: rocRAND's
// host-callable engine (a third-party implementation of Salmon et al., SC'11).
// Reads "c0 c1 c2 c3 k0 k1" lines (hex) on stdin, prints "o0 o1 o2 o3".
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Exposed : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    Exposed e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.apply(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
