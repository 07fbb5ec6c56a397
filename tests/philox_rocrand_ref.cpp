// Host-side reference values of Philox4x32-10 taken from rocRAND's
// header-only engine (a library routine), used to pin the oracle's own
// implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints
// the four output words of the ten-round bijection at that counter and key.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct philox_probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_probe eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
