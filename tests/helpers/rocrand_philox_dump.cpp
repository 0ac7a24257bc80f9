// Prints Philox4x32-10 outputs computed by rocRAND's header-only engine for
// counters/keys read from stdin (one "c0 c1 c2 c3 k0 k1" line each, hex).
// Used only by the test suite as a library cross-check of the oracle.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

namespace {
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

int main()
{
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
