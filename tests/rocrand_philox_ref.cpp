// Test helper: Philox4x32-10 from the rocRAND library headers, on the host.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output
// words.  Used only to cross-check the oracle's own Philox.
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

namespace {
// The engine keeps its ten-round block function protected; a subclass
// makes it callable with an explicit counter and key.
struct Engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};
}  // namespace

int main()
{
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
