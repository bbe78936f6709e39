// Prints rocRAND's Philox4x32-10 block function for counters/keys read from stdin.
// Input lines: c0 c1 c2 c3 k0 k1 (decimal); output lines: r0 r1 r2 r3.
// Used only as a library pin for the CPU oracle's Philox.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// The block function is a protected member; expose it unchanged.
struct block_fn : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    block_fn e;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
