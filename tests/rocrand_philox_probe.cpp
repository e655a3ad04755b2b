// Host-side probe: evaluates rocRAND's Philox4x32-10 block function on counters and
// keys read from stdin ("c0 c1 c2 c3 k0 k1" per line, decimal) and prints the four
// output words. Used only as an independent implementation to pin the reference's
// generator; the product library does not include rocRAND.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    Probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
