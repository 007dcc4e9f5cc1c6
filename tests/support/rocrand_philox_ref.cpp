// Independent Philox4x32-10 reference for the oracle's RNG pin: rocRAND's own ten-round bijection,
// reached through a subclass of its engine. Reads lines "c0 c1 c2 c3 k0 k1" (decimal u32) from stdin,
// prints the four output words per line. Host code only; no GPU call is made.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Ref : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Ref ref;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = ref.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
