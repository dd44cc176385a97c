// Prints Philox4x32-10 outputs computed by rocRAND's own implementation of the
// generator (Salmon et al., SC'11), for the counter/key pairs given on stdin.
// Used by the RNG pin of the oracle; built and run by the test at test time.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Ref : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Ref ref;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = ref.rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
