// Independent Philox4x32-10 reference: rocRAND's header-only engine, run on the
// host.  Reads "seed c0 c1 c2 c3" lines on stdin, prints the four output words.
// rocRAND's engine advanced by subsequence c2 | c3<<32 and by c0 + c1*2^32
// blocks of four words sits exactly on counter (c0, c1, c2, c3) with key = seed.
// The c1 part is added as four discards of c1<<32 words (= c1<<30 blocks each)
// so that no offset overflows 64 bits.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        rocrand_device::philox4x32_10_engine e(seed, c2 | (c3 << 32), 4ull * c0);
        for (int i = 0; i < 4; ++i) e.discard(c1 << 32);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
