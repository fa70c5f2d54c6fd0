// Prints Philox4x32-10 outputs computed by rocRAND's host-side engine, one
// line per counter read from stdin: "c0 c1 c2 c3 k0 k1" -> "r0 r1 r2 r3".
// rocRAND is an installed library, independent of this repository; the test
// suite compares its outputs with the CPU reference bit for bit.
//
// rocRAND's engine seeded with (seed, subsequence, offset) starts from the
// counter (offset/4 as 64 bits, subsequence as 64 bits) and key (seed low
// word, seed high word); with offset a multiple of 4 its next four outputs
// are the ten-round block of that counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long blk = ((unsigned long long)c1 << 32) | c0;
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, blk * 4ull, &st);
        unsigned r0 = rocrand(&st), r1 = rocrand(&st), r2 = rocrand(&st), r3 = rocrand(&st);
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
