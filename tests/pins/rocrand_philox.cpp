// Independent Philox4x32-10 reference for the oracle's stream: AMD rocRAND's
// header-only philox4x32_10 engine, built for the host.  Reads lines
// "c0 c1 c2 c3 seed" (decimal) on stdin and prints the four output words.
// rocRAND's engine maps (seed, subsequence, offset) to key = seed and
// counter = (offset/4 low 64 bits, subsequence high 64 bits), and next4() at a
// block boundary returns the ten-round block of that counter.
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, seed;
    while (std::scanf("%llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        const unsigned long long sub = (c3 << 32) | c2;
        const unsigned long long blk = (c1 << 32) | c0;
        if (blk >> 62) { std::printf("ERR\n"); continue; }
        rocrand_device::philox4x32_10_engine eng(seed, sub, blk * 4ull);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
