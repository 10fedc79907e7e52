// Known-answer generator for the oracle's Philox4x32-10: runs the installed
// rocRAND device/host header generator (an independent implementation) and
// prints, for each "seed subsequence block" triple read from stdin, the four
// 32-bit outputs of that counter block.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, block;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &block) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, 4ull * block, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
