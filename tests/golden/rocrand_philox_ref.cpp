// Host-side reference outputs of rocRAND's Philox4x32-10 engine, used only to
// cross-check the oracle's Philox.  rocrand_init(seed, subsequence, offset)
// sets key = seed and counter = (offset/4 as 64 bits, subsequence as 64 bits),
// so the four outputs after init(seed, slot | tag << 32, 4*T) are the block for
// counter (lo T, hi T, slot, tag).  Reads lines "seed T slot tag", prints hex.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main()
{
    unsigned long long seed, T, slot, tag;
    while (std::scanf("%llu %llu %llu %llu", &seed, &T, &slot, &tag) == 4) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, slot | (tag << 32), 4ull * T, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
