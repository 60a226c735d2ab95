// Known-answer generator for the Philox4x32-10 pin: calls rocRAND's
// host-callable Philox4x32-10 state (an independent implementation of the
// same published generator) and prints one 4-word block per query line.
// Input lines: seed counter0 counter1 counter2 counter3
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned int c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        // rocrand_init(seed, subsequence, offset): key = seed, counter words 2..3
        // = subsequence, counter words 0..1 = offset / 4 (4 outputs per block).
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
