// Host-only driver around rocRAND's Philox4x32-10 engine, used by the tests to
// pin the oracle's Philox.  rocRAND's engine(seed, subsequence, offset) starts at
// counter (offset/4 low, offset/4 high, subsequence low, subsequence high) with
// key (seed low, seed high); with offset a multiple of 4 its first next4()
// returns the raw Philox block of that counter.
// Reads lines "c0 c1 c2 c3 seed" and prints the four output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned c0, c1, c2, c3;
    unsigned long long seed;
    while (std::scanf("%u %u %u %u %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        unsigned long long offset = ((static_cast<unsigned long long>(c1) << 32) | c0) * 4ull;
        unsigned long long subseq = (static_cast<unsigned long long>(c3) << 32) | c2;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
