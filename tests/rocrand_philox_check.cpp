// Host-side reference outputs of Philox4x32-10 from rocRAND's engine (an independent
// implementation), for cross-checking the project's three implementations.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) and prints the four output words.
// Philox(key, ctr) with ctr = (c0, c1, c2, c3) is rocRAND's engine seeded with
// key (k1:k0), subsequence (c3:c2) and offset 4 * (c1:c0), read with next4().
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned int c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
