// Host-only driver around rocRAND's open-source Philox4x32-10 engine header,
// used as an independent implementation to pin the oracle's generator.
// Reads lines "c0 c1 c2 c3 k0 k1" on stdin and prints the four output words
// of the block for counter (c0,c1,c2,c3) and key (k0,k1).
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        // rocRAND's engine: key = seed words, counter words (2,3) = subsequence,
        // counter words (0,1) = offset / 4.
        unsigned long long seed = (unsigned long long)k[0] | ((unsigned long long)k[1] << 32);
        unsigned long long sub = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long off = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
