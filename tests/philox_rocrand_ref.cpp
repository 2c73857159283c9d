// Host-side evaluation of rocRAND's Philox4x32-10 engine, used by the oracle
// tests as an independent implementation of the generator.  Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal u32) on stdin and prints the 4 output words.
// The engine is seeded with key = k1:k0, subsequence = c3:c2 and offset =
// 4 * (c1:c0), so its first block is Philox(counter = (c0,c1,c2,c3), key).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
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
