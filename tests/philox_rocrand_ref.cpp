// Host-side reference for the Philox4x32-10 pin: reads lines
// "c0 c1 c2 c3 k0 k1" (hex) and prints the four output words of one block,
// computed by rocRAND's philox4x32_10 engine (an independent implementation
// of the same published generator) through its public API:
// key = seed, counter = (offset/4 lo, hi, subsequence lo, hi).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        unsigned w0 = rocrand(&st), w1 = rocrand(&st), w2 = rocrand(&st), w3 = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
